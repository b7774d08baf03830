"""The C-ABI library loads without a GPU, exports every entry point the public
header declares, and rejects bad arguments on the host with the documented
status codes (no kernel is launched by any of these calls)."""
import ctypes
import os
import re

import pytest

from paper_2607_04230_amd import hm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hm_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = hm.load()
    headers = sorted(h for h in os.listdir(os.path.join(ROOT, "include")) if h.endswith(".h"))
    assert headers == ["hm.h", "hm_bench.h"]
    names = _declared("hm.h")
    assert "hm_raster_vis" in names and len(names) >= 11
    bench = _declared("hm_bench.h")
    for n in names + bench:
        assert hasattr(L, n), n
    assert set(names) == set(hm.EXPORTS)
    assert set(bench) == set(hm.BENCH_EXPORTS)


def test_version_and_defaults():
    L = hm.load()
    assert L.hm_version() >= 100
    fr = hm.frame(1, 1920, 1080)
    p = hm.raster_defaults(fr)
    assert p.tile in (8, 16, 32) and p.block % 64 == 0 and p.algo == hm.RASTER_TILED


def test_workspace_sizes_scale():
    fr = hm.frame(1, 1920, 1080)
    a = hm.workspace_size(hm.CALL_RASTER, fr, cap=1000)
    b = hm.workspace_size(hm.CALL_RASTER, fr, cap=2_000_000)
    assert b > a > 0
    assert hm.workspace_size(hm.CALL_RESOLVE, fr) >= 1920 * 1080 * 16
    assert hm.workspace_size(hm.CALL_LOD, fr, n_bundles=2000) > 2000 * 16


def _status(fn, *args):
    return fn(*args)


def test_validation_errors_are_reported():
    L = hm.load()
    fr = hm.frame(1, 64, 64)
    bad = hm.frame(1, 0, 64)
    out = ctypes.c_size_t()
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(bad), 0, 10, None, ctypes.byref(out)) == 2
    assert b"outside" in L.hm_last_error()
    assert L.hm_workspace_size(7, ctypes.byref(fr), 0, 10, None, ctypes.byref(out)) == 1
    p = hm.raster_defaults(fr)
    p.tile = 24
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(fr), 0, 10, ctypes.byref(p),
                               ctypes.byref(out)) == 2
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(fr), 0, 0xFFFFFFFF, None,
                               ctypes.byref(out)) == 2
    # the per-pixel tile expansion takes at most 256 threads; the row walker more
    p = hm.raster_defaults(fr)
    p.block = 512
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(fr), 0, 10, ctypes.byref(p),
                               ctypes.byref(out)) == 2
    assert b"256" in L.hm_last_error()
    p.algo = hm.RASTER_TILED_ROWS
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(fr), 0, 10, ctypes.byref(p),
                               ctypes.byref(out)) == 0
    p.algo = 5
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(fr), 0, 10, ctypes.byref(p),
                               ctypes.byref(out)) == 1
    # NULL strands / arrays -> invalid, before any launch
    st = hm.Strands(None, None, None, None, 1, 10)
    rp = hm.raster_defaults(fr)
    assert L.hm_raster_vis(ctypes.byref(st), None, ctypes.byref(fr), ctypes.byref(rp), None,
                           None, None, 0, None) == 1
    # workspace too small -> HM_ERR_WORKSPACE
    dummy = ctypes.c_void_p(0x1000)
    st = hm.Strands(dummy, dummy, dummy, dummy, 1, 10)
    assert L.hm_raster_vis(ctypes.byref(st), dummy, ctypes.byref(fr), ctypes.byref(rp), None,
                           dummy, dummy, 16, None) == 3
    assert b"workspace" in L.hm_last_error()
    # mismatched scene counts
    fr2 = hm.frame(2, 64, 64)
    assert L.hm_raster_vis(ctypes.byref(st), dummy, ctypes.byref(fr2), ctypes.byref(rp), None,
                           dummy, dummy, 1 << 30, None) == 1
    # resolve: unknown mode, radius too large
    sp = hm.ShadeParams()
    sp.mode = 9
    assert L.hm_resolve_shade(ctypes.byref(st), dummy, dummy, ctypes.byref(fr), ctypes.byref(sp),
                              dummy, dummy, 1 << 30, None) == 1
    from paper_2607_04230_amd.scenes import ResolveParams
    sp = hm.shade_params(ResolveParams(filter_radius=9), hm.RESOLVE_FILTER)
    assert L.hm_resolve_shade(ctypes.byref(st), dummy, dummy, ctypes.byref(fr), ctypes.byref(sp),
                              dummy, dummy, 1 << 30, None) == 2
    # backward only for the soft resolve
    sp = hm.shade_params(ResolveParams(), hm.RESOLVE_FILTER)
    assert L.hm_resolve_shade_bwd(ctypes.byref(st), dummy, dummy, ctypes.byref(fr),
                                  ctypes.byref(sp), dummy, dummy, dummy, None) == 1
    # LOD: bad layer count
    m = hm.HairMesh(dummy, dummy, dummy, dummy, dummy, dummy, 4, 1, 10)
    lp = hm.LodParams(1, 3.0, 1)
    assert L.hm_lod_select(ctypes.byref(m), dummy, ctypes.byref(fr), ctypes.byref(lp), dummy,
                           dummy, dummy, dummy, 1 << 20, None) == 2
    assert b"n_layers" in L.hm_last_error()
    # fused generation + raster: scene counts must agree, r_min >= 0, a known
    # payload; segment-id keys need the stream's arrays, G-buffer keys do not
    P = ctypes.c_void_p
    L.hm_generate_raster.argtypes = [P, P, P, P, P, P, P, P, ctypes.c_float, ctypes.c_int32, P,
                                     P, P]
    gp = hm.GenParams()
    SEG, GBUF = hm.PAYLOAD_SEGMENT, hm.PAYLOAD_GBUFFER
    assert L.hm_generate_raster(ctypes.byref(m), dummy, None, None, ctypes.byref(gp),
                                ctypes.byref(st), dummy, ctypes.byref(fr2), 0.0, SEG,
                                None, dummy, None) == 2          # the mesh's n_layers is 1
    m2 = hm.HairMesh(dummy, dummy, dummy, dummy, dummy, dummy, 4, 4, 10)
    assert L.hm_generate_raster(ctypes.byref(m2), dummy, None, None, ctypes.byref(gp),
                                ctypes.byref(st), dummy, ctypes.byref(fr2), 0.0, SEG,
                                None, dummy, None) == 1
    assert b"n_scenes" in L.hm_last_error()
    assert L.hm_generate_raster(ctypes.byref(m2), dummy, None, None, ctypes.byref(gp),
                                ctypes.byref(st), dummy, ctypes.byref(fr), -1.0, SEG,
                                None, dummy, None) == 2
    assert L.hm_generate_raster(ctypes.byref(m2), dummy, None, None, ctypes.byref(gp),
                                ctypes.byref(st), dummy, ctypes.byref(fr), 0.0, 7,
                                None, dummy, None) == 1
    assert b"payload" in L.hm_last_error()
    no_stream = hm.Strands(None, None, None, dummy, 1, 1000)
    assert L.hm_generate_raster(ctypes.byref(m2), dummy, None, None, ctypes.byref(gp),
                                ctypes.byref(no_stream), dummy, ctypes.byref(fr), 0.0, SEG,
                                None, dummy, None) == 1
    assert b"NULL array" in L.hm_last_error()
    # (with G-buffer keys the same arguments pass validation; the call would
    # launch, so it is exercised by the GPU tests only)
    # generation with binning: the tiled algorithm, segment ids and one view
    # per scene only; matching scene counts; its own workspace size
    L.hm_generate_raster_tiled.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t,
                                           P]
    # (sized for this stream's cap of 10, so that no call below gets as far as
    # a launch on these placeholder pointers)
    need = hm.workspace_size(hm.CALL_GEN_RASTER, fr, n_bundles=m2.n_bundles, cap=st.cap,
                             rparams=rp)
    assert need > hm.workspace_size(hm.CALL_RASTER, fr, cap=st.cap, rparams=rp)

    def gen_tiled(rparams, frame=fr, ws_bytes=need):
        return L.hm_generate_raster_tiled(ctypes.byref(m2), dummy, None, None, ctypes.byref(gp),
                                          ctypes.byref(st), dummy, ctypes.byref(frame),
                                          ctypes.byref(rparams), None, dummy, dummy, ws_bytes,
                                          None)
    for field, value in (("algo", hm.RASTER_DIRECT), ("payload", GBUF), ("shared_views", 1)):
        bad = hm.RasterParams.from_buffer_copy(rp)
        setattr(bad, field, value)
        assert gen_tiled(bad) == 1, field
    assert gen_tiled(rp, frame=fr2) == 1
    assert b"n_scenes" in L.hm_last_error()
    assert gen_tiled(rp, ws_bytes=need - 1) == 3
    assert b"workspace" in L.hm_last_error()
    # atomic-rate microkernels: argument checks before any launch
    L.hm_bench_atomics.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
    assert L.hm_bench_atomics(5, dummy, 4096, 1, 16, None) == 1
    assert L.hm_bench_atomics(0, None, 4096, 1, 16, None) == 1
    assert L.hm_bench_atomics(0, dummy, 8, 1, 16, None) == 2
    L.hm_bench_traffic.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]
    assert L.hm_bench_traffic(0, dummy, 1000, dummy, 16, None) == 1     # not a multiple of 16
    assert L.hm_bench_traffic(0, dummy, 1024, None, 16, None) == 1      # read needs a sink
    assert L.hm_bench_traffic(2, dummy, 1024, dummy, 16, None) == 1
    assert L.hm_bench_traffic(1, dummy, 1024, None, 0, None) == 1
    # compressed G-buffer keys: known payloads only, no shared views, CENTER resolve
    rp = hm.raster_defaults(fr)
    rp.payload = 2
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(fr), 0, 10, ctypes.byref(rp),
                               ctypes.byref(out)) == 1
    rp.payload, rp.shared_views = hm.PAYLOAD_GBUFFER, 1
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(fr), 0, 10, ctypes.byref(rp),
                               ctypes.byref(out)) == 1
    rp.shared_views = 0
    a = ctypes.c_size_t()
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(fr), 0, 1000, ctypes.byref(rp),
                               ctypes.byref(a)) == 0
    rp.payload = hm.PAYLOAD_SEGMENT
    b = ctypes.c_size_t()
    assert L.hm_workspace_size(hm.CALL_RASTER, ctypes.byref(fr), 0, 1000, ctypes.byref(rp),
                               ctypes.byref(b)) == 0
    assert a.value >= b.value + 16 * 1000          # per-point tangents
    sp = hm.shade_params(ResolveParams(), hm.RESOLVE_FILTER)
    sp.payload = hm.PAYLOAD_GBUFFER
    assert L.hm_resolve_shade(ctypes.byref(st), dummy, dummy, ctypes.byref(fr), ctypes.byref(sp),
                              dummy, dummy, 1 << 30, None) == 1
    assert b"CENTER" in L.hm_last_error()
    # shadows: single scene, layer count and opacity ranges, workspace
    dp = hm.DomParams(64, 64, 4, 1000, 0.5, 0.05)
    ws = hm.workspace_size(hm.CALL_DOM, fr, cap=1000)
    assert ws >= 16 * 1000
    assert L.hm_dom_accumulate(ctypes.byref(st), dummy, ctypes.byref(dp), dummy, dummy, dummy,
                               8, None) == 3
    for field, val in (("n_layers", 0), ("n_layers", 9), ("layer_codes", 0), ("alpha", 0.0)):
        bad_dp = hm.DomParams(64, 64, 4, 1000, 0.5, 0.05)
        setattr(bad_dp, field, val)
        assert L.hm_dom_accumulate(ctypes.byref(st), dummy, ctypes.byref(bad_dp), dummy, dummy,
                                   dummy, 1 << 30, None) == 2, field
    assert L.hm_dom_shadow(ctypes.byref(st), dummy, dummy, ctypes.byref(fr2), dummy,
                           ctypes.byref(dp), dummy, dummy, dummy, dummy, 4, dummy, None) == 1
    assert b"single scene" in L.hm_last_error()
    # a shadowed soft resolve is refused (its backward has no shadow term)
    sp = hm.shade_params(ResolveParams(), hm.RESOLVE_SOFT)
    sp.shadow = 0x1000
    assert L.hm_resolve_shade(ctypes.byref(st), dummy, dummy, ctypes.byref(fr), ctypes.byref(sp),
                              dummy, dummy, 1 << 30, None) == 1


_LAYOUT = {
    "hm_camera": ("Camera", ["R", "eye", "fx", "zfar"]),
    "hm_frame": ("Frame", ["n_scenes", "height"]),
    "hm_hair_mesh": ("HairMesh", None),
    "hm_strands": ("Strands", None),
    "hm_lod_params": ("LodParams", None),
    "hm_gen_params": ("GenParams", None),
    "hm_raster_params": ("RasterParams", None),
    "hm_shade_params": ("ShadeParams", None),
    "hm_dom_params": ("DomParams", None),
    "hm_frame_desc": ("FrameDesc", None),
}


_C_NAME = {"lam": "lambda"}     # a Python keyword on the C side


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and every field offset of the header's structs, compiled by the
    host C compiler, equal those of the Python binding's ctypes mirrors."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hm.h"', 'int main(void) {']
    for cname, (pyname, _) in _LAYOUT.items():
        if not hasattr(hm, pyname):
            continue
        py = getattr(hm, pyname)
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            c = _C_NAME.get(f[0], f[0])
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {c}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    seen = 0
    for line in out.splitlines():
        cname, field, val = line.split()
        py = getattr(hm, _LAYOUT[cname][0])
        got = ctypes.sizeof(py) if field == "size" else getattr(py, field).offset
        assert got == int(val), (cname, field, got, val)
        seen += 1
    assert seen > 60
