"""Python binding of libhm (argument marshalling only).

Every function takes torch CUDA tensors, passes their device pointers and the
current torch stream to the C ABI declared in include/hm.h, and raises
RuntimeError with the library's message on any non-OK status.  There is no
fallback: if libhm.so is missing or no GPU is present, calls fail loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhm.so")

HM_OK = 0
LOD_OFF, LOD_ON = 0, 1
RASTER_TILED, RASTER_DIRECT, RASTER_TILED_ROWS = 0, 1, 2
RESOLVE_FILTER, RESOLVE_SOFT, RESOLVE_CENTER = 0, 1, 2
PAYLOAD_SEGMENT, PAYLOAD_GBUFFER = 0, 1
CALL_LOD, CALL_RASTER, CALL_RESOLVE, CALL_DOM, CALL_GEN_RASTER = 0, 1, 2, 3, 4

_u32, _i32, _f32, _vp, _sz = ctypes.c_uint32, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t


class Camera(ctypes.Structure):
    _fields_ = [("R", _f32 * 9), ("eye", _f32 * 3), ("fx", _f32), ("fy", _f32), ("cx", _f32),
                ("cy", _f32), ("znear", _f32), ("zfar", _f32)]


class Frame(ctypes.Structure):
    _fields_ = [("n_scenes", _u32), ("width", _u32), ("height", _u32)]


class HairMesh(ctypes.Structure):
    _fields_ = [("layer_pos", _vp), ("quads", _vp), ("bundle_key", _vp), ("bundle_nstrands", _vp),
                ("bundle_cmax", _vp), ("bundle_scene", _vp), ("n_bundles", _u32),
                ("n_layers", _u32), ("n_verts", _u32)]


class Strands(ctypes.Structure):
    _fields_ = [("pos_w", _vp), ("rgb", _vp), ("flags", _vp), ("scene_off", _vp),
                ("n_scenes", _u32), ("cap", _u32)]


class LodParams(ctypes.Structure):
    _fields_ = [("mode", _i32), ("lam", _f32), ("seed", _u32)]


class GenParams(ctypes.Structure):
    _fields_ = [("seed", _u32), ("width", _f32), ("curl_amp", _f32), ("curl_turns", _f32),
                ("base_rgb", _f32 * 3)]


class RasterParams(ctypes.Structure):
    _fields_ = [("r_min", _f32), ("algo", _i32), ("tile", _u32), ("chunk", _u32),
                ("max_tiles_per_seg", _u32), ("block", _u32), ("grid", _u32),
                ("shared_views", _u32), ("payload", _u32)]


class ShadeParams(ctypes.Structure):
    _fields_ = [("light_dir", _f32 * 3), ("light_rgb", _f32 * 3), ("ka", _f32), ("kd", _f32),
                ("ks", _f32), ("spec_squarings", _i32), ("filter_radius", _i32), ("s_par", _f32),
                ("s_perp", _f32), ("sigma_c", _f32), ("iso_scale", _f32), ("depth_reject", _f32),
                ("depth_mismatch", _f32), ("strip_half", _f32), ("iso_len", _f32),
                ("soft_sigma", _f32), ("bg", _f32 * 3), ("mode", _i32), ("shadow", _vp),
                ("payload", _i32)]


class DomParams(ctypes.Structure):
    _fields_ = [("width", _u32), ("height", _u32), ("n_layers", _u32), ("layer_codes", _u32),
                ("r_min", _f32), ("alpha", _f32)]


EXPORTS = ["hm_lod_select", "hm_generate_strands", "hm_raster_vis", "hm_resolve_shade",
           "hm_resolve_shade_bwd", "hm_workspace_size", "hm_raster_defaults", "hm_last_error",
           "hm_version", "hm_timing_enable", "hm_timing_collect", "hm_render_frame",
           "hm_graph_create", "hm_graph_launch", "hm_graph_destroy", "hm_lod_depth_offset",
           "hm_dom_accumulate", "hm_dom_shadow", "hm_generate_raster",
           "hm_resolve_shade_noalloc", "hm_generate_raster_tiled"]
# measurement helpers (include/hm_bench.h)
BENCH_EXPORTS = ["hm_bench_atomics", "hm_bench_traffic", "hm_bench_reciprocal"]


def lod_depth_offset(table, bundle_nstrands, delta_out):
    """Per-bundle depth correction delta = -log(N_LOD / N_b) (float32 tensor out)."""
    L = load()
    L.hm_lod_depth_offset.argtypes = [_vp, _vp, _u32, _vp, _vp]
    L.hm_lod_depth_offset.restype = _i32
    _check(L.hm_lod_depth_offset(_ptr(table), _ptr(bundle_nstrands), table.shape[0],
                                 _ptr(delta_out), _stream()), "hm_lod_depth_offset")


def bench_atomics(kind: int, buf, iters: int, grid: int):
    """Enqueue the atomic-rate microkernel (0: LDS, 1: global over buf) on the
    current stream; grid * 256 * iters 64-bit atomic minima."""
    L = load()
    L.hm_bench_atomics.argtypes = [_i32, _vp, _sz, _u32, _u32, _vp]
    L.hm_bench_atomics.restype = _i32
    _check(L.hm_bench_atomics(kind, _ptr(buf), buf.numel(), iters, grid, _stream()),
           "hm_bench_atomics")


def bench_traffic(kind: int, buf, sink, grid: int = 2048):
    """Enqueue the known-size stream microkernel on the current stream: kind 0
    reads all of buf once (sink: >= grid int32 words), kind 1 writes it."""
    L = load()
    L.hm_bench_traffic.argtypes = [_i32, _vp, _sz, _vp, _u32, _vp]
    L.hm_bench_traffic.restype = _i32
    nbytes = buf.numel() * buf.element_size()
    _check(L.hm_bench_traffic(kind, _ptr(buf), nbytes, _ptr(sink), grid, _stream()),
           "hm_bench_traffic")


def bench_reciprocal(lo: int, hi: int, counts):
    """Enqueue the exhaustive check of the raster's refined reciprocal over the
    binary32 bit patterns [lo, hi); adds (mismatches, values tested) to counts
    (a two-element int32 device tensor)."""
    L = load()
    L.hm_bench_reciprocal.argtypes = [_u32, _u32, _vp, _vp]
    L.hm_bench_reciprocal.restype = _i32
    _check(L.hm_bench_reciprocal(lo, hi, _ptr(counts), _stream()), "hm_bench_reciprocal")


def generate_raster(mesh, table, strand_base, strand_rgb, gp, st, cams, fr, r_min, scene_z,
                    vis, payload: int = 0):
    """Strand generation fused with the direct raster: the stream and
    segment-id keys (payload 0), or G-buffer keys and no stream (payload 1)."""
    L = load()
    L.hm_generate_raster.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _f32, _i32, _vp, _vp,
                                     _vp]
    _check(L.hm_generate_raster(ctypes.byref(mesh), _ptr(table), _ptr(strand_base),
                                _ptr(strand_rgb), ctypes.byref(gp), ctypes.byref(st), _ptr(cams),
                                ctypes.byref(fr), r_min, payload, _ptr(scene_z), _ptr(vis),
                                _stream()),
           "hm_generate_raster")


def dom_accumulate(st, light, dp, light_vis, counts, ws):
    """Deep-opacity-map fragment counts [n_layers][H][W] (uint32 / int32 tensor out)."""
    L = load()
    L.hm_dom_accumulate.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    _check(L.hm_dom_accumulate(ctypes.byref(st), _ptr(light), ctypes.byref(dp), _ptr(light_vis),
                               _ptr(counts), _ptr(ws), ws.numel() * ws.element_size(),
                               _stream()),
           "hm_dom_accumulate")


def dom_shadow(st, vis, cam, fr, light, dp, light_vis, counts, table, bundle_nstrands, shadow):
    """Light transmittance per camera pixel [H][W] (float32 tensor out)."""
    L = load()
    L.hm_dom_shadow.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u32, _vp, _vp]
    _check(L.hm_dom_shadow(ctypes.byref(st), _ptr(vis), _ptr(cam), ctypes.byref(fr), _ptr(light),
                           ctypes.byref(dp), _ptr(light_vis), _ptr(counts), _ptr(table),
                           _ptr(bundle_nstrands), table.shape[0], _ptr(shadow), _stream()),
           "hm_dom_shadow")


class FrameDesc(ctypes.Structure):
    _fields_ = [("mesh", HairMesh), ("cams", _vp), ("frame", Frame), ("lod", LodParams),
                ("table", _vp), ("ws_lod", _vp), ("ws_lod_bytes", _sz), ("strand_base", _vp),
                ("strand_rgb", _vp), ("gen", GenParams), ("strands", Strands), ("totals", _vp),
                ("raster", RasterParams), ("scene_z", _vp), ("vis", _vp), ("ws_raster", _vp),
                ("ws_raster_bytes", _sz), ("shade", ShadeParams), ("out_rgba", _vp),
                ("ws_resolve", _vp), ("ws_resolve_bytes", _sz)]


def render_frame(d: "FrameDesc"):
    L = load()
    L.hm_render_frame.argtypes = [ctypes.POINTER(FrameDesc), _vp]
    L.hm_render_frame.restype = _i32
    _check(L.hm_render_frame(ctypes.byref(d), _stream()), "hm_render_frame")


class Graph:
    """A frame captured once into a HIP graph (hm_graph_create) and replayed
    with hm_graph_launch; the descriptor's buffers must stay alive."""

    def __init__(self, d: "FrameDesc", stream_handle: int):
        L = load()
        L.hm_graph_create.argtypes = [ctypes.POINTER(FrameDesc), _vp, ctypes.POINTER(_vp)]
        L.hm_graph_create.restype = _i32
        L.hm_graph_launch.argtypes = [_vp, _vp]
        L.hm_graph_launch.restype = _i32
        L.hm_graph_destroy.argtypes = [_vp]
        L.hm_graph_destroy.restype = _i32
        self._d = d
        h = _vp()
        _check(L.hm_graph_create(ctypes.byref(d), stream_handle, ctypes.byref(h)), "hm_graph_create")
        self.handle = h

    def launch(self, stream_handle: int = None):
        _check(load().hm_graph_launch(self.handle, _stream() if stream_handle is None
                                      else stream_handle), "hm_graph_launch")

    def close(self):
        if self.handle:
            load().hm_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libhm.so not built at {path}; run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.hm_lod_select.argtypes = [P(HairMesh), _vp, P(Frame), P(LodParams), _vp, _vp, _vp, _vp,
                                _sz, _vp]
    L.hm_generate_strands.argtypes = [P(HairMesh), _vp, _vp, _vp, P(GenParams), P(Strands), _vp]
    L.hm_raster_vis.argtypes = [P(Strands), _vp, P(Frame), P(RasterParams), _vp, _vp, _vp, _sz,
                                _vp]
    L.hm_resolve_shade.argtypes = [P(Strands), _vp, _vp, P(Frame), P(ShadeParams), _vp, _vp, _sz,
                                   _vp]
    L.hm_resolve_shade_noalloc.argtypes = [P(Strands), _vp, _vp, P(Frame), P(ShadeParams), _vp,
                                           _vp]
    L.hm_resolve_shade_bwd.argtypes = [P(Strands), _vp, _vp, P(Frame), P(ShadeParams), _vp, _vp,
                                       _vp, _vp]
    L.hm_workspace_size.argtypes = [_i32, P(Frame), _u32, _u32, P(RasterParams), P(_sz)]
    L.hm_raster_defaults.argtypes = [P(Frame), P(RasterParams)]
    L.hm_last_error.restype = ctypes.c_char_p
    L.hm_last_error.argtypes = []
    L.hm_version.restype = _i32
    for name in EXPORTS:
        if name not in ("hm_last_error", "hm_version"):
            getattr(L, name).restype = _i32
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != HM_OK:
        msg = load().hm_last_error().decode()
        raise RuntimeError(f"{what} failed (status {rc}): {msg}")


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise RuntimeError("libhm takes device tensors only")
    if not t.is_contiguous():
        raise RuntimeError("libhm takes contiguous tensors only")
    return t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


# ----------------------------------------------------------------- descriptors
def frame(n_scenes: int, width: int, height: int) -> Frame:
    return Frame(n_scenes, width, height)


def hair_mesh(d: dict) -> HairMesh:
    lp = d["layer_pos"]
    return HairMesh(_ptr(lp), _ptr(d["quads"]), _ptr(d["bundle_key"]), _ptr(d["bundle_nstrands"]),
                    _ptr(d["bundle_cmax"]), _ptr(d["bundle_scene"]), d["quads"].shape[0],
                    lp.shape[0], lp.shape[1])


def strands(pos_w, rgb, flags, scene_off, cap: int) -> Strands:
    return Strands(_ptr(pos_w), _ptr(rgb), _ptr(flags), _ptr(scene_off), scene_off.shape[0] - 1,
                   cap)


def raster_defaults(fr: Frame) -> RasterParams:
    p = RasterParams()
    _check(load().hm_raster_defaults(ctypes.byref(fr), ctypes.byref(p)), "hm_raster_defaults")
    return p


def shade_params(rp, mode: int, bg=(0.0, 0.0, 0.0)) -> ShadeParams:
    s = ShadeParams()
    s.light_dir[:] = list(rp.light_dir)
    s.light_rgb[:] = list(rp.light_rgb)
    s.ka, s.kd, s.ks = rp.ka, rp.kd, rp.ks
    s.spec_squarings = rp.spec_squarings
    s.filter_radius = rp.filter_radius
    s.s_par, s.s_perp, s.sigma_c, s.iso_scale = rp.s_par, rp.s_perp, rp.sigma_c, rp.iso_scale
    s.depth_reject, s.depth_mismatch = rp.depth_reject, rp.depth_mismatch
    s.strip_half, s.iso_len, s.soft_sigma = rp.strip_half, rp.iso_len, rp.soft_sigma
    s.bg[:] = list(bg)
    s.mode = mode
    return s


def workspace_size(call: int, fr: Frame, n_bundles: int = 0, cap: int = 0,
                   rparams: Optional[RasterParams] = None) -> int:
    out = ctypes.c_size_t()
    rc = load().hm_workspace_size(call, ctypes.byref(fr), n_bundles, cap,
                                  ctypes.byref(rparams) if rparams is not None else None,
                                  ctypes.byref(out))
    _check(rc, "hm_workspace_size")
    return int(out.value)


# ----------------------------------------------------------------- calls
def lod_select(mesh: HairMesh, cams, fr: Frame, mode: int, lam: float, seed: int, table,
               scene_off, totals, ws):
    p = LodParams(mode, lam, seed)
    rc = load().hm_lod_select(ctypes.byref(mesh), _ptr(cams), ctypes.byref(fr), ctypes.byref(p),
                              _ptr(table), _ptr(scene_off), _ptr(totals), _ptr(ws),
                              ws.numel() * ws.element_size(), _stream())
    _check(rc, "hm_lod_select")


def generate_strands(mesh: HairMesh, table, strand_base, strand_rgb, gp: GenParams,
                     st: Strands):
    rc = load().hm_generate_strands(ctypes.byref(mesh), _ptr(table), _ptr(strand_base),
                                    _ptr(strand_rgb), ctypes.byref(gp), ctypes.byref(st),
                                    _stream())
    _check(rc, "hm_generate_strands")


def raster_vis(st: Strands, cams, fr: Frame, rp: RasterParams, scene_z, vis, ws):
    rc = load().hm_raster_vis(ctypes.byref(st), _ptr(cams), ctypes.byref(fr), ctypes.byref(rp),
                              _ptr(scene_z), _ptr(vis), _ptr(ws), ws.numel() * ws.element_size(),
                              _stream())
    _check(rc, "hm_raster_vis")


def generate_raster_tiled(mesh: HairMesh, table, strand_base, strand_rgb, gp: GenParams,
                          st: Strands, cams, fr: Frame, rp: RasterParams, scene_z, vis, ws):
    """Strand generation that bins as it assembles, then the tiled raster:
    the stream and vis of generate_strands + raster_vis in one call."""
    L = load()
    L.hm_generate_raster_tiled.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                           _vp, _vp, _sz, _vp]
    _check(L.hm_generate_raster_tiled(ctypes.byref(mesh), _ptr(table), _ptr(strand_base),
                                      _ptr(strand_rgb), ctypes.byref(gp), ctypes.byref(st),
                                      _ptr(cams), ctypes.byref(fr), ctypes.byref(rp),
                                      _ptr(scene_z), _ptr(vis), _ptr(ws),
                                      ws.numel() * ws.element_size(), _stream()),
           "hm_generate_raster_tiled")


def resolve_shade(st: Strands, vis, cams, fr: Frame, sp: ShadeParams, out, ws):
    rc = load().hm_resolve_shade(ctypes.byref(st), _ptr(vis), _ptr(cams), ctypes.byref(fr),
                                 ctypes.byref(sp), _ptr(out), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream())
    _check(rc, "hm_resolve_shade")


def resolve_shade_noalloc(st: Strands, vis, cams, fr: Frame, sp: ShadeParams, out):
    """hm_resolve_shade without a workspace (the library's static scratch)."""
    rc = load().hm_resolve_shade_noalloc(ctypes.byref(st), _ptr(vis), _ptr(cams),
                                         ctypes.byref(fr), ctypes.byref(sp), _ptr(out), _stream())
    _check(rc, "hm_resolve_shade_noalloc")


def timing_enable(on: bool):
    L = load()
    L.hm_timing_enable.argtypes = [_i32]
    L.hm_timing_enable.restype = _i32
    _check(L.hm_timing_enable(1 if on else 0), "hm_timing_enable")


def timing_collect() -> dict:
    """{kernel: (total_ms, launches)} for launches recorded since the last call."""
    L = load()
    L.hm_timing_collect.argtypes = [ctypes.c_char_p, _sz]
    L.hm_timing_collect.restype = _i32
    buf = ctypes.create_string_buffer(1 << 16)
    _check(L.hm_timing_collect(buf, len(buf)), "hm_timing_collect")
    out = {}
    for line in buf.value.decode().splitlines():
        name, ms, n = line.rsplit(" ", 2)
        base = name.lstrip("(").split("<")[0]          # template arguments folded
        t, c = out.get(base, (0.0, 0))
        out[base] = (t + float(ms), c + int(n))
    return out


def resolve_shade_bwd(st: Strands, vis, cams, fr: Frame, sp: ShadeParams, d_out, grad_pos,
                      grad_rgb):
    rc = load().hm_resolve_shade_bwd(ctypes.byref(st), _ptr(vis), _ptr(cams), ctypes.byref(fr),
                                     ctypes.byref(sp), _ptr(d_out), _ptr(grad_pos),
                                     _ptr(grad_rgb), _stream())
    _check(rc, "hm_resolve_shade_bwd")
