"""GPU parity of strand generation fused with the raster (Sec. 3.1.1 with
3.1.2: one workgroup or wave per bundle generates, projects and rasterizes): the
stream and the visibility buffer bit for bit against the oracle and against
the separate generate + tiled raster calls, RGBA of the resolve within 1e-4."""
import numpy as np
import pytest

from paper_2607_04230_amd import scenes
from paper_2607_04230_amd.scenes import ResolveParams

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _fused(sc, torch, cap=None):
    from paper_2607_04230_amd.render import DeviceScene
    print(f"[fused] {sc.name} {sc.width}x{sc.height} scenes={sc.n_scenes} cap={cap}", flush=True)
    ds = DeviceScene(sc, cap=cap)
    ds.render_fused()
    torch.cuda.synchronize()
    return ds


def _separate(sc, torch, cap=None):
    from paper_2607_04230_amd.render import DeviceScene
    ds = DeviceScene(sc, cap=cap)
    ds.render()
    torch.cuda.synchronize()
    return ds


# The generator runs one wave per bundle when the bundles are many or small
# (tiny: 64 bundles, 9216 CPs <= 512 per bundle) and one workgroup per bundle
# otherwise; a stream bound of 40000 CPs (> 512 per bundle) selects the
# workgroup shape for the same scene.
@pytest.mark.parametrize("cap", [None, 40000], ids=["wave", "workgroup"])
def test_tiny_fused_matches_oracle(O, torch, cap):
    sc = scenes.config_tiny()
    ref = O.render(sc)
    ds = _fused(sc, torch, cap=cap)
    pos, rgb, fl = ds.host_stream()
    assert np.array_equal(fl, ref["flags"])
    assert np.array_equal(pos.view(np.uint32), ref["pos_w"].view(np.uint32))
    assert np.array_equal(rgb.view(np.uint32), ref["rgb"].view(np.uint32))
    assert np.array_equal(ds.host_vis(), ref["vis"])
    assert np.abs(ds.out.cpu().numpy().astype(np.float64) - ref["out"]).max() <= TOL


def test_head_1080p_fused_matches_oracle(O, torch):
    """The benchmarked fused workload: the full head at 1920x1080 with its
    occluder, stream and visibility bit for bit, RGBA within 1e-4."""
    sc = scenes.config_head()
    ref = O.render(sc, n_threads=O.host_threads())
    ds = _fused(sc, torch)
    pos, rgb, fl = ds.host_stream()
    assert np.array_equal(fl, ref["flags"])
    assert np.array_equal(pos.view(np.uint32), ref["pos_w"].view(np.uint32))
    assert np.array_equal(rgb.view(np.uint32), ref["rgb"].view(np.uint32))
    assert np.array_equal(ds.host_vis(), ref["vis"])
    assert np.abs(ds.out.cpu().numpy().astype(np.float64) - ref["out"]).max() <= TOL


def test_head_with_occluder_fused_matches_oracle_and_tiled(O, torch):
    sc = scenes.config_head(width=640, height=360, strands_per_quad=16)
    assert sc.scene_z is not None
    ds = _fused(sc, torch)
    sep = _separate(sc, torch)
    assert np.array_equal(ds.host_vis(), sep.host_vis())
    assert torch.equal(ds.out, sep.out)
    pos, rgb, fl = ds.host_stream()
    soff = ds.scene_off.cpu().numpy().view(np.uint32)
    vis = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    assert np.array_equal(ds.host_vis(), vis)


def test_batched_fused_matches_tiled_and_oracle(O, torch):
    """Uneven scenes in one frame: every bundle rasterizes into its own scene."""
    sc = scenes.config_batched(n_scenes=12, res=256, n_min=1e3, n_max=2e4)
    ds = _fused(sc, torch)
    sep = _separate(sc, torch)
    assert np.array_equal(ds.host_vis(), sep.host_vis())
    assert torch.equal(ds.out, sep.out)
    pos, rgb, fl = ds.host_stream()
    soff = ds.scene_off.cpu().numpy().view(np.uint32)
    for s in (0, 5, 11):
        order = np.arange(soff[s], soff[s + 1], dtype=np.uint32)
        vis = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z,
                       order=order)
        assert np.array_equal(ds.host_vis()[s], vis[s]), s


@pytest.mark.parametrize("cap", [1001, 5000])
def test_fused_truncated_stream(O, torch, cap):
    sc = scenes.config_tiny()
    table, soff, (ns, ncp) = O.lod_select(sc)
    assert cap < ncp
    pos, rgb, fl = O.generate(sc, table, ncp, cap=cap)
    soff_c = np.minimum(soff, cap).astype(np.uint32)
    vis = O.raster(pos, fl, soff_c, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    ds = _fused(sc, torch, cap=cap)
    gp, gr, gf = ds.host_stream()
    assert np.array_equal(gf, fl)
    assert np.array_equal(gp.view(np.uint32), pos.view(np.uint32))
    assert np.array_equal(ds.host_vis(), vis)
    out = O.resolve(pos, rgb, fl, vis, sc.cams, sc.width, sc.height, ResolveParams(), sc.mode,
                    sc.bg)
    assert np.abs(ds.out.cpu().numpy().astype(np.float64) - out).max() <= TOL


def test_fused_strands_longer_than_the_lds_chunk(O, torch):
    """1500 control points per strand do not fit the chunk's screen records
    in LDS: those segments are projected again from the stream; the buffer
    is still bit-identical to the oracle's."""
    sc = scenes.micro_scene(5, n_cp=1500, res=48)
    ref = O.render(sc)
    ds = _fused(sc, torch)
    pos, rgb, fl = ds.host_stream()
    assert np.array_equal(pos.view(np.uint32), ref["pos_w"].view(np.uint32))
    assert np.array_equal(ds.host_vis(), ref["vis"])
    assert (ref["vis"][:, 0] != np.uint64(0xFFFFFFFFFFFFFFFF)).sum() > 50


def test_fused_wave_shape_with_strands_longer_than_its_lds_slice(O, torch):
    """3 bundles of 300-CP strands with the stream bound at 1500 CPs (<= 512
    per bundle): one wave per bundle, whose quarter of the LDS holds at most
    256 screen records, so every segment is projected again from the stream;
    the truncated stream and the buffer match the oracle bit for bit."""
    sc = scenes.micro_scene(5, n_cp=300, res=48)
    cap = 1500
    table, soff, (ns, ncp) = O.lod_select(sc)
    assert cap < ncp and cap <= 512 * sc.quads.shape[0]
    pos, rgb, fl = O.generate(sc, table, ncp, cap=cap)
    soff_c = np.minimum(soff, cap).astype(np.uint32)
    vis = O.raster(pos, fl, soff_c, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    ds = _fused(sc, torch, cap=cap)
    gp, gr, gf = ds.host_stream()
    assert np.array_equal(gf, fl)
    assert np.array_equal(gp.view(np.uint32), pos.view(np.uint32))
    assert np.array_equal(gr.view(np.uint32), rgb.view(np.uint32))
    assert np.array_equal(ds.host_vis(), vis)
    assert (vis != np.uint64(0xFFFFFFFFFFFFFFFF)).sum() > 80      # 105 keys in both layers


# ----------------------------------------------------------------- stream-free
# Generation fused with the raster and the compressed G-buffer keys: no
# stream is written (the stream buffers are filled with a sentinel first and
# must come back untouched), the keys equal the oracle's G-buffer raster of
# the stream it generates, and the centre resolve of the keys alone matches the
# oracle's within 1e-4.
def _fused_gbuf(sc, torch, cap=None):
    from paper_2607_04230_amd.render import DeviceScene
    print(f"[fused gbuf] {sc.name} {sc.width}x{sc.height} scenes={sc.n_scenes} cap={cap}",
          flush=True)
    ds = DeviceScene(sc, cap=cap)
    ds.use_gbuffer()
    for t in (ds.pos_w, ds.rgb):
        t.fill_(float("nan"))
    ds.flags.fill_(0xA5)
    ds.render_fused()
    torch.cuda.synchronize()
    return ds


def _gbuf_ref(O, sc, cap=None):
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, table, ncp, cap=cap)
    if cap is not None:
        soff = np.minimum(soff, cap).astype(np.uint32)
    vis = O.raster_gbuf(pos, rgb, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    out = O.resolve_gbuf(vis, sc.cams, sc.width, sc.height, ResolveParams(), sc.bg)
    return vis, out


def _check_stream_free(ds, vis, out):
    assert bool(ds.pos_w.isnan().all()) and bool(ds.rgb.isnan().all())
    assert bool((ds.flags == 0xA5).all())
    assert np.array_equal(ds.host_vis(), vis)
    assert (vis[:, 0] != np.uint64(0xFFFFFFFFFFFFFFFF)).any()
    assert np.abs(ds.out.cpu().numpy().astype(np.float64) - out).max() <= TOL


@pytest.mark.parametrize("cap", [None, 40000], ids=["wave", "workgroup"])
def test_tiny_stream_free_gbuffer_matches_oracle(O, torch, cap):
    sc = scenes.config_tiny()
    vis, out = _gbuf_ref(O, sc)
    _check_stream_free(_fused_gbuf(sc, torch, cap=cap), vis, out)


def test_head_1080p_stream_free_gbuffer_matches_oracle(O, torch):
    """The benchmarked stream-free frame: the full head at 1920x1080."""
    sc = scenes.config_head()
    vis, out = _gbuf_ref(O, sc)
    _check_stream_free(_fused_gbuf(sc, torch), vis, out)


def test_stream_free_gbuffer_equals_separate_gbuffer_raster(torch):
    """Same keys as generate + tiled G-buffer raster, on a batched frame."""
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_batched(n_scenes=6, res=256, n_min=1e3, n_max=2e4)
    ds = _fused_gbuf(sc, torch)
    sep = DeviceScene(sc)
    sep.use_gbuffer()
    sep.render()
    torch.cuda.synchronize()
    assert np.array_equal(ds.host_vis(), sep.host_vis())
    assert torch.equal(ds.out, sep.out)


@pytest.mark.parametrize("cap", [1001, 5000])
def test_stream_free_gbuffer_truncated(O, torch, cap):
    sc = scenes.config_tiny()
    vis, out = _gbuf_ref(O, sc, cap=cap)
    _check_stream_free(_fused_gbuf(sc, torch, cap=cap), vis, out)


@pytest.mark.parametrize("n_cp,cap", [(1500, None), (300, 1500)], ids=["workgroup", "wave"])
def test_stream_free_gbuffer_strands_longer_than_the_lds_chunk(O, torch, n_cp, cap):
    """Strands whose points do not fit the LDS chunk: each segment generates
    its four points again (no stream to read back); same keys as the oracle."""
    sc = scenes.micro_scene(5, n_cp=n_cp, res=48)
    vis, out = _gbuf_ref(O, sc, cap=cap)
    _check_stream_free(_fused_gbuf(sc, torch, cap=cap), vis, out)
