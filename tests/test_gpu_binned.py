"""GPU parity of strand generation that bins as it assembles (Sec. 3.1.1
with the tile raster of Sec. 3.1.2, hm_generate_raster_tiled): the stream and
both visibility layers bit for bit against the separate calls
(hm_generate_strands + hm_raster_vis) and against the oracle, on every
generator shape (one workgroup or one wave per bundle, strands longer than the
LDS chunk), truncated streams, multi-scene frames, long segments and other
tile shapes."""
import numpy as np
import pytest

from paper_2607_04230_amd import hm, scenes

pytestmark = pytest.mark.gpu

TOL = 1e-4
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _params(fr, **kw):
    rp = hm.raster_defaults(fr)
    for k, v in kw.items():
        setattr(rp, k, v)
    return rp


def _binned(sc, torch, cap=None, **kw):
    from paper_2607_04230_amd.render import DeviceScene
    print(f"[binned] {sc.name} {sc.width}x{sc.height} scenes={sc.n_scenes} cap={cap} {kw}",
          flush=True)
    ds = DeviceScene(sc, cap=cap)
    if kw:
        ds.set_raster_params(_params(ds.fr, **kw))
    ds.lod()
    ds.generate_raster_tiled()
    torch.cuda.synchronize()
    return ds


def _separate(sc, torch, cap=None, **kw):
    from paper_2607_04230_amd.render import DeviceScene
    ds = DeviceScene(sc, cap=cap)
    if kw:
        ds.set_raster_params(_params(ds.fr, **kw))
    ds.lod()
    ds.generate()
    ds.raster()
    torch.cuda.synchronize()
    return ds


def _same(a, b):
    pa, ra, fa = a.host_stream()
    pb, rb, fb = b.host_stream()
    assert np.array_equal(fa, fb)
    assert np.array_equal(pa.view(np.uint32), pb.view(np.uint32))
    assert np.array_equal(ra.view(np.uint32), rb.view(np.uint32))
    assert np.array_equal(a.host_vis(), b.host_vis())


@pytest.mark.parametrize("cap", [None, 40000], ids=["wave", "workgroup"])
def test_tiny_binned_matches_oracle(O, torch, cap):
    """tiny: 64 bundles of <= 512 CPs run one wave per bundle; a stream bound
    above 512 CPs per bundle selects one workgroup per bundle."""
    sc = scenes.config_tiny()
    ref = O.render(sc)
    ds = _binned(sc, torch, cap=cap)
    pos, rgb, fl = ds.host_stream()
    assert np.array_equal(fl, ref["flags"])
    assert np.array_equal(pos.view(np.uint32), ref["pos_w"].view(np.uint32))
    assert np.array_equal(ds.host_vis(), ref["vis"])
    _same(ds, _separate(sc, torch, cap=cap))


def test_head_1080p_binned_frame_matches_oracle(O, torch):
    """The benchmarked workload through the binned frame (LOD, generation with
    binning, tile raster, filtered resolve): stream and vis bit for bit, RGBA
    within 1e-4 of the oracle."""
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_head()
    ref = O.render(sc, n_threads=O.host_threads())
    ds = DeviceScene(sc)
    ds.render_binned()
    torch.cuda.synchronize()
    pos, rgb, fl = ds.host_stream()
    assert np.array_equal(fl, ref["flags"])
    assert np.array_equal(pos.view(np.uint32), ref["pos_w"].view(np.uint32))
    assert np.array_equal(rgb.view(np.uint32), ref["rgb"].view(np.uint32))
    assert np.array_equal(ds.host_vis(), ref["vis"])
    assert np.abs(ds.out.cpu().numpy().astype(np.float64) - ref["out"]).max() <= TOL


def test_lod_workload_binned_equals_separate(torch):
    """32 heads at 2560x1440 after LOD (bundles of every detail level)."""
    sc = scenes.config_lod()
    a = _binned(sc, torch)
    _same(a, _separate(sc, torch))
    assert (a.host_vis() != EMPTY).sum() > 100000


def test_batched_binned_equals_separate(O, torch):
    """64 scenes of uneven strand counts in one frame; three scenes also
    against the oracle."""
    sc = scenes.config_batched()
    a = _binned(sc, torch)
    _same(a, _separate(sc, torch))
    pos, rgb, fl = a.host_stream()
    soff = a.scene_off.cpu().numpy().view(np.uint32)
    vis = a.host_vis()
    for s in (0, 31, 63):
        order = np.arange(soff[s], soff[s + 1], dtype=np.uint32)
        ref = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z,
                       order=order)
        assert np.array_equal(vis[s], ref[s]), s


@pytest.mark.parametrize("cap", [1001, 5000])
def test_binned_truncated_stream(O, torch, cap):
    sc = scenes.config_tiny()
    table, soff, (ns, ncp) = O.lod_select(sc)
    assert cap < ncp
    pos, rgb, fl = O.generate(sc, table, ncp, cap=cap)
    soff_c = np.minimum(soff, cap).astype(np.uint32)
    vis = O.raster(pos, fl, soff_c, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    ds = _binned(sc, torch, cap=cap)
    gp, gr, gf = ds.host_stream()
    assert np.array_equal(gf, fl)
    assert np.array_equal(gp.view(np.uint32), pos.view(np.uint32))
    assert np.array_equal(ds.host_vis(), vis)
    _same(ds, _separate(sc, torch, cap=cap))


@pytest.mark.parametrize("n_cp,cap", [(1500, None), (300, 1500)], ids=["workgroup", "wave"])
def test_binned_strands_longer_than_the_lds_chunk(O, torch, n_cp, cap):
    """Strands whose screen records do not fit the generator's LDS: their
    segments are projected again from the stream just written."""
    sc = scenes.micro_scene(5, n_cp=n_cp, res=48)
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, table, ncp, cap=cap)
    if cap is not None:
        soff = np.minimum(soff, cap).astype(np.uint32)
    vis = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    ds = _binned(sc, torch, cap=cap)
    assert np.array_equal(ds.host_vis(), vis)
    assert (vis != EMPTY).sum() > 80
    _same(ds, _separate(sc, torch, cap=cap))


@pytest.mark.parametrize("kw", [dict(max_tiles_per_seg=1), dict(max_tiles_per_seg=4),
                                dict(tile=16, chunk=256), dict(tile=8, chunk=2048),
                                dict(block=128)],
                         ids=["K1", "K4", "tile16", "tile8", "block128"])
def test_binned_launch_shapes(torch, kw):
    """Long-segment lists (K = 1, 4), other tiles, chunks and workgroups: the
    same stream and buffer as the separate calls with the same parameters."""
    sc = scenes.config_head(width=640, height=360, strands_per_quad=16)
    _same(_binned(sc, torch, **kw), _separate(sc, torch, **kw))


def test_binned_calls_are_repeatable(torch):
    """Two calls in a row into the same buffers (counters and tables cleared
    by each call) give the same buffer."""
    sc = scenes.config_tiny()
    ds = _binned(sc, torch)
    first = ds.host_vis().copy()
    ds.generate_raster_tiled()
    torch.cuda.synchronize()
    assert np.array_equal(ds.host_vis(), first)
