"""GPU parity of the compressed G-buffer keys (Sec. 3.1.2, deferred atomic
shading): visibility buffers bit for bit against the oracle for every launch
shape, depth bits and coverage equal to the segment-id buffer's, and the
centre resolve from the keys alone within 1e-4 of the oracle's."""
import numpy as np
import pytest

from paper_2607_04230_amd import hm, scenes
from paper_2607_04230_amd.scenes import ResolveParams

pytestmark = pytest.mark.gpu

TOL = 1e-4
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _ref(O, sc):
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, table, ncp)
    vis = O.raster_gbuf(pos, rgb, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    out = O.resolve_gbuf(vis, sc.cams, sc.width, sc.height, ResolveParams(), sc.bg)
    return vis, out


def _gpu(sc, torch, rp=None):
    from paper_2607_04230_amd.render import DeviceScene
    print(f"[gbuf] {sc.name} {sc.width}x{sc.height}", flush=True)
    ds = DeviceScene(sc)
    if rp is not None:
        ds.set_raster_params(rp)
    ds.use_gbuffer()
    ds.render()
    torch.cuda.synchronize()
    return ds


@pytest.mark.parametrize("name", ["tiny", "head", "head1080p"])
def test_gbuffer_keys_and_resolve_match_oracle(O, torch, name):
    if name == "tiny":
        sc = scenes.config_tiny()
    elif name == "head":
        sc = scenes.config_head(width=640, height=360, strands_per_quad=16)
    else:                                   # the benchmarked G-buffer workload
        sc = scenes.config_head()
    vis, out = _ref(O, sc)
    ds = _gpu(sc, torch)
    g = ds.host_vis()
    bad = np.argwhere(g != vis)
    assert bad.shape[0] == 0, f"{bad.shape[0]} keys differ, first {bad[:4].tolist()}"
    hit = (vis[:, 0] != EMPTY)
    assert hit.sum() > 1000
    assert np.abs(ds.out.cpu().numpy().astype(np.float64) - out).max() <= TOL


@pytest.mark.parametrize("algo,block,K", [(hm.RASTER_TILED, 128, 16),
                                          (hm.RASTER_TILED_ROWS, 256, 8),
                                          (hm.RASTER_DIRECT, 256, 8),
                                          (hm.RASTER_TILED, 256, 1)])
def test_gbuffer_keys_invariant_to_launch_shape(O, torch, algo, block, K):
    sc = scenes.config_tiny()
    vis, _ = _ref(O, sc)
    rp = hm.raster_defaults(hm.frame(1, sc.width, sc.height))
    rp.algo, rp.block, rp.max_tiles_per_seg = algo, block, K
    ds = _gpu(sc, torch, rp)
    assert np.array_equal(ds.host_vis(), vis)


def test_gbuffer_depth_and_coverage_equal_segment_keys(torch):
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_head(width=640, height=360, strands_per_quad=16)
    a = DeviceScene(sc)
    a.render()
    b = _gpu(sc, torch)
    va, vb = a.host_vis(), b.host_vis()
    assert np.array_equal(va >> np.uint64(40), vb >> np.uint64(40))
    assert np.array_equal(va == EMPTY, vb == EMPTY)


def test_gbuffer_keys_multi_scene(O, torch):
    """Uneven scenes in one frame: every scene's compressed keys and centre
    resolve match the oracle's."""
    sc = scenes.config_batched(n_scenes=6, res=128, n_min=1e3, n_max=1e4)
    vis, out = _ref(O, sc)
    ds = _gpu(sc, torch)
    assert np.array_equal(ds.host_vis(), vis)
    assert np.abs(ds.out.cpu().numpy().astype(np.float64) - out).max() <= TOL
