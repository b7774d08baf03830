"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Integer outputs (LOD table, flags, visibility keys) and
the generated stream must match bit for bit; RGBA within 1e-4 absolute."""
import numpy as np
import pytest

from paper_2607_04230_amd import hm, scenes
from paper_2607_04230_amd.scenes import ResolveParams

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _gpu(sc, torch, rparams=None, mode=None):
    from paper_2607_04230_amd.render import DeviceScene
    ds = DeviceScene(sc, rparams=rparams, mode=mode)
    ds.render()
    torch.cuda.synchronize()
    return ds


def _compare_stream(ds, ref):
    assert np.array_equal(ds.table.cpu().numpy().view(np.uint32), ref["table"])
    assert np.array_equal(ds.scene_off.cpu().numpy().view(np.uint32), ref["scene_off"])
    tot = ds.totals.cpu().numpy()
    assert (int(tot[0]), int(tot[1])) == (ref["n_strands"], ref["n_cp"])
    pos, rgb, fl = ds.host_stream()
    assert np.array_equal(fl, ref["flags"])
    assert np.array_equal(pos.view(np.uint32), ref["pos_w"].view(np.uint32))
    assert np.array_equal(rgb.view(np.uint32), ref["rgb"].view(np.uint32))


def _rgba_err(out_gpu, ref_out, vis, label=""):
    """Max |gpu - oracle| over RGBA; prints the worst pixels (with their layer
    hits) so that a failure names its cause."""
    out = out_gpu.astype(np.float64)
    d = np.abs(out - ref_out).max(-1)
    err = float(d.max())
    if err > TOL:
        E = np.uint64(0xFFFFFFFFFFFFFFFF)
        flat = np.argsort(d.ravel())[::-1][:8]
        for f in flat:
            s, j, i = np.unravel_index(f, d.shape)
            kc, ka = vis[s, 0, j, i], vis[s, 1, j, i]
            print(f"{label} worst s={s} j={j} i={i} err={d[s, j, i]:.3e} centre={kc != E} "
                  f"cons={ka != E} gpu={out[s, j, i]} ref={ref_out[s, j, i]}")
        print(f"{label} pixels over tol: {(d > TOL).sum()} of {d.size}")
    return err


def test_tiny_end_to_end(O, torch):
    sc = scenes.config_tiny()
    ref = O.render(sc)
    ds = _gpu(sc, torch)
    _compare_stream(ds, ref)
    assert np.array_equal(ds.host_vis(), ref["vis"])
    assert _rgba_err(ds.out.cpu().numpy(), ref["out"], ref["vis"], "tiny") <= TOL


@pytest.mark.parametrize("algo,tile,chunk,K,block", [
    (hm.RASTER_DIRECT, 32, 256, 4, 256),
    (hm.RASTER_TILED, 8, 64, 2, 64),
    (hm.RASTER_TILED, 16, 1, 8, 128),
    (hm.RASTER_TILED, 32, 4096, 64, 256),
    (hm.RASTER_TILED, 16, 300, 3, 128),
    (hm.RASTER_TILED, 32, 100, 1, 256),
    (hm.RASTER_TILED_ROWS, 8, 64, 2, 64),
    (hm.RASTER_TILED_ROWS, 32, 4096, 64, 512),
    (hm.RASTER_TILED_ROWS, 16, 300, 3, 128),
])
def test_tiny_vis_invariant_to_launch_shape(O, torch, algo, tile, chunk, K, block):
    sc = scenes.config_tiny()
    ref = O.render(sc, want=("vis",))
    p = hm.RasterParams(0.0, algo, tile, chunk, K, block, 0)
    ds = _gpu(sc, torch, rparams=p)
    assert np.array_equal(ds.host_vis(), ref["vis"])


def test_every_autotune_candidate_gives_the_same_buffer(O, torch):
    from paper_2607_04230_amd import autotune
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_head(width=480, height=270, strands_per_quad=8)
    ref = O.render(sc, want=("vis",))
    ds = DeviceScene(sc)
    ds.lod()
    ds.generate()
    for c in autotune.DEFAULT_CANDIDATES:
        ds.set_raster_params(autotune.params_of(c, sc.r_min))
        ds.vis.fill_(0)
        ds.raster()
        torch.cuda.synchronize()
        assert np.array_equal(ds.host_vis(), ref["vis"]), c


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("r_min", [0.0, 0.5, 1.5])
def test_micro_scenes_brute_force(O, torch, seed, r_min):
    sc = scenes.micro_scene(seed, res=40 + seed)
    sc.r_min = r_min
    ref = O.render(sc, want=("vis",))
    brute = O.raster(ref["pos_w"], ref["flags"], ref["scene_off"], sc.cams, sc.width, sc.height,
                     r_min, brute=True)
    ds = _gpu(sc, torch)
    _compare_stream(ds, ref)
    assert np.array_equal(ds.host_vis(), brute)


def test_head_1080p_full(O, torch):
    sc = scenes.config_head()
    ref = O.render(sc)
    ds = _gpu(sc, torch)
    _compare_stream(ds, ref)
    assert np.array_equal(ds.host_vis(), ref["vis"])
    assert _rgba_err(ds.out.cpu().numpy(), ref["out"], ref["vis"], "head") <= TOL


def test_center_mode(O, torch):
    sc = scenes.config_head(width=640, height=360)
    sc.mode = scenes.MODE_CENTER
    ref = O.render(sc)
    ds = _gpu(sc, torch)
    assert _rgba_err(ds.out.cpu().numpy(), ref["out"], ref["vis"], "centre") <= TOL


def test_soft_forward_diff_config(O, torch):
    sc = scenes.config_diff()
    ref = O.render(sc)
    ds = _gpu(sc, torch)
    assert np.array_equal(ds.host_vis(), ref["vis"])
    assert _rgba_err(ds.out.cpu().numpy(), ref["out"], ref["vis"], "soft") <= TOL


def test_empty_frame_camera_facing_away(O, torch):
    # every segment is behind the camera: both layers stay empty and every
    # pixel is background
    sc = scenes.config_tiny()
    sc.cams = scenes.look_at_camera((0.0, 1.3, 2.6), (0.0, 1.3, 6.0), sc.width,
                                    sc.height)[None].astype(np.float32)
    ref = O.render(sc)
    ds = _gpu(sc, torch)
    _compare_stream(ds, ref)
    vis = ds.host_vis()
    assert np.array_equal(vis, ref["vis"])
    assert (vis == np.uint64(0xFFFFFFFFFFFFFFFF)).all()
    out = ds.out.cpu().numpy()
    assert _rgba_err(out, ref["out"], ref["vis"], "empty") <= TOL
    assert (out[..., 3] == 0.0).all()


def test_tiny_stream_with_the_workgroup_generator(O, torch):
    """A stream bound of 40000 CPs (> 512 per bundle of the 64) selects one
    workgroup per bundle instead of one wave; the stream is the same."""
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_tiny()
    ref = O.render(sc, want=("vis",))
    ds = DeviceScene(sc, cap=40000)
    ds.render()
    torch.cuda.synchronize()
    _compare_stream(ds, ref)
    assert np.array_equal(ds.host_vis(), ref["vis"])


@pytest.mark.parametrize("cap", [2, 1001, 5000])
def test_stream_truncated_to_capacity(O, torch, cap):
    # a stream capacity below the LOD total keeps the first cap control
    # points, the last one flagged as a tip; raster and resolve read nothing
    # past cap
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_tiny()
    table, soff, (ns, ncp) = O.lod_select(sc)
    assert cap < ncp
    pos, rgb, fl = O.generate(sc, table, ncp, cap=cap)
    soff_c = np.minimum(soff, cap).astype(np.uint32)
    vis = O.raster(pos, fl, soff_c, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    out = O.resolve(pos, rgb, fl, vis, sc.cams, sc.width, sc.height, ResolveParams(), sc.mode,
                    sc.bg)
    ds = DeviceScene(sc, cap=cap)
    ds.render()
    torch.cuda.synchronize()
    gp, gr, gf = ds.host_stream()
    assert gp.shape[0] == cap
    assert np.array_equal(gf, fl)
    assert np.array_equal(gp.view(np.uint32), pos.view(np.uint32))
    assert np.array_equal(ds.host_vis(), vis)
    assert _rgba_err(ds.out.cpu().numpy(), out, vis, "truncated") <= TOL


def test_refined_reciprocal_is_correctly_rounded(torch):
    """The raster computes the depth's 1/z with the hardware reciprocal plus one
    Newton step when the camera keeps every 1/z within [2^-126, 2^126); that
    must equal the correctly rounded division bit for bit for every binary32
    value there (all 2.1e9 of them are tried)."""
    lo, hi = 0x00800000, 0x7E800000
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    hm.bench_reciprocal(lo, hi, counts)
    torch.cuda.synchronize()
    bad, seen = (int(v) & 0xFFFFFFFF for v in counts.cpu().numpy())
    assert seen == hi - lo
    assert bad == 0
