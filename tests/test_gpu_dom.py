"""GPU parity of the deep-opacity-map shadows (Sec. 3.4) with the LOD depth
correction (Sec. 3.2.3): the light view's visibility buffer and the per-layer
fragment counts bit for bit, the transmittance within 1e-6 and the shadowed
RGBA within 1e-4 of the oracle, on the same seeded scenes."""
import numpy as np
import pytest

from paper_2607_04230_amd import scenes
from paper_2607_04230_amd.scenes import ResolveParams, ShadowParams

pytestmark = pytest.mark.gpu

TOL = 1e-4
TOL_T = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _oracle_shadowed(O, sc, shp):
    with O.threads(O.host_threads()):
        return _oracle_shadowed_1(O, sc, shp)


def _oracle_shadowed_1(O, sc, shp):
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, table, ncp)
    vis = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    light = scenes.light_camera(sc, shp)
    lvis = O.raster(pos, fl, np.array([0, ncp], np.uint32), light, shp.width, shp.height,
                    shp.r_min)
    counts = O.dom_accumulate(pos, fl, light[0], shp.width, shp.height, shp.r_min, lvis[0],
                              shp.layer_codes(), n_layers=shp.n_layers)
    T = O.dom_shadow(pos, fl, vis[0, 0], sc.cams[0], sc.width, sc.height, light[0], shp.width,
                     shp.height, lvis[0], counts, shp.layer_codes(), table, sc.bundle_nstrands,
                     shp.alpha)
    out = O.resolve(pos, rgb, fl, vis, sc.cams, sc.width, sc.height, ResolveParams(), sc.mode,
                    sc.bg, shadow=T[None])
    return dict(table=table, vis=vis, lvis=lvis, counts=counts, T=T, out=out)


def _check(O, torch, sc, shp, label):
    from paper_2607_04230_amd.render import DeviceScene
    print(f"[dom] {label}: {sc.width}x{sc.height}, light {shp.width}x{shp.height}, "
          f"{shp.n_layers} layers of {shp.layer_codes()} codes", flush=True)
    ds = DeviceScene(sc)
    ds.render_shadowed(shp)
    torch.cuda.synchronize()
    ref = _oracle_shadowed(O, sc, shp)
    assert np.array_equal(ds.table.cpu().numpy().view(np.uint32), ref["table"])
    assert np.array_equal(ds.host_vis(), ref["vis"])
    assert np.array_equal(ds.light_vis.cpu().numpy().view(np.uint64), ref["lvis"])
    gc = ds.dom_counts.cpu().numpy().view(np.uint32)
    assert np.array_equal(gc, ref["counts"]), f"{label}: counts differ at " \
        f"{np.argwhere(gc != ref['counts'])[:5].tolist()}"
    assert ref["counts"][1:].sum() > 0          # fragments behind the first layer
    gT = ds.shadow.cpu().numpy().astype(np.float64)
    assert np.abs(gT - ref["T"]).max() <= TOL_T, label
    shadowed = ref["T"] < 0.99
    assert shadowed.sum() > 100, label
    gout = ds.out.cpu().numpy().astype(np.float64)
    assert np.abs(gout - ref["out"]).max() <= TOL, label
    return ds, ref


def test_tiny_shadowed(O, torch):
    sc = scenes.config_tiny()
    _check(O, torch, sc, ShadowParams(width=128, height=128, distance=3.0, layer_world=0.02),
           "tiny")


def test_head_shadowed_center_and_filter(O, torch):
    sc = scenes.config_head(width=640, height=360, strands_per_quad=16)
    shp = ShadowParams(width=256, height=256)
    ds, ref = _check(O, torch, sc, shp, "head filter")
    # re-render the same frame centre-only: the shadow multiplies the direct terms
    from paper_2607_04230_amd import hm
    ds.sp.mode = hm.RESOLVE_CENTER
    ds.resolve()
    torch.cuda.synchronize()
    pos, rgb, fl = ds.host_stream()
    out = O.resolve(pos, rgb, fl, ref["vis"], sc.cams, sc.width, sc.height, ResolveParams(), 2,
                    sc.bg, shadow=ref["T"][None])
    assert np.abs(ds.out.cpu().numpy().astype(np.float64) - out).max() <= TOL


def test_head_1080p_shadowed_with_a_1024_map(O, torch):
    """The benchmarked shadow workload: the full head at 1920x1080 with a
    1024^2 deep opacity map of 4 layers."""
    sc = scenes.config_head()
    _check(O, torch, sc, ShadowParams(width=1024, height=1024), "head 1080p, 1024^2 map")


def test_lod_scene_shadowed(O, torch):
    """LOD on: bundles that lost strands query the map at a corrected depth."""
    sc = scenes.config_lod(width=640, height=360, n_heads=3, d_near=6.0, d_far=14.0)
    table, _, _ = O.lod_select(sc)
    ns = table[:, 0].astype(np.int64)
    assert ((ns > 0) & (ns < sc.bundle_nstrands)).sum() > 1000
    shp = ShadowParams(width=384, height=384, distance=20.0, vfov_deg=40.0, znear=1.0,
                       zfar=50.0, layer_world=0.05)
    _check(O, torch, sc, shp, "lod")


def test_shadow_calls_are_repeatable(O, torch):
    """Counts are overwritten, not accumulated, by a second call."""
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_tiny()
    shp = ShadowParams(width=128, height=128, distance=3.0, layer_world=0.02)
    ds = DeviceScene(sc)
    ds.render_shadowed(shp)
    torch.cuda.synchronize()
    c1, t1 = ds.dom_counts.clone(), ds.shadow.clone()
    ds.shadows(shp)
    torch.cuda.synchronize()
    assert torch.equal(c1, ds.dom_counts) and torch.equal(t1, ds.shadow)


def test_light_seeing_nothing_leaves_the_frame_unshadowed(O, torch):
    """A light camera whose depth range ends before the groom sees no strand:
    the map is empty, every T is 1 and the shadowed frame equals the
    unshadowed one bit for bit."""
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_tiny()
    shp = ShadowParams(width=64, height=64, distance=-3.0, znear=0.1, zfar=0.5)
    ds = DeviceScene(sc)
    ds.render()
    torch.cuda.synchronize()
    plain = ds.out.clone()
    ds.shadows(shp)
    ds.resolve()
    torch.cuda.synchronize()
    assert (ds.light_vis.cpu().numpy().view(np.uint64) == np.uint64(0xFFFFFFFFFFFFFFFF)).all()
    assert int(ds.dom_counts.sum().item()) == 0
    assert bool((ds.shadow == 1.0).all())
    assert torch.equal(ds.out, plain)


def test_empty_camera_view_has_unit_shadow(O, torch):
    """Every segment behind the camera: no centre hit, so T = 1 everywhere
    while the light's map still counts the groom's fragments."""
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_tiny()
    sc.cams = scenes.look_at_camera((0.0, 1.3, 2.6), (0.0, 1.3, 6.0), sc.width,
                                    sc.height)[None].astype(np.float32)
    shp = ShadowParams(width=128, height=128, distance=3.0, layer_world=0.02)
    ds = DeviceScene(sc)
    ds.render_shadowed(shp)
    torch.cuda.synchronize()
    assert int(ds.dom_counts.sum().item()) > 0
    assert bool((ds.shadow == 1.0).all())
    assert (ds.out.cpu().numpy()[..., 3] == 0.0).all()
