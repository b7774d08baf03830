"""GPU parity at full size on the LOD (32 heads, 1440p) and batched (64 scenes)
workloads against the oracle (run on the host's cores; its threaded loops give
the sequential results): LOD table and strand stream, both visibility layers
of every pixel bit for bit, every RGBA pixel within 1e-4; plus equivalence of
the batched launch with per-scene launches and of HIP-graph replays with the
eager frame."""
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


def _render(sc, torch):
    from paper_2607_04230_amd.render import DeviceScene
    ds = DeviceScene(sc)
    ds.render()
    torch.cuda.synchronize()
    return ds


def _check_stream(ds, table, soff, ncp, pos, rgb, fl):
    assert np.array_equal(ds.table.cpu().numpy().view(np.uint32), table)
    assert np.array_equal(ds.scene_off.cpu().numpy().view(np.uint32), soff)
    gp, gr, gf = ds.host_stream()
    assert gp.shape[0] == ncp
    assert np.array_equal(gf, fl)
    assert np.array_equal(gp.view(np.uint32), pos.view(np.uint32))
    assert np.array_equal(gr.view(np.uint32), rgb.view(np.uint32))


def test_lod_workload_whole_frame(O, torch):
    """The whole 2560x1440 frame of 32 heads: LOD table, stream, both
    visibility layers bit for bit and every RGBA pixel within 1e-4."""
    sc = scenes.config_lod()
    ref = O.render(sc, n_threads=O.host_threads())
    assert ref["n_strands"] < sc.n_full_strands      # LOD removed strands
    ds = _render(sc, torch)
    _check_stream(ds, ref["table"], ref["scene_off"], ref["n_cp"], ref["pos_w"], ref["rgb"],
                  ref["flags"])
    gvis = ds.host_vis()
    assert np.array_equal(gvis, ref["vis"])
    assert (ref["vis"] != EMPTY).sum() > 100000
    gout = ds.out.cpu().numpy().astype(np.float64)
    assert np.abs(gout - ref["out"]).max() <= TOL


def test_lod_depth_offset_matches_oracle(O, torch):
    sc = scenes.config_lod()
    table, _, _ = O.lod_select(sc)
    ds = _render(sc, torch)
    delta = torch.empty(sc.n_bundles, dtype=torch.float32, device="cuda")
    hm.lod_depth_offset(ds.table, ds.mesh_t["bundle_nstrands"], delta)
    torch.cuda.synchronize()
    got = delta.cpu().numpy().astype(np.float64)
    ref = O.lod_depth_offset(table, sc.bundle_nstrands)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isinf(got), ~fin)
    assert np.abs(got[fin] - ref[fin]).max() <= 1e-6
    assert (ref[fin] > 0).any()            # some bundles lost strands


@pytest.fixture(scope="module")
def batched(O, torch):
    sc = scenes.config_batched()
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, table, ncp)
    ds = _render(sc, torch)
    return sc, table, soff, ncp, pos, rgb, fl, ds


def test_batched_workload_every_scene(O, torch, batched):
    """All 64 scenes of the batched frame: both visibility layers bit for bit
    and every RGBA pixel within 1e-4 of the oracle."""
    sc, table, soff, ncp, pos, rgb, fl, ds = batched
    _check_stream(ds, table, soff, ncp, pos, rgb, fl)
    rp = ResolveParams()
    with O.threads(O.host_threads()):
        vis = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
        out = O.resolve(pos, rgb, fl, vis, sc.cams, sc.width, sc.height, rp, sc.mode, sc.bg)
    gvis = ds.host_vis()
    gout = ds.out.cpu().numpy().astype(np.float64)
    for s in range(sc.n_scenes):
        assert np.array_equal(gvis[s], vis[s]), f"scene {s}"
        assert np.abs(gout[s] - out[s]).max() <= TOL, f"scene {s}"


def test_batched_equals_per_scene_launches(torch, batched):
    from paper_2607_04230_amd.render import DeviceScene
    sc, table, soff, ncp, pos, rgb, fl, ds = batched
    for s in (0, 17, 40):
        one = scenes.select_scene(sc, s)
        d1 = DeviceScene(one)
        d1.render()
        torch.cuda.synchronize()
        v1 = d1.host_vis()[0]
        vb = ds.host_vis()[s]
        ids1, idsb = v1 & np.uint64((1 << 40) - 1), vb & np.uint64((1 << 40) - 1)
        hit = (v1 != EMPTY) & (ids1 != np.uint64((1 << 40) - 2))
        assert np.array_equal(v1 >> np.uint64(40), vb >> np.uint64(40))
        assert np.array_equal(ids1[hit] + np.uint64(soff[s]), idsb[hit])
        assert np.array_equal(d1.out.cpu().numpy()[0], ds.out.cpu().numpy()[s])


def test_graph_replays_match_eager(torch):
    from paper_2607_04230_amd.render import DeviceScene
    sc = scenes.config_head(width=640, height=360, strands_per_quad=16)
    ds = DeviceScene(sc)
    ds.render()
    torch.cuda.synchronize()
    ref_vis, ref_out = ds.vis.clone(), ds.out.clone()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g = ds.capture_graph()
        for rep in range(3):
            ds.vis.fill_(0)
            ds.out.fill_(-1.0)
            ds.pos_w.zero_()
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(ds.vis, ref_vis), rep
            assert torch.equal(ds.out, ref_out), rep
            x = torch.randn(1000, device="cuda").sum()          # eager work in between
            torch.cuda.synchronize()
    g.close()


def test_multiview_one_stream_many_views(O, torch):
    """Strands assembled once, projected into several views (stereo pair plus a
    side view): each view equals the oracle's single-view render of the same
    stream."""
    from paper_2607_04230_amd.render import DeviceScene
    base = scenes.config_head(width=640, height=360, strands_per_quad=16, occluder=False)
    views = np.stack([base.cams[0],
                      scenes.look_at_camera((0.065, 0.4, 4.0), (0.0, 0.4, 0.0), 640, 360),
                      scenes.look_at_camera((3.0, 1.2, 2.5), (0.0, 0.4, 0.0), 640, 360)])
    ds = DeviceScene(base)
    ds.lod()
    ds.generate()
    rp = hm.raster_defaults(hm.frame(3, 640, 360))
    rp.shared_views = 1
    fr = hm.frame(3, 640, 360)
    cams = torch.from_numpy(views.copy()).cuda()
    vis = torch.empty((3, 2, 360, 640), dtype=torch.int64, device="cuda")
    ws = torch.empty(hm.workspace_size(hm.CALL_RASTER, fr, cap=ds.cap, rparams=rp),
                     dtype=torch.uint8, device="cuda")
    hm.raster_vis(ds.st, cams, fr, rp, None, vis, ws)
    out = torch.empty((3, 360, 640, 4), dtype=torch.float32, device="cuda")
    wsr = torch.empty(hm.workspace_size(hm.CALL_RESOLVE, fr), dtype=torch.uint8, device="cuda")
    hm.resolve_shade(ds.st, vis, cams, fr, ds.sp, out, wsr)
    torch.cuda.synchronize()
    pos, rgb, fl = ds.host_stream()
    soff = np.array([0, pos.shape[0]], np.uint32)
    gvis = vis.cpu().numpy().view(np.uint64)
    gout = out.cpu().numpy().astype(np.float64)
    rp_ = ResolveParams()
    for v in range(3):
        ref = O.raster(pos, fl, soff, views[v:v + 1], 640, 360, 0.0)
        assert np.array_equal(gvis[v], ref[0]), v
        o = O.resolve(pos, rgb, fl, ref, views[v:v + 1], 640, 360, rp_, base.mode, base.bg)
        assert np.abs(gout[v] - o[0]).max() <= TOL, v


def _with_empty_scenes(n_used):
    """A batch whose scenes 0, 2, 4, ... and the last have no bundles: scene s
    of the builder becomes scene 2s + 1 of 2 n_used + 2 (every scene keeps a
    valid camera)."""
    sc = scenes.config_batched(n_scenes=n_used, res=64, n_min=1e3, n_max=4e3)
    S = 2 * n_used + 2
    cams = np.repeat(sc.cams[:1], S, axis=0).copy()
    cams[1::2][:n_used] = sc.cams
    sc.cams = cams
    sc.bundle_scene = (2 * sc.bundle_scene.astype(np.int64) + 1).astype(np.uint32)
    sc.scene_z = None
    return sc


@pytest.mark.parametrize("n_used", [3, 5], ids=["one-workgroup-lod", "multi-workgroup-lod"])
def test_scene_offsets_with_scenes_without_bundles(O, torch, n_used):
    """Scenes without bundles start at the next used scene's first CP (the
    total after the last bundle). 6000 bundles take the one-workgroup LOD
    pass, 10000 the multi-workgroup one; both match the oracle's table and
    offsets, and the stream generated from them matches too."""
    from paper_2607_04230_amd.render import DeviceScene
    sc = _with_empty_scenes(n_used)
    assert sc.n_bundles == 2000 * n_used
    table, soff, (ns, ncp) = O.lod_select(sc)
    assert soff[0] == 0 and soff[-1] == ncp
    assert all(soff[2 * s] == soff[2 * s + 1] for s in range(n_used + 1))
    pos, rgb, fl = O.generate(sc, table, ncp)
    ds = DeviceScene(sc)
    ds.lod()
    ds.generate()
    torch.cuda.synchronize()
    tot = ds.totals.cpu().numpy()
    assert (int(tot[0]), int(tot[1])) == (ns, ncp)
    _check_stream(ds, table, soff, ncp, pos, rgb, fl)
