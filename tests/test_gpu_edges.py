"""GPU parity on the degenerate cases the readings of the method define:

* a bundle that crosses the near plane takes L = 1 (Sec. 3.2: its screen
  AABB is not defined), one entirely behind it is culled;
* a segment with one endpoint outside the open depth range (znear, zfar) is
  not drawn (reading of Sec. 3.1.2: no clipping, the segment is dropped);
* fewer than two control points per strand are taken as two (a strand has at
  least one segment), by the LOD table and by the generator alike.

Everything is compared with the oracle bit for bit (tables, stream, keys) and
RGBA within 1e-4."""
import numpy as np
import pytest

from paper_2607_04230_amd import scenes

pytestmark = pytest.mark.gpu

TOL = 1e-4
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _gpu(sc, torch):
    from paper_2607_04230_amd.render import DeviceScene
    ds = DeviceScene(sc)
    ds.render()
    torch.cuda.synchronize()
    return ds


def _same_as_oracle(ds, ref):
    assert np.array_equal(ds.table.cpu().numpy().view(np.uint32), ref["table"])
    tot = ds.totals.cpu().numpy()
    assert (int(tot[0]), int(tot[1])) == (ref["n_strands"], ref["n_cp"])
    pos, rgb, fl = ds.host_stream()
    assert np.array_equal(fl, ref["flags"])
    assert np.array_equal(pos.view(np.uint32), ref["pos_w"].view(np.uint32))
    assert np.array_equal(ds.host_vis(), ref["vis"])
    err = float(np.abs(ds.out.cpu().numpy().astype(np.float64) - ref["out"]).max())
    assert err <= TOL, err


def _depth_range_scene():
    """A 12-bundle groom whose camera's near plane (z = 2.0) cuts through
    nine bundles and lies wholly in front of one, and whose far plane
    (z = 2.4) cuts the farthest bundle."""
    sc = scenes.micro_scene(11, n_bundles=12, n_layers=4, strands=6, n_cp=9, res=64, width=0.02)
    sc.cams = sc.cams.copy()
    sc.cams[0, 16], sc.cams[0, 17] = 2.0, 2.4
    sc.lod_mode = scenes.LOD_ON
    sc.lod_lambda = 0.05
    return sc


def _bundle_depths(sc):
    R = sc.cams[0, :9].reshape(3, 3).astype(np.float64)
    eye = sc.cams[0, 9:12].astype(np.float64)
    out = []
    for b in range(sc.n_bundles):
        P = sc.layer_pos[:, sc.quads[b]].reshape(-1, 3).astype(np.float64)
        Z = (P - eye) @ R[2]
        out.append((Z.min(), Z.max()))
    return out


def test_near_plane_bundles_and_clipped_segments(O, torch):
    sc = _depth_range_scene()
    ref = O.render(sc)
    zn, zf = float(sc.cams[0, 16]), float(sc.cams[0, 17])
    kinds = {"behind": [], "cross": [], "front": []}
    for b, (lo, hi) in enumerate(_bundle_depths(sc)):
        kinds["behind" if hi <= zn else ("cross" if lo <= zn else "front")].append(b)
    assert kinds["behind"] and len(kinds["cross"]) >= 3 and kinds["front"]
    t = ref["table"]
    N = sc.bundle_nstrands
    for b in kinds["behind"]:
        assert t[b, 0] == 0                       # culled
    for b in kinds["cross"]:
        assert t[b, 0] == N[b] and t[b, 1] == 9   # L = 1: all strands, C = C_max
    assert any(t[b, 0] < N[b] for b in kinds["front"])   # small L elsewhere
    # segments with exactly one endpoint outside (znear, zfar) exist and are not drawn
    pos, fl = ref["pos_w"], ref["flags"]
    inside = np.array([O.project(sc.cams[0], p) is not None for p in pos])
    seg = np.nonzero(((fl & 2) == 0)[:-1])[0]
    one_out = seg[inside[seg] != inside[seg + 1]]
    assert len(one_out) >= 10
    ids = (ref["vis"].astype(np.uint64) & np.uint64((1 << 40) - 1)).astype(np.int64)
    assert not np.isin(one_out, ids).any()
    assert (ref["vis"] != EMPTY).sum() > 100
    ds = _gpu(sc, torch)
    _same_as_oracle(ds, ref)


@pytest.mark.parametrize("lod_mode", [scenes.LOD_OFF, scenes.LOD_ON])
def test_fewer_than_two_control_points(O, torch, lod_mode):
    sc = scenes.micro_scene(4, n_bundles=4, strands=3, n_cp=5, res=48)
    sc.bundle_cmax = np.array([1, 0, 5, 2], np.uint32)
    sc.lod_mode = lod_mode
    ref = O.render(sc)
    assert ref["table"][0, 1] == 2 and ref["table"][1, 1] == 2
    ds = _gpu(sc, torch)
    _same_as_oracle(ds, ref)
