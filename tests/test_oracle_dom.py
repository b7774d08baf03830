"""Pins of the oracle's deep-opacity-map shadows (Sec. 3.4, map after Yuksel &
Keyser 2008) and their LOD depth correction (Sec. 3.2.3): per-pixel counts
against one-segment rasters, layer placement of two strands a known depth
apart, the transmittance of a hand-placed shaded point in closed form, the
limits of the correction and of the opacity, and the place of the shadow
factor in the shading (direct terms only)."""
import math

import numpy as np
import pytest

from paper_2607_04230_amd import scenes
from paper_2607_04230_amd.scenes import ResolveParams

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
W = H = 32
F = 400.0                  # light focal length (px): one pixel is 1/400 world unit at z = 1
ZN, ZF = 0.5, 2.0
L = 100_000                # layer thickness in depth codes
L_WORLD = L / 16777216.0 * (ZF - ZN)


def _light():
    """Pinhole at the origin looking +z, principal point at pixel (0, 0):
    world (X, Y, Z) lands on pixel (F X / Z, -F Y / Z)."""
    c = np.zeros(18, np.float32)
    c[0] = c[4] = c[8] = 1.0
    c[12] = c[13] = F
    c[16], c[17] = ZN, ZF
    return c


def _strand(z, y_px, xs_px, w_px):
    """A straight strand parallel to the image plane at depth z along pixel row
    y_px, control points at pixel abscissae xs_px, projected width w_px."""
    pos = np.array([[x * z / F, -y_px * z / F, z, w_px * z / F] for x in xs_px], np.float32)
    fl = np.zeros(len(xs_px), np.uint8)
    fl[0], fl[-1] = 1, 2
    return pos, fl


def _two_strands(dz_layers=2.5):
    z1 = 1.0
    z2 = z1 + dz_layers * L_WORLD
    p1, f1 = _strand(z1, 12.7, [3.3, 11.6, 19.2, 27.4], 1.3)
    p2, f2 = _strand(z2, 12.7, [1.4, 9.9, 20.7, 30.2], 1.3)
    return np.concatenate([p1, p2]), np.concatenate([f1, f2]), z1, z2


def _light_vis(O, pos, fl, r_min=0.0):
    soff = np.array([0, pos.shape[0]], np.uint32)
    return O.raster(pos, fl, soff, _light()[None], W, H, r_min)[0]


def _solo_cover(O, pos, fl, r_min=0.0):
    """Per segment: its conservative pixel set, rasterized alone."""
    out = []
    for v in range(pos.shape[0] - 1):
        if fl[v] & 2:
            continue
        sp = pos[v:v + 2].copy()
        sf = np.array([1, 2], np.uint8)
        vis = O.raster(sp, sf, np.array([0, 2], np.uint32), _light()[None], W, H, r_min)[0]
        out.append((v, vis[1] != EMPTY))
    return out


@pytest.mark.parametrize("r_min", [0.0, 0.7])
def test_counts_equal_per_segment_rasters(O, r_min):
    """Summed over layers, a light pixel's count is the number of segments
    whose own conservative raster reaches it."""
    pos, fl, _, _ = _two_strands()
    lv = _light_vis(O, pos, fl, r_min)
    counts = O.dom_accumulate(pos, fl, _light(), W, H, r_min, lv, L, n_layers=4)
    ref = np.zeros((H, W), np.int64)
    for _, m in _solo_cover(O, pos, fl, r_min):
        ref += m
    assert ref.sum() > 100
    assert np.array_equal(counts.sum(0).astype(np.int64), ref)


@pytest.mark.parametrize("n_layers,layer2", [(4, 2), (3, 2), (2, 1), (1, 0)])
def test_layer_of_a_strand_behind_another(O, n_layers, layer2):
    """The far strand, 2.5 layers behind the near one, lands in layer 2
    (clamped to the last layer) wherever the near strand is in front, and in
    layer 0 where it is the nearest fragment itself."""
    pos, fl, _, _ = _two_strands()
    lv = _light_vis(O, pos, fl)
    counts = O.dom_accumulate(pos, fl, _light(), W, H, 0.0, lv, L, n_layers=n_layers)
    n1 = np.zeros((H, W), np.int64)
    n2 = np.zeros((H, W), np.int64)
    for v, m in _solo_cover(O, pos, fl):
        (n1 if v < 4 else n2)[m] += 1
    front = n1 > 0
    exp = np.zeros((n_layers, H, W), np.int64)
    exp[0] += n1
    exp[layer2][front] += n2[front]
    exp[0][~front] += n2[~front]
    assert (front & (n2 > 0)).sum() > 20 and (~front & (n2 > 0)).sum() > 4
    assert np.array_equal(counts.astype(np.int64), exp)


def _shadow_setup(O, beta_den=1, alpha=0.05, n_layers=4):
    """Camera = light; a hand-made camera visibility buffer names far-strand
    segment 5 (pixel abscissae 9.9 .. 20.7) at row 12, columns 12 .. 17, so
    the shaded point of pixel (i, 12) is (i + 0.5, 12.7) on the far strand,
    in light pixel (i, 12), behind the near strand."""
    pos, fl, z1, z2 = _two_strands()
    lv = _light_vis(O, pos, fl)
    counts = O.dom_accumulate(pos, fl, _light(), W, H, 0.0, lv, L, n_layers=n_layers)
    vis = np.full((H, W), EMPTY, np.uint64)
    q_cam = np.uint64(1000) << np.uint64(40)
    cols = list(range(12, 18))
    for i in cols:
        vis[12, i] = q_cam | np.uint64(5)
    table = np.array([[1, 4, 0, 0], [1, 4, 1, 4]], np.uint32)
    nstr = np.array([1, beta_den], np.uint32)
    T = O.dom_shadow(pos, fl, vis, _light(), W, H, _light(), W, H, lv, counts, L, table, nstr,
                     alpha)
    return T, counts, lv, cols, z2


def test_shadow_of_a_point_behind_a_strand(O):
    alpha = 0.05
    T, counts, lv, cols, z2 = _shadow_setup(O, alpha=alpha)
    a32 = float(np.float32(alpha))
    # depth code of the shaded point, binary64 linear depth (X.z = z2 exactly)
    q = int((float(np.float32(z2)) - ZN) / (ZF - ZN) * 16777216.0)
    for i in cols:
        q0 = int(lv[1, 12, i] >> np.uint64(40))
        d = q - q0
        assert 2 * L < d < 3 * L
        f = (d - 2 * L) / L
        o = counts[0, 12, i] + counts[1, 12, i] + f * counts[2, 12, i]
        assert counts[0, 12, i] > 0 and counts[1, 12, i] == 0 and counts[2, 12, i] > 0
        assert T[12, i] == pytest.approx(math.exp(-a32 * o), rel=1e-12)
        # the opacity lies between the full layers before the point and all of them
        assert math.exp(-a32 * counts[:3, 12, i].sum()) < T[12, i] < math.exp(-a32 * counts[0, 12, i])
    other = np.ones_like(T, bool)
    other[12, cols] = False
    assert (T[other] == 1.0).all()


def test_lod_correction_moves_the_point_towards_the_light(O):
    """beta = N_LOD / N_b < 1 shortens the depth below the first fragment:
    less opacity in front; beta -> 0 reaches the first fragment (T = 1)."""
    T1 = _shadow_setup(O, beta_den=1)[0]
    Th = _shadow_setup(O, beta_den=2)[0]
    T0, _, _, cols, _ = _shadow_setup(O, beta_den=100_000_000)
    r = np.s_[12, cols[0]:cols[-1] + 1]
    assert (Th[r] > T1[r]).all()
    assert (T0[r] == 1.0).all()


def test_shadow_limits(O):
    """A vanishing opacity gives T = 1; the last layer is taken whole once passed."""
    T, *_ = _shadow_setup(O, alpha=1e-30)
    assert np.all(np.abs(T - 1.0) < 1e-20)
    # two layers: the far strand (2.5 layers back) is past the last layer's
    # start, f = min((d - L) / L, 1) = 1, so its own fragments count whole
    T2, counts, _, cols, _ = _shadow_setup(O, n_layers=2)
    a32 = float(np.float32(0.05))
    for i in cols:
        o = counts[0, 12, i] + counts[1, 12, i]
        assert T2[12, i] == pytest.approx(math.exp(-a32 * o), rel=1e-12)


def _resolve_inputs(O):
    sc = scenes.config_tiny(width=96, height=96)
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, table, ncp)
    vis = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    return sc, pos, rgb, fl, vis


@pytest.mark.parametrize("mode", [0, 2])
def test_unit_shadow_is_the_unshadowed_resolve(O, mode):
    sc, pos, rgb, fl, vis = _resolve_inputs(O)
    rp = ResolveParams()
    a = O.resolve(pos, rgb, fl, vis, sc.cams, sc.width, sc.height, rp, mode, sc.bg)
    b = O.resolve(pos, rgb, fl, vis, sc.cams, sc.width, sc.height, rp, mode, sc.bg,
                  shadow=np.ones((1, sc.height, sc.width)))
    assert np.array_equal(a, b)


def test_full_shadow_leaves_the_ambient_term(O):
    """With T = 0 and a constant albedo c the centre shading is c * E * ka."""
    sc, pos, rgb, fl, vis = _resolve_inputs(O)
    c = np.array([0.6, 0.35, 0.2], np.float32)
    rgb = rgb.copy()
    rgb[:, :3] = c
    rp = ResolveParams()
    out = O.resolve(pos, rgb, fl, vis, sc.cams, sc.width, sc.height, rp, 2, sc.bg,
                    shadow=np.zeros((1, sc.height, sc.width)))[0]
    ids = vis[0, 0] & np.uint64((1 << 40) - 1)
    hit = (vis[0, 0] != EMPTY) & (ids != np.uint64((1 << 40) - 2))
    assert hit.sum() > 50
    ref = c.astype(np.float64) * np.asarray(rp.light_rgb, np.float64) * rp.ka
    np.testing.assert_allclose(out[hit][:, :3], np.broadcast_to(ref, (hit.sum(), 3)),
                               rtol=1e-12, atol=0)
