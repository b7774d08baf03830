"""Pins of the CPU oracle's hash, LOD and strand generation against values the
paper's equations fix, closed forms and special cases (no GPU needed)."""
import math

import numpy as np
import pytest

from paper_2607_04230_amd import scenes


# ------------------------------------------------------------------ hash
def test_pcg_is_a_permutation_and_mixes(O):
    xs = np.arange(1 << 16, dtype=np.uint32) * np.uint32(40503)
    hs = np.array([O.pcg(int(x)) for x in xs], np.uint64)
    assert np.unique(hs).size == xs.size                    # no collisions (bijection)
    # avalanche: one flipped input bit flips about half of the output bits
    flips = []
    for x in range(0, 4000, 7):
        h = O.pcg(x)
        for b in range(0, 32, 5):
            flips.append(bin(h ^ O.pcg(x ^ (1 << b))).count("1"))
    assert 14.5 < np.mean(flips) < 17.5


def test_strand_uv_uniform_and_independent(O):
    uv = np.array([O.strand_rand(1001, key, k) for key in range(200) for k in range(100)])
    assert (uv >= 0).all() and (uv < 1).all()
    for c in range(3):
        hist, _ = np.histogram(uv[:, c], bins=20, range=(0, 1))
        chi2 = ((hist - uv.shape[0] / 20) ** 2 / (uv.shape[0] / 20)).sum()
        assert chi2 < 45.0                                  # 19 dof, p ~ 1e-3
    cc = np.corrcoef(uv.T)
    assert abs(cc[0, 1]) < 0.03 and abs(cc[0, 2]) < 0.03 and abs(cc[1, 2]) < 0.03
    # seeds and keys change the stream
    assert not np.array_equal(O.strand_rand(1, 5, 0), O.strand_rand(2, 5, 0))
    assert not np.array_equal(O.strand_rand(1, 5, 0), O.strand_rand(1, 6, 0))


# ------------------------------------------------------------------ LOD counts
# Values worked by hand from eqs. (strand-lod), (cp-lod), (cp-snap) in binary32.
@pytest.mark.parametrize("L,cmax,nl,expect", [
    (1.0, 127, 6, 65), (0.5, 127, 6, 65), (0.25, 127, 6, 33), (0.2, 127, 6, 33),
    (0.01, 127, 6, 9), (0.0004, 127, 6, 5),
    (1.0, 17, 6, 17), (0.5, 17, 6, 9), (0.25, 17, 6, 5), (0.01, 17, 6, 5),
    (0.0004, 127, 4, 3), (1.0, 17, 2, 17), (0.0, 17, 2, 2),
])
def test_lod_control_points(O, L, cmax, nl, expect):
    _, c = O.lod_counts(L, 64, 0.0, cmax, nl)
    assert c == expect


@pytest.mark.parametrize("L,N,delta,expect", [
    (0.5, 64, 0.25, 33), (1.0, 64, 0.5, 64), (0.0, 64, 0.7, 1), (0.3, 16, 0.1, 5),
    (1.0, 1, 0.99, 1), (0.125, 64, 0.0, 8), (0.125, 64, 0.01, 9),
])
def test_lod_strand_count(O, L, N, delta, expect):
    n, _ = O.lod_counts(L, N, delta, 17, 6)
    assert n == expect


def _cam_identity(width, height, f=100.0, znear=0.1, zfar=100.0):
    c = np.zeros(18, np.float32)
    c[0] = c[4] = c[8] = 1.0          # camera at origin looking +z, y up
    c[12] = c[13] = f
    c[14], c[15] = width / 2.0, height / 2.0
    c[16], c[17] = znear, zfar
    return c


def _quad_scene(centre, side, depth, width=200, height=100, lam=1.0, n_layers=2, mode=1):
    """One bundle: fronto-parallel square layers of side `side` at camera z = depth."""
    cx, cy = centre
    corners = np.array([[cx - side / 2, cy - side / 2], [cx + side / 2, cy - side / 2],
                        [cx + side / 2, cy + side / 2], [cx - side / 2, cy + side / 2]])
    lp = np.zeros((n_layers, 4, 3), np.float32)
    for l in range(n_layers):
        lp[l, :, :2] = corners
        lp[l, :, 2] = depth
    ns, cm, sc, ky, base = scenes._bundle_arrays(1, 64, 17)
    cam = _cam_identity(width, height)[None]
    return scenes.Scene("quad", lp, np.arange(4, dtype=np.uint32)[None], ky, ns, cm, sc, base,
                        None, cam, width, height, None, lod_mode=mode, lod_lambda=lam)


def test_lod_value_closed_form(O):
    # projected AABB of a fronto-parallel square of side s at depth z is f s / z square:
    # L = sqrt(2) f s / z / R_y * lambda
    f, H = 100.0, 100
    for side, depth, lam in [(0.1, 2.0, 3.0), (0.05, 10.0, 7.0), (0.3, 5.0, 1.0)]:
        sc = _quad_scene((0.0, 0.0), side, depth, height=H, lam=lam)
        table, _, _ = O.lod_select(sc)
        L = min(math.sqrt(2.0) * f * side / depth / H * lam, 1.0)
        n_exp, c_exp = O.lod_counts(L, 64, O.lod_delta(sc.seed, 0), 17, 2)
        assert tuple(table[0, :2]) == (n_exp, c_exp)
        assert n_exp == max(1, min(64, math.ceil(L * (64 + O.lod_delta(sc.seed, 0)))))


def test_lod_cull_and_near(O):
    # fully left of the viewport -> culled
    sc = _quad_scene((-20.0, 0.0), 0.1, 2.0)
    t, _, tot = O.lod_select(sc)
    assert t[0, 0] == 0 and tot == (0, 0)
    # behind the camera -> culled
    sc = _quad_scene((0.0, 0.0), 0.1, -2.0)
    t, _, _ = O.lod_select(sc)
    assert t[0, 0] == 0
    # straddling the near plane -> full detail
    sc = _quad_scene((0.0, 0.0), 0.1, 2.0, n_layers=2)
    sc.layer_pos[0, :, 2] = 0.05
    t, _, _ = O.lod_select(sc)
    assert tuple(t[0, :2]) == (64, 17)
    # LOD off: N and C_max regardless of size
    sc = _quad_scene((0.0, 0.0), 0.001, 50.0, mode=0)
    t, _, tot = O.lod_select(sc)
    assert tuple(t[0]) == (64, 17, 0, 0) and tot == (64, 64 * 17)


def test_lod_prefix_sums_and_scene_offsets(O):
    sc = scenes.config_batched(n_scenes=5, n_min=500, n_max=5000)
    t, soff, (ns, ncp) = O.lod_select(sc)
    n = t[:, 0].astype(np.int64)
    c = t[:, 1].astype(np.int64)
    assert (t[:, 2] == np.concatenate([[0], np.cumsum(n)[:-1]])).all()
    assert (t[:, 3] == np.concatenate([[0], np.cumsum(n * c)[:-1]])).all()
    assert ns == n.sum() and ncp == (n * c).sum()
    for s in range(5):
        first = np.nonzero(sc.bundle_scene == s)[0][0]
        assert soff[s] == t[first, 3]
    assert soff[5] == ncp


def test_lod_depth_offset_closed_forms(O):
    # half the strands kept -> ln 2; nothing removed -> 0 (Sec. 3.2.3); all
    # removed -> +inf; an empty bundle -> 0
    table = np.array([[32, 9, 0, 0], [64, 17, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0], [16, 5, 0, 0]],
                     np.uint32)
    N = np.array([64, 64, 64, 0, 64], np.uint32)
    d = O.lod_depth_offset(table, N)
    assert d[0] == pytest.approx(math.log(2.0), abs=1e-15)
    assert d[1] == 0.0 and math.isinf(d[2]) and d[3] == 0.0
    assert d[4] == pytest.approx(2.0 * math.log(2.0), abs=1e-15)
    # Beer-Lambert: exp(-sigma * beta * d) == exp(-sigma * d) shifted by delta in log-depth
    beta, sigma, depth = 0.25, 3.0, 0.7
    assert math.exp(-sigma * beta * depth) == pytest.approx(
        math.exp(-sigma * math.exp(math.log(depth) - (-math.log(beta)))), rel=1e-12)


# ------------------------------------------------------------------ generation
def test_taylor_sin_cos_match_libm(O):
    for a in np.linspace(-math.pi, math.pi, 2001, endpoint=False):
        a32 = float(np.float32(a))
        assert abs(O.sin32(a32) - math.sin(a32)) < 1e-6
        assert abs(O.cos32(a32) - math.cos(a32)) < 1e-6


def _straight_scene(n_layers=4, C=13, curl=0.0, axis=(0.0, 1.0, 0.0), spacing=0.25):
    """One bundle whose layers are translated copies along `axis`, evenly spaced."""
    axis = np.asarray(axis, np.float64)
    axis /= np.linalg.norm(axis)
    base = np.array([[0.1, 0.0, 0.2], [0.3, 0.05, 0.2], [0.35, 0.0, 0.45], [0.05, 0.02, 0.4]])
    lp = np.stack([base + axis * spacing * l for l in range(n_layers)]).astype(np.float32)
    ns, cm, sc, ky, sb = scenes._bundle_arrays(1, 8, C)
    cam = scenes.look_at_camera((0, 0.5, 3), (0, 0.5, 0), 64, 64)[None]
    return scenes.Scene("straight", lp, np.arange(4, dtype=np.uint32)[None], ky, ns, cm, sc, sb,
                        None, cam, 64, 64, None, curl_amp=curl, strand_width=0.01)


def _bilinear(lp_layer, u, v):
    A, B, C, D = (lp_layer[i].astype(np.float64) for i in range(4))
    return (1 - u) * (1 - v) * A + u * (1 - v) * B + u * v * C + (1 - u) * v * D


def test_generation_straight_bundle_is_linear(O):
    sc = _straight_scene()
    t, _, (_, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, t, ncp)
    C, L = 13, 4
    for k in range(8):
        u, v, _ = O.strand_rand(sc.seed, 0, k)
        root = _bilinear(sc.layer_pos[0], u, v)
        tip = _bilinear(sc.layer_pos[L - 1], u, v)
        for j in range(C):
            w = j / (C - 1)
            exp = root + w * (tip - root)             # Hermite of collinear equal steps is linear
            assert np.abs(pos[k * C + j, :3] - exp).max() < 2e-6
        assert fl[k * C] == 1 and fl[k * C + C - 1] == 2 and (fl[k * C + 1:k * C + C - 1] == 0).all()
    assert (pos[:, 3] == np.float32(0.01)).all()
    assert (rgb[:, :3] == np.asarray(sc.base_rgb, np.float32)).all() and (rgb[:, 3] == 1).all()


def test_generation_interpolates_layers(O):
    # curved layers: Hermite passes through the bilinear layer points at w = i/(L-1)
    sc = scenes.config_tiny()
    sc.curl_amp = 0.0
    t, _, (_, ncp) = O.lod_select(sc)
    pos, _, _ = O.generate(sc, t, ncp)
    C, L = 9, 4
    sc.bundle_cmax[:] = 10          # (C-1) = 9 divisible by (L-1) = 3
    t2, _, (_, ncp2) = O.lod_select(sc)
    pos2, _, _ = O.generate(sc, t2, ncp2)
    for b in (0, 17, 63):
        q = sc.quads[b]
        for k in (0, 5, 15):
            u, v, _ = O.strand_rand(sc.seed, int(sc.bundle_key[b]), k)
            base = t2[b, 3] + k * 10
            for i in range(L):
                exp = _bilinear(sc.layer_pos[i][q], u, v)
                assert np.abs(pos2[base + 3 * i, :3] - exp).max() < 2e-6
            # endpoints with C = 9 too
            b9 = t[b, 3] + k * C
            assert np.abs(pos[b9, :3] - _bilinear(sc.layer_pos[0][q], u, v)).max() < 2e-6
            assert np.abs(pos[b9 + C - 1, :3] - _bilinear(sc.layer_pos[L - 1][q], u, v)).max() < 2e-6


def test_generation_curl_is_helix_about_axis(O):
    amp, turns = 0.03, 3.0
    axis = np.array([0.2, 1.0, 0.1])
    axis /= np.linalg.norm(axis)
    sc_c = _straight_scene(curl=amp, axis=axis, C=17)
    sc_0 = _straight_scene(curl=0.0, axis=axis, C=17)
    t, _, (_, ncp) = O.lod_select(sc_c)
    p1, _, _ = O.generate(sc_c, t, ncp)
    p0, _, _ = O.generate(sc_0, t, ncp)
    e1 = np.cross(axis, [0.0, 0.0, 1.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(axis, e1)
    C = 17
    for k in range(8):
        _, _, ph = O.strand_rand(sc_c.seed, 0, k)
        for j in range(C):
            w = j / (C - 1)
            th = 2 * math.pi * (turns * w + ph)
            exp = amp * w * (math.cos(th) * e1 + math.sin(th) * e2)
            assert np.abs(p1[k * C + j, :3] - p0[k * C + j, :3] - exp).max() < 3e-6


def test_generation_colour_routing_and_lod_prefix(O):
    sc = scenes.config_head(width=64, height=36, occluder=False)
    t, _, (_, ncp) = O.lod_select(sc)
    pos, rgb, _ = O.generate(sc, t, ncp)
    for b in (0, 999, 1999):
        for k in (0, 63):
            o = t[b, 3] + k * 17
            assert (rgb[o:o + 17, :3] == sc.strand_rgb[sc.strand_base[b] + k]).all()
    # strand k is the same whatever the bundle's strand count (LOD keeps a prefix)
    sc2 = scenes.config_head(width=64, height=36, occluder=False, strands_per_quad=64)
    sc2.bundle_nstrands[:] = 7
    t2, _, (_, ncp2) = O.lod_select(sc2)
    pos2, _, _ = O.generate(sc2, t2, ncp2)
    for b in (3, 1500):
        for k in range(7):
            assert (pos2[t2[b, 3] + k * 17: t2[b, 3] + (k + 1) * 17] ==
                    pos[t[b, 3] + k * 17: t[b, 3] + (k + 1) * 17]).all()


def test_generate_truncated_stream_rule(O):
    sc = scenes.config_tiny()
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, table, ncp)
    for cap in (1, 2, 17, ncp - 1):
        p2, r2, f2 = O.generate(sc, table, ncp, cap=cap)
        assert p2.shape[0] == cap and np.array_equal(p2, pos[:cap]) and np.array_equal(r2, rgb[:cap])
        assert np.array_equal(f2[:-1], fl[:cap - 1]) and f2[-1] == (fl[cap - 1] | 2)
    p3, _, f3 = O.generate(sc, table, ncp, cap=ncp + 5)
    assert np.array_equal(f3, fl) and p3.shape[0] == ncp
