"""Pins of the CPU oracle's rasterization (visibility buffer) against closed
forms, a binary64 brute force of the geometric definitions and the
order-independence of the atomic-min (Sec. 3.1.2)."""
import math

import numpy as np
import pytest

from paper_2607_04230_amd import scenes

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def _cam_unit(width, height, znear=0.5, zfar=2.0):
    """fx = fy = 1, cx = cy = 0, looking +z from the origin: at z = 1 a world
    point (X, Y) lands on pixel coordinates (X, -Y)."""
    c = np.zeros(18, np.float32)
    c[0] = c[4] = c[8] = 1.0
    c[12] = c[13] = 1.0
    c[16], c[17] = znear, zfar
    return c


def _segment_stream(p0, p1, w):
    pos = np.array([[p0[0], p0[1], p0[2], w], [p1[0], p1[1], p1[2], w]], np.float32)
    return pos, np.array([1, 2], np.uint8)


def _raster1(O, pos, fl, cam, W, H, r_min=0.0, brute=True, scene_z=None):
    soff = np.array([0, pos.shape[0]], np.uint32)
    return O.raster(pos, fl, soff, cam[None], W, H, r_min, scene_z, brute=brute)[0]


@pytest.mark.parametrize("x0,ya,yb,w", [(10.3, 3.2, 17.7, 0.8), (5.61, 0.2, 30.9, 2.3),
                                        (20.05, 7.9, 8.3, 0.37), (0.3, -4.2, 40.3, 1.1)])
def test_vertical_strand_closed_form(O, x0, ya, yb, w):
    W, H = 32, 32
    cam = _cam_unit(W, H)
    # world Y = -pixel y at z = 1
    pos, fl = _segment_stream((x0, -ya, 1.0), (x0, -yb, 1.0), w)
    vis = _raster1(O, pos, fl, cam, W, H)
    r = w / 2
    ci = [i for i in range(W) if abs(i + 0.5 - x0) <= r]
    cj = [j for j in range(H) if ya <= j + 0.5 < yb]                     # half-open flat caps
    ai = [i for i in range(W) if x0 - 1 - r <= i <= x0 + r]
    aj = [j for j in range(H) if ya - 1 - r <= j <= yb + r]
    assert (vis[0] != EMPTY).sum() == len(ci) * len(cj)
    assert (vis[1] != EMPTY).sum() == len(ai) * len(aj)
    for i in ci:
        for j in cj:
            assert vis[0, j, i] != EMPTY


@pytest.mark.parametrize("y0,xa,xb,w", [(12.7, 2.2, 25.4, 0.6), (3.05, 30.6, 1.3, 1.7)])
def test_horizontal_strand_closed_form(O, y0, xa, xb, w):
    W, H = 32, 32
    cam = _cam_unit(W, H)
    pos, fl = _segment_stream((xa, -y0, 1.0), (xb, -y0, 1.0), w)
    vis = _raster1(O, pos, fl, cam, W, H)
    r = w / 2
    lo, hi = min(xa, xb), max(xa, xb)
    ci = [i for i in range(W) if (xa <= i + 0.5 < xb) or (xb < i + 0.5 <= xa)]
    cj = [j for j in range(H) if abs(j + 0.5 - y0) <= r]
    ai = [i for i in range(W) if lo - 1 - r <= i <= hi + r]
    aj = [j for j in range(H) if y0 - 1 - r <= j <= y0 + r]
    assert (vis[0] != EMPTY).sum() == len(ci) * len(cj)
    assert (vis[1] != EMPTY).sum() == len(ai) * len(aj)


def test_depth_code_fronto_parallel(O):
    W, H = 16, 16
    for z in (0.6, 1.0, 1.37, 1.99):
        cam = _cam_unit(W, H)
        pos, fl = _segment_stream((2.3 * z, -8.1 * z, z), (13.7 * z, -8.1 * z, z), z)
        vis = _raster1(O, pos, fl, cam, W, H)
        keys = vis[0][vis[0] != EMPTY]
        q = int(keys[0]) >> 40
        exp = math.floor((z - 0.5) / 1.5 * 2 ** 24)
        assert abs(q - exp) <= 2
        assert all((int(k) >> 40) == q for k in keys)
        assert all((int(k) & ((1 << 40) - 1)) == 0 for k in keys)


def _brute64(pa, pb, W, H, r_min):
    """Binary64 geometric definitions on projected endpoints (x, y, w_px, 1/z):
    centre = pixel centre within the local half width of the segment with the
    foot of the perpendicular in [0, 1); conservative = segment meets the pixel
    square dilated by the larger half width.  Returns masks and a margin that
    is small where a binary32 decision could legitimately go either way."""
    x0, y0, w0, _ = map(float, pa)
    x1, y1, w1, _ = map(float, pb)
    ii, jj = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    dx, dy = x1 - x0, y1 - y0
    L2 = dx * dx + dy * dy
    t = ((ii - x0) * dx + (jj - y0) * dy) / L2
    dist = np.abs((ii - x0) * dy - (jj - y0) * dx) / math.sqrt(L2)
    r = np.maximum(0.5 * (w0 + t * (w1 - w0)), r_min)
    centre = (t >= 0) & (t < 1) & (dist <= r)
    m_c = np.minimum(np.minimum(np.abs(t), np.abs(t - 1)) * math.sqrt(L2), np.abs(dist - r))
    ra = max(0.5 * max(w0, w1), r_min)
    cons = np.zeros((H, W), bool)
    m_a = np.full((H, W), np.inf)
    for j in range(H):
        for i in range(W):
            bx0, bx1, by0, by1 = i - ra, i + 1 + ra, j - ra, j + 1 + ra
            # clip the segment to the box (Liang-Barsky in binary64)
            t0, t1, ok = 0.0, 1.0, True
            for p, q in ((-dx, x0 - bx0), (dx, bx1 - x0), (-dy, y0 - by0), (dy, by1 - y0)):
                if p == 0:
                    ok &= q >= 0
                else:
                    tt = q / p
                    if p < 0:
                        t0 = max(t0, tt)
                    else:
                        t1 = min(t1, tt)
            cons[j, i] = ok and t0 <= t1
            # margin: distance from the segment to the box border region
            cxs = [bx0, bx1]
            cys = [by0, by1]
            gaps = [abs((cx - x0) * dy - (cy - y0) * dx) / math.sqrt(L2) for cx in cxs for cy in cys]
            gaps += [abs(x0 - bx0), abs(x0 - bx1), abs(x1 - bx0), abs(x1 - bx1),
                     abs(y0 - by0), abs(y0 - by1), abs(y1 - by0), abs(y1 - by1)]
            m_a[j, i] = min(gaps)
    return centre, cons, m_c, m_a


@pytest.mark.parametrize("seed", range(12))
def test_predicates_match_binary64_geometry(O, seed):
    rng = np.random.default_rng(seed)
    W, H = 24, 24
    cam = _cam_unit(W, H, znear=0.2, zfar=5.0)
    r_min = [0.0, 0.5][seed % 2]
    for _ in range(6):
        z0, z1 = rng.uniform(0.5, 3.0, 2)
        a = np.array([rng.uniform(-2, W + 2), rng.uniform(-2, H + 2)])
        b = a + rng.normal(0, 6, 2)
        w = rng.uniform(0.05, 2.5)
        pos, fl = _segment_stream((a[0] * z0, -a[1] * z0, z0), (b[0] * z1, -b[1] * z1, z1), w)
        pa = O.project(cam, pos[0])
        pb = O.project(cam, pos[1])
        vis = _raster1(O, pos, fl, cam, W, H, r_min=r_min)
        centre, cons, m_c, m_a = _brute64(pa, pb, W, H, r_min)
        ok_c = m_c > 1e-4
        ok_a = m_a > 1e-4
        assert ((vis[0] != EMPTY) == centre)[ok_c].all()
        assert ((vis[1] != EMPTY) == cons)[ok_a].all()
        # depth at the clamped closest point, perspective-correct (binary64)
        jj, ii = np.nonzero(vis[1] != EMPTY)
        for j, i in zip(jj, ii):
            dx, dy = float(pb[0] - pa[0]), float(pb[1] - pa[1])
            t = ((i + 0.5 - pa[0]) * dx + (j + 0.5 - pa[1]) * dy) / (dx * dx + dy * dy)
            t = min(max(t, 0.0), 1.0)
            iz = float(pa[3]) + t * (float(pb[3]) - float(pa[3]))
            q = ((1.0 / iz) - 0.2) / 4.8 * 2 ** 24
            assert abs((int(vis[1, j, i]) >> 40) - q) < 4


def test_brute_force_equals_bbox_enumeration(O):
    for seed in range(6):
        sc = scenes.micro_scene(seed)
        t, soff, (_, ncp) = O.lod_select(sc)
        pos, _, fl = O.generate(sc, t, ncp)
        for r_min in (0.0, 0.5):
            a = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, r_min, brute=False)
            b = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, r_min, brute=True)
            assert np.array_equal(a, b)
    sc = scenes.config_tiny(width=96, height=96)
    t, soff, (_, ncp) = O.lod_select(sc)
    pos, _, fl = O.generate(sc, t, ncp)
    a = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, 0.0, brute=False)
    b = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, 0.0, brute=True)
    assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def tiny(O):
    sc = scenes.config_tiny()
    t, soff, (_, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, t, ncp)
    vis = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height)
    return sc, soff, pos, rgb, fl, vis


def test_order_independence_union_idempotence(O, tiny):
    sc, soff, pos, _, fl, vis = tiny
    n = pos.shape[0]
    rng = np.random.default_rng(7)
    perm = rng.permutation(n).astype(np.uint32)
    v2 = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, order=perm)
    assert np.array_equal(vis, v2)
    A, Bp = perm[: n // 3], perm[n // 3:]
    va = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, order=A)
    vb = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, order=Bp)
    assert np.array_equal(np.minimum(va, vb), vis)
    dup = np.concatenate([perm, perm[: n // 2]])
    v3 = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, order=dup)
    assert np.array_equal(vis, v3)


def test_key_validity_and_layer_nesting(O, tiny):
    sc, soff, pos, _, fl, vis = tiny
    v0, v1 = vis[0, 0], vis[0, 1]
    for layer in (v0, v1):
        k = layer[layer != EMPTY].astype(np.uint64)
        ids = (k & np.uint64((1 << 40) - 1)).astype(np.int64)
        assert (ids < pos.shape[0] - 1).all()
        assert ((fl[ids] & 2) == 0).all()                  # a segment starts at a non-tip CP
        assert ((k >> np.uint64(40)) < (1 << 24)).all()
    # centre hits are (all but exact-border cases) conservative hits, with a key not larger
    both = v0 != EMPTY
    assert (v1[both] != EMPTY).mean() > 0.999
    assert (v1[both] <= v0[both]).mean() > 0.999


def test_scene_depth_prefill_occludes(O):
    W, H = 16, 16
    cam = _cam_unit(W, H, znear=0.5, zfar=2.0)
    pos, fl = _segment_stream((2.3, -8.1, 1.5), (13.7, -8.1, 1.5), 1.5)
    pos[:, :2] *= 1.5
    zwall = np.full((1, H, W), np.inf, np.float32)
    zwall[0, :, :8] = 1.0                               # opaque wall in front on the left half
    vis = _raster1(O, pos, fl, cam, W, H, scene_z=zwall)
    ids = (vis.astype(np.uint64) & np.uint64((1 << 40) - 1))
    opaque = (1 << 40) - 2
    assert (ids[0, 8, :8] == opaque).all()              # wall wins on the left
    assert (ids[0, 8, 9:13] == 0).all()                 # strand visible on the right
    assert (int(vis[0, 0, 0]) >> 40) == O.qdepth(1.0, 0.5, 2.0)


def test_cover_counts_equal_per_segment_rasters(O):
    # the raster's work count is the number of (segment, pixel) pairs each
    # predicate accepts: rasterizing every segment alone and counting its
    # non-empty pixels must give the same totals
    for seed in range(3):
        sc = scenes.micro_scene(seed)
        t, soff, (_, ncp) = O.lod_select(sc)
        pos, _, fl = O.generate(sc, t, ncp)
        for r_min in (0.0, 0.5):
            seg, uc, ua = O.cover_counts(pos, fl, soff, sc.cams, sc.width, sc.height, r_min)
            n, c0, c1 = 0, 0, 0
            for v in range(ncp - 1):
                if fl[v] & 2:                    # tip: no segment starts here
                    continue
                one = np.ascontiguousarray(pos[v:v + 2])
                vis = O.raster(one, np.array([1, 2], np.uint8), np.array([0, 2], np.uint32),
                               sc.cams, sc.width, sc.height, r_min)
                n += 1
                c0 += int((vis[0, 0] != EMPTY).sum())
                c1 += int((vis[0, 1] != EMPTY).sum())
            assert (seg, uc, ua) == (n, c0, c1)
            assert 0 < uc <= ua


def test_stored_work_counts_match_the_oracle(O):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "work_counts.json")) as f:
        stored = json.load(f)["head"]
    sc = scenes.config_head()
    t, soff, (ns, ncp) = O.lod_select(sc)
    pos, _, fl = O.generate(sc, t, ncp)
    seg, uc, ua = O.cover_counts(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min)
    assert (ns, ncp, seg, uc, ua) == (stored["strands"], stored["control_points"],
                                      stored["segments"], stored["centre_pairs"],
                                      stored["conservative_pairs"])
