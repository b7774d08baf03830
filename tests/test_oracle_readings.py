"""Pins of the oracle terms that the symmetric special cases cannot see.

* Eq. (bilateral), Sec. 3.3.1: the spatial weight is anisotropic,
  exp(-d_par^2 / sigma_par^2 - d_perp^2 / sigma_perp^2) with d_par measured
  along the screen tangent of the source strand; the colour term is
  exp(-|C_P - C_Q|^2 / sigma_c^2).  The expected means below are written out
  from those closed forms with the numbers of the hand-built buffers: a swap of
  sigma_par and sigma_perp, d_par taken along the normal, or sigma_c in place
  of sigma_c^2 each move them by far more than the tolerance.
* Code 1 (Appendix B), calcTangent: the interior layer tangent is the central
  difference next - prev; the Hermite control points of three non-collinear
  layers are worked by hand.
* The same tangent rule on the styled polyline (root: next - current, tip:
  current - previous, interior: next - previous), which the centre shading and
  the compressed G-buffer tangent use.
* A strand has at least one segment: fewer than two control points per strand
  are taken as two.
"""
import math

import numpy as np

from paper_2607_04230_amd import scenes
from paper_2607_04230_amd.scenes import ResolveParams

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def _cam(width, height, f=50.0):
    """R = identity, eye (0, 0, -5): world (x, y, 0) -> pixel (W/2 + 10x, H/2 - 10y)."""
    c = np.zeros(18, np.float32)
    c[0] = c[4] = c[8] = 1.0
    c[9:12] = (0.0, 0.0, -5.0)
    c[12] = c[13] = f
    c[14], c[15] = width / 2.0, height / 2.0
    c[16], c[17] = 0.5, 20.0
    return c


def _strands(segs, colours, width=0.01):
    """Two-point strands (root, tip) with constant colour each."""
    n = 2 * len(segs)
    pos = np.zeros((n, 4), np.float32)
    rgb = np.ones((n, 4), np.float32)
    fl = np.zeros(n, np.uint8)
    for k, ((a, b), c) in enumerate(zip(segs, colours)):
        pos[2 * k, :3], pos[2 * k + 1, :3] = a, b
        rgb[2 * k, :3] = rgb[2 * k + 1, :3] = c
        fl[2 * k], fl[2 * k + 1] = 1, 2
    pos[:, 3] = width
    return pos, rgb, fl


def _vis(W, H, hits, q=5000):
    """Both layers hold key q << 40 | id at the given {(j, i): id} pixels."""
    vis = np.full((1, 2, H, W), EMPTY, np.uint64)
    for (j, i), sid in hits.items():
        vis[0, 0, j, i] = vis[0, 1, j, i] = np.uint64((q << 40) | sid)
    return vis


# P = pixel (12, 12) shows segment 0, horizontal on screen (tangent (1, 0)).
# Its neighbours two pixels away along the tangent show segments 2 and 4, two
# pixels away across it segments 6 and 8; every segment has its own colour.
_COL = np.array([(0.5, 0.5, 0.5), (0.9, 0.1, 0.2), (0.1, 0.8, 0.3), (0.2, 0.3, 0.9),
                 (0.7, 0.6, 0.1)], np.float32)
_HITS = {(12, 12): 0, (12, 14): 2, (12, 10): 4, (14, 12): 6, (10, 12): 8}


def _anisotropic_case(O, sigma_c):
    W = H = 24
    seg = ((-0.8, 0.0, 0.0), (0.8, 0.0, 0.0))        # pixels (4, 12) -> (20, 12)
    pos, rgb, fl = _strands([seg] * 5, _COL)
    # shading = albedo (ambient only), so the centre colour of a pixel is its
    # segment's colour
    rp = ResolveParams(ka=1.0, kd=0.0, ks=0.0, s_par=0.4, s_perp=0.1, sigma_c=sigma_c)
    out = O.resolve(pos, rgb, fl, _vis(W, H, _HITS), _cam(W, H)[None], W, H, rp, 0)[0]
    return out[12, 12], _COL.astype(np.float64)


def test_filter_weight_is_anisotropic_along_the_screen_tangent(O):
    px, C = _anisotropic_case(O, sigma_c=1e9)
    # sigma_par = r s_par = 2 px, sigma_perp = r s_perp = 0.5 px: a neighbour two
    # pixels along the tangent weighs exp(-4/4) = e^-1, across it exp(-4/0.25) = e^-16
    w_along, w_across = math.exp(-1.0), math.exp(-16.0)
    num = C[0] + w_along * (C[1] + C[2]) + w_across * (C[3] + C[4])
    den = 1.0 + 2.0 * w_along + 2.0 * w_across
    assert px[3] == 1.0                               # the strip (row 12) is all centre hits
    assert np.abs(px[:3] - num / den).max() < 1e-8
    # the swapped weights would give a clearly different mean
    swapped = (C[0] + w_across * (C[1] + C[2]) + w_along * (C[3] + C[4])) / den
    assert np.abs(px[:3] - swapped).max() > 0.05


def test_filter_colour_term_uses_sigma_c_squared(O):
    px, C = _anisotropic_case(O, sigma_c=0.9)
    sc2 = 0.9 * 0.9
    ws = [1.0, math.exp(-1.0), math.exp(-1.0), math.exp(-16.0), math.exp(-16.0)]
    wc = [math.exp(-float(((C[k] - C[0]) ** 2).sum()) / sc2) for k in range(5)]
    w = np.array(ws) * np.array(wc)
    exp = (w[:, None] * C).sum(0) / w.sum()
    assert np.abs(px[:3] - exp).max() < 1e-8
    # sigma_c where sigma_c^2 belongs
    wc_bad = [math.exp(-float(((C[k] - C[0]) ** 2).sum()) / 0.9) for k in range(5)]
    wb = np.array(ws) * np.array(wc_bad)
    assert np.abs(px[:3] - (wb[:, None] * C).sum(0) / wb.sum()).max() > 1e-3


def test_promoted_pixel_has_no_colour_term(O):
    # the same neighbourhood around a conservative-only pixel: the colour term
    # is off (w_c = 1), so only the spatial weights remain
    W = H = 24
    seg = ((-0.8, 0.0, 0.0), (0.8, 0.0, 0.0))
    pos, rgb, fl = _strands([seg] * 5, _COL)
    rp = ResolveParams(ka=1.0, kd=0.0, ks=0.0, s_par=0.4, s_perp=0.1, sigma_c=0.9)
    vis = _vis(W, H, _HITS)
    vis[0, 0, 12, 12] = EMPTY                         # P keeps only its conservative hit
    out = O.resolve(pos, rgb, fl, vis, _cam(W, H)[None], W, H, rp, 0)[0]
    C = _COL.astype(np.float64)
    w_along, w_across = math.exp(-1.0), math.exp(-16.0)
    exp = (w_along * (C[1] + C[2]) + w_across * (C[3] + C[4])) / (2 * w_along + 2 * w_across)
    assert np.abs(out[12, 12, :3] / out[12, 12, 3] - exp).max() < 1e-8
    assert out[12, 12, 3] == 2.0 / 3.0                # strip: 2 centre of 3 hits


def _one_bundle(points, n_cp):
    """One bundle whose four quad corners coincide on every layer, so that
    each layer's bilinear point is the given point whatever (u, v)."""
    L = len(points)
    lp = np.zeros((L, 4, 3), np.float32)
    for l, p in enumerate(points):
        lp[l, :] = p
    B = 1
    return scenes.Scene("bent", lp, np.arange(4, dtype=np.uint32).reshape(1, 4),
                        np.zeros(B, np.uint32), np.ones(B, np.uint32),
                        np.full(B, n_cp, np.uint32), np.zeros(B, np.uint32),
                        np.zeros(B, np.uint32), None, _cam(32, 32)[None], 32, 32, None,
                        seed=7, strand_width=0.01, curl_amp=0.0, curl_turns=3.0)


def test_interior_layer_tangent_is_central_difference(O):
    P0, P1, P2 = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([1.0, 1, 0])
    sc = _one_bundle([P0, P1, P2], 5)
    table, _, (_, ncp) = O.lod_select(sc)
    pos, _, _ = O.generate(sc, table, ncp)
    assert ncp == 5
    T0 = np.array([1.0, 0, 0])                        # root: next - current
    T1 = np.array([1.0, 1.0, 0]) / math.sqrt(2.0)     # interior: next - previous
    T2 = np.array([0.0, 1.0, 0])                      # tip: current - previous
    # w = 1/4 and 3/4 fall in the middle (t = 1/2) of intervals 0 and 1, whose
    # chords are 1: h00 = h01 = 1/2, h10 = 1/8, h11 = -1/8
    cp1 = 0.5 * P0 + 0.125 * T0 + 0.5 * P1 - 0.125 * T1
    cp3 = 0.5 * P1 + 0.125 * T1 + 0.5 * P2 - 0.125 * T2
    np.testing.assert_allclose(pos[1, :3], cp1, atol=1e-6)
    np.testing.assert_allclose(pos[3, :3], cp3, atol=1e-6)
    np.testing.assert_array_equal(pos[[0, 2, 4], :3], np.array([P0, P1, P2], np.float32))
    # one-sided interior tangents would move CP 1 by at least 0.08
    for T1_bad in (np.array([1.0, 0, 0]), np.array([0.0, 1.0, 0])):
        bad = 0.5 * P0 + 0.125 * T0 + 0.5 * P1 - 0.125 * T1_bad
        assert np.abs(bad - cp1).max() > 0.08


def _bent_strand():
    P = np.array([(-0.5, 0.0, 0.0), (0.0, 0.0, 0.0), (0.3, 0.5, 0.0)], np.float32)
    pos = np.zeros((3, 4), np.float32)
    pos[:, :3] = P
    pos[:, 3] = 0.01
    rgb = np.ones((3, 4), np.float32)
    fl = np.array([1, 0, 2], np.uint8)
    return pos, rgb, fl


def test_styled_polyline_tangents_in_centre_shading(O):
    # diffuse only, light along +x, albedo 1: shading = sqrt(1 - T_x^2) for a
    # tangent in the image plane
    W, H = 24, 12
    pos, rgb, fl = _bent_strand()
    rp = ResolveParams(light_dir=(1.0, 0.0, 0.0), ka=0.0, kd=1.0, ks=0.0)
    # segment 0 spans pixels x 7 -> 12 on row y = 6 (centres at 5.5 above: the
    # keys are placed by hand, the shading takes the closest point)
    hits = {(5, 12): 0, (5, 9): 0, (5, 14): 1}
    out = O.resolve(pos, rgb, fl, _vis(W, H, hits), _cam(W, H)[None], W, H, rp, 2)[0]
    P = pos[:, :2].astype(np.float64)                       # the binary32 inputs, exactly

    def unit(d):
        return d / np.linalg.norm(d)

    Troot = unit(P[1] - P[0])
    Tmid = unit(P[2] - P[0])                                 # central difference at P1
    Ttip = unit(P[2] - P[1])
    # pixel (12, 5): centre x = 12.5 lies past the end (x = 12), t3 = 1: T = T(P1)
    assert abs(out[5, 12, 0] - math.sqrt(1 - Tmid[0] ** 2)) < 1e-9
    # pixel (9, 5): x = 9.5 is half way (fronto-parallel, so t3 = ts = 1/2)
    Th = unit(0.5 * Troot + 0.5 * Tmid)
    assert abs(out[5, 9, 0] - math.sqrt(1 - Th[0] ** 2)) < 1e-9
    # pixel (14, 5) on segment 1 (screen (12, 6) -> (15, 1)); t3 = ts (fronto-parallel)
    a = np.array([12.0 + 10.0 * P[1, 0], 6.0 - 10.0 * P[1, 1]])
    b = np.array([12.0 + 10.0 * P[2, 0], 6.0 - 10.0 * P[2, 1]])
    d = b - a
    ts = float(np.clip(((np.array([14.5, 5.5]) - a) @ d) / (d @ d), 0, 1))
    T = unit((1 - ts) * Tmid + ts * Ttip)
    assert abs(out[5, 14, 0] - math.sqrt(1 - T[0] ** 2)) < 1e-9
    # one-sided interior tangents give other values at pixel (12, 5)
    for bad in (Troot, Ttip):
        assert abs(out[5, 12, 0] - math.sqrt(1 - bad[0] ** 2)) > 0.1


def test_styled_polyline_tangent_in_gbuffer_code(O):
    # the G-buffer key of a pixel past the end of segment 0 carries the
    # octahedral code of the interior tangent at P1 (central difference)
    W, H = 24, 12
    pos, rgb, fl = _bent_strand()
    soff = np.array([0, 3], np.uint32)
    vis = O.raster_gbuf(pos, rgb, fl, soff, _cam(W, H)[None], W, H, 1.0)
    k = int(vis[0, 1, 6, 12])                # conservative layer at the joint
    assert k != int(EMPTY)
    code = (k >> 24) & 0xFFFF
    P = pos[:, :3].astype(np.float64)

    def unit(d):
        return d / np.linalg.norm(d)

    Tmid, Troot, Ttip = unit(P[2] - P[0]), unit(P[1] - P[0]), unit(P[2] - P[1])

    # octahedral codes (upper hemisphere, z = 0): u = x / (|x| + |y|), rounded;
    # the three tangents land at least 0.04 of a code step from a rounding edge
    def oct_code(t):
        l1 = abs(float(t[0])) + abs(float(t[1]))
        u, v = float(t[0]) / l1, float(t[1]) / l1
        return (int((u * 0.5 + 0.5) * 255 + 0.5) << 8) | int((v * 0.5 + 0.5) * 255 + 0.5)
    # segment 0 at pixel (12, 6) has ts = 1 (the closest point is the joint), so
    # t3 = 1 up to one rounding and the tangent is T(P1); segment 1 has ts = 0
    # there, tangent T(P1) too.  Either key carries T(P1)'s code.
    assert code == oct_code(Tmid)
    assert code not in (oct_code(Troot), oct_code(Ttip))


def test_fewer_than_two_control_points_are_taken_as_two(O):
    sc = scenes.micro_scene(4, n_bundles=3, strands=2, n_cp=5)
    sc.bundle_cmax = np.array([1, 0, 5], np.uint32)
    for mode in (0, 1):
        table, _, (ns, ncp) = O.lod_select(sc, mode=mode)
        assert table[0, 1] == 2 and table[1, 1] == 2
        assert table[2, 1] in (3, 5)
        pos, _, fl = O.generate(sc, table, ncp)
        assert np.isfinite(pos).all()
        assert (fl[table[0, 3]:table[0, 3] + 2] == (1, 2)).all()


def test_gbuffer_colour_is_perspective_correct_through_the_far_endpoint(O):
    # Sec. 3.1.2 stores shading data at the covered point; the interpolation
    # parameter along the segment is the perspective-correct
    # t3 = ts * (1/z_1) / (1/z(ts)) with 1/z_1 of the segment's second endpoint.
    # A receding segment (z 5 -> 7) from black to red: the red code at pixel
    # (11, 6) follows t3, not the screen parameter ts or a t3 built from 1/z_0.
    W, H = 24, 12
    pos = np.array([(-0.5, 0.0, 0.0, 0.01), (0.5, 0.0, 2.0, 0.01)], np.float32)
    rgb = np.array([(0.0, 0.0, 0.0, 1.0), (1.0, 0.0, 0.0, 1.0)], np.float32)
    fl = np.array([1, 2], np.uint8)
    cam = _cam(W, H)
    vis = O.raster_gbuf(pos, rgb, fl, np.array([0, 2], np.uint32), cam[None], W, H, 1.0)
    k = int(vis[0, 0, 6, 11])
    assert k != int(EMPTY)
    red = (k >> 18) & 63
    x0, x1 = 12.0 + 50.0 * -0.5 / 5.0, 12.0 + 50.0 * 0.5 / 7.0      # screen x of the ends
    ts = (11.5 - x0) / (x1 - x0)                                     # y is constant
    iz = (1 / 5.0) + ts * (1 / 7.0 - 1 / 5.0)
    t3 = ts * (1 / 7.0) / iz
    assert abs(red - (t3 * 63 + 0.5)) <= 1.0
    for wrong in (ts, ts * (1 / 5.0) / iz):
        assert abs(red - (wrong * 63 + 0.5)) > 4.0
