"""Pins of the CPU oracle's deferred resolve: shading special cases, the
reconstruction filter's normalised convolution, alpha counting and depth
thresholds (Sec. 3.3, 3.4), and the soft-coverage resolve."""
import math

import numpy as np
import pytest
from scipy import ndimage

from paper_2607_04230_amd import scenes
from paper_2607_04230_amd.scenes import ResolveParams

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def _cam(width, height, eye=(0.0, 0.0, -5.0), f=50.0, cx=None, cy=None, znear=0.5, zfar=20.0):
    c = np.zeros(18, np.float32)
    c[0] = c[4] = c[8] = 1.0
    c[9:12] = eye
    c[12] = c[13] = f
    c[14] = width / 2.0 if cx is None else cx
    c[15] = height / 2.0 if cy is None else cy
    c[16], c[17] = znear, zfar
    return c


def _stream(points, width, rgbs=None):
    """One strand through `points` (list of xyz)."""
    n = len(points)
    pos = np.zeros((n, 4), np.float32)
    pos[:, :3] = points
    pos[:, 3] = width
    rgb = np.ones((n, 4), np.float32)
    if rgbs is not None:
        rgb[:, :3] = rgbs
    fl = np.zeros(n, np.uint8)
    fl[0] |= 1
    fl[-1] |= 2
    return pos, rgb, fl


def _render(O, pos, rgb, fl, cam, W, H, rp, mode, r_min=0.0):
    soff = np.array([0, pos.shape[0]], np.uint32)
    vis = O.raster(pos, fl, soff, cam[None], W, H, r_min)
    out = O.resolve(pos, rgb, fl, vis, cam[None], W, H, rp, mode)
    return vis, out[0]


def test_shading_perpendicular_cases(O):
    # strand along +x at z = 0 seen from (0, 0, -5): T = (1,0,0)
    W, H = 32, 16
    cam = _cam(W, H, cx=W / 2 + 0.5)
    pos, rgb, fl = _stream([(-1.0, 0.0, 0.0), (1.0, 0.0, 0.0)], 0.3,
                           rgbs=[(0.2, 0.4, 0.6), (0.6, 0.0, 1.0)])
    # light along +y: T.L = 0 (diffuse = kd) and T.H = 0 (specular = ks)
    rp = ResolveParams(light_dir=(0.0, 1.0, 0.0), ka=0.1, kd=0.7, ks=0.3)
    vis, out = _render(O, pos, rgb, fl, cam, W, H, rp, mode=2)
    px = out[H // 2, W // 2]                    # pixel centre over the segment midpoint
    alb = np.array([0.4, 0.2, 0.8])             # t3 = 0.5 for a fronto-parallel segment
    assert np.abs(px[:3] - (alb * (0.1 + 0.7) + 0.3)).max() < 1e-6
    assert px[3] == 1.0
    # light along +x: T.L = 1 (no diffuse); V = (0,0,-1) there, so T.H = 1/sqrt(2)
    rp = ResolveParams(light_dir=(1.0, 0.0, 0.0), ka=0.1, kd=0.7, ks=0.3)
    vis, out = _render(O, pos, rgb, fl, cam, W, H, rp, mode=2)
    px = out[H // 2, W // 2]
    assert np.abs(px[:3] - (alb * 0.1 + 0.3 * 0.5 ** 32)).max() < 1e-6


def _flat_groom(rng, n_strands=40, z=0.0, W=48, H=48, width=0.012):
    """Fronto-parallel random strands in the plane z = const (equal depth codes)."""
    pos, rgb, fl = [], [], []
    for s in range(n_strands):
        a = rng.uniform(-0.4, 0.4, 2)
        d = rng.normal(0, 1, 2)
        d /= np.linalg.norm(d)
        pts = [(a[0] + t * d[0] * 0.25, a[1] + t * d[1] * 0.25 + 0.05 * math.sin(3 * t), z)
               for t in np.linspace(0, 1, 5)]
        c = rng.uniform(0.1, 0.9, 3)
        p_, r_, f_ = _stream(pts, width, rgbs=np.tile(c, (5, 1)))
        pos.append(p_)
        rgb.append(r_)
        fl.append(f_)
    return np.concatenate(pos), np.concatenate(rgb), np.concatenate(fl)


def test_filter_constant_colour_is_preserved(O):
    rng = np.random.default_rng(3)
    W, H = 48, 48
    pos, rgb, fl = _flat_groom(rng)
    rgb[:, :3] = (0.3, 0.5, 0.7)
    cam = _cam(W, H, f=250.0)
    rp = ResolveParams(ka=1.0, kd=0.0, ks=0.0)
    vis, out = _render(O, pos, rgb, fl, cam, W, H, rp, mode=0)
    a = out[..., 3]
    m = a > 0
    assert m.sum() > 200
    c32 = np.array([0.3, 0.5, 0.7], np.float32).astype(np.float64)
    assert np.abs(out[m][:, :3] - a[m][:, None] * c32).max() < 1e-12


def test_filter_reduces_to_gaussian_blur(O):
    # sigma_c -> inf and s_par == s_perp: normalised Gaussian convolution over centre hits
    rng = np.random.default_rng(5)
    W, H = 48, 48
    pos, rgb, fl = _flat_groom(rng, n_strands=60)
    cam = _cam(W, H, f=250.0)
    rp = ResolveParams(ka=1.0, kd=0.0, ks=0.0, sigma_c=1e9, s_par=0.3, s_perp=0.3)
    soff = np.array([0, pos.shape[0]], np.uint32)
    vis = O.raster(pos, fl, soff, cam[None], W, H, 0.0)
    out, cc = O.resolve(pos, rgb, fl, vis, cam[None], W, H, rp, 0, want_center=True)
    out, cc = out[0], cc[0]
    hitc = vis[0, 0] != EMPTY
    q = (vis[0, 0][hitc].astype(np.uint64) >> np.uint64(40))
    assert q.max() - q.min() <= 1                     # one depth: no rejection
    r, sig = 5, 5 * 0.3
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1]
    K = np.exp(-(xx ** 2 + yy ** 2) / sig ** 2)
    num = np.stack([ndimage.correlate(cc[..., c] * hitc, K, mode="constant") for c in range(3)], -1)
    den = ndimage.correlate(hitc.astype(np.float64), K, mode="constant")
    exp = num / np.where(den > 0, den, 1)[..., None]
    a = out[..., 3]
    m = hitc & (a > 0)
    got = out[..., :3][m] / a[m][:, None]
    assert m.sum() > 300
    assert np.abs(got - exp[m]).max() < 1e-9


def _hand_vis(W, H, centre, cons, ids=None):
    """vis [1][2][H][W] from dicts {(j, i): q}, all naming segment 0 unless ids given."""
    vis = np.full((1, 2, H, W), EMPTY, np.uint64)
    for layer, d in ((0, centre), (1, cons)):
        for (j, i), qv in d.items():
            sid = 0 if ids is None else ids.get((layer, j, i), 0)
            vis[0, layer, j, i] = np.uint64((qv << 40) | sid)
    return vis


def test_alpha_strip_counts(O):
    # horizontal segment -> the strip through P is P's row (|dy| <= 0.5)
    W, H = 24, 12
    cam = _cam(W, H, f=50.0)
    pos, rgb, fl = _stream([(-0.8, 0.0, 0.0), (0.8, 0.0, 0.0)], 0.01)
    q = 1000
    centre = {(6, i): q for i in (8, 10, 11)}
    cons = {(6, i): q for i in range(6, 16)}
    cons[(5, 10)] = q                                   # off the strip: not counted
    vis = _hand_vis(W, H, centre, cons)
    rp = ResolveParams()
    out = O.resolve(pos, rgb, fl, vis, cam[None], W, H, rp, 0)[0]
    # P = (6, 10): window cols 5..15 of row 6 -> cons hits at 6..15 (10), centre 3
    assert out[6, 10, 3] == pytest.approx(3 / 10, abs=1e-15)
    # P = (6, 14) (promoted): window cols 9..19 -> cons 9..15 (7 px), centre 10, 11 (2)
    assert out[6, 14, 3] == pytest.approx(2 / 7, abs=1e-15)
    # a full centre-hit strip gives alpha 1
    centre = {(6, i): q for i in range(0, 24)}
    vis = _hand_vis(W, H, centre, dict(centre))
    out = O.resolve(pos, rgb, fl, vis, cam[None], W, H, rp, 0)[0]
    assert (out[6, :, 3] == 1.0).all()


def test_depth_thresholds_in_code_units(O):
    W, H = 24, 12
    cam = _cam(W, H, f=50.0)
    pos, rgb, fl = _stream([(-0.8, 0.0, 0.0), (0.8, 0.0, 0.0)], 0.01)
    rp = ResolveParams()
    dq_rej, dq_mis = O.depth_code_thresholds(rp)
    assert (dq_rej, dq_mis) == (24326, 8389)
    q = 100000
    # mismatch: conservative nearer by exactly the threshold -> output alpha 1
    for dq, mism in ((dq_mis, True), (dq_mis - 1, False)):
        centre = {(6, 10): q, (6, 11): q}
        cons = {(6, 10): q - dq, (6, 11): q, (6, 12): q}
        out = O.resolve(pos, rgb, fl, _hand_vis(W, H, centre, cons), cam[None], W, H, rp, 0)[0]
        assert (out[6, 10, 3] == 1.0) == mism
    # rejection: a centre neighbour exactly dq_rej away still contributes colour
    rp2 = ResolveParams(ka=1.0, kd=0.0, ks=0.0)
    pos2, rgb2, fl2 = _stream([(-0.8, 0.0, 0.0), (0.8, 0.0, 0.0), (0.8, 0.0, 0.0),
                               (-0.8, 0.0, 0.0)], 0.01)
    rgb2[:2, :3] = (1.0, 0.0, 0.0)
    rgb2[2:, :3] = (0.0, 0.0, 1.0)
    fl2[:] = (1, 2, 1, 2)
    for dq, used in ((dq_rej, True), (dq_rej + 1, False)):
        centre = {(6, 10): q, (6, 11): q + dq}
        ids = {(0, 6, 11): 2, (1, 6, 11): 2}
        vis = _hand_vis(W, H, centre, dict(centre), ids=ids)
        out = O.resolve(pos2, rgb2, fl2, vis, cam[None], W, H, rp2, 0)[0]
        assert (out[6, 10, 2] > 0) == used


# ------------------------------------------------------------------ soft coverage
def _soft(O, pos, rgb, fl, vis, cam, W, H, rp):
    import torch
    return O.soft_forward(torch.as_tensor(pos.astype(np.float64)),
                          torch.as_tensor(rgb.astype(np.float64)), fl, vis, cam[None], W, H,
                          rp).numpy()[0]


def test_soft_coverage_integrates_to_width(O):
    # Poisson summation: the row sum of a(d) over pixel centres, averaged over M = 8
    # sub-pixel offsets of a long vertical strand, equals its pixel width.
    W, H = 40, 9
    cam = np.zeros(18, np.float32)
    cam[0] = cam[4] = cam[8] = 1.0
    cam[12] = cam[13] = 1.0
    cam[16], cam[17] = 0.5, 2.0
    rp = ResolveParams()
    for w in (0.3, 0.8, 1.7):
        sums = []
        for m in range(8):
            x0 = 20.1 + m / 8
            pos, rgb, fl = _stream([(x0, 2.0, 1.0), (x0, -12.0, 1.0)], w)
            centre = {(4, i): 5 for i in range(W)}
            vis = _hand_vis(W, H, centre, dict(centre))
            out = _soft(O, pos, rgb, fl, vis, cam, W, H, rp)
            sums.append(out[4, :, 3].sum())
        assert abs(np.mean(sums) - w) < 1e-6
        assert np.std(sums) > 1e-6 or w > 1.5             # a single offset is not the integral


def test_soft_coverage_limits(O):
    W, H = 16, 8
    cam = np.zeros(18, np.float32)
    cam[0] = cam[4] = cam[8] = 1.0
    cam[12] = cam[13] = 1.0
    cam[16], cam[17] = 0.5, 2.0
    rp = ResolveParams()
    pos, rgb, fl = _stream([(8.5, 2.0, 1.0), (8.5, -12.0, 1.0)], 1e-7)
    vis = _hand_vis(W, H, {(4, 8): 5}, {(4, 8): 5})
    out = _soft(O, pos, rgb, fl, vis, cam, W, H, rp)
    assert 0 < out[4, 8, 3] < 1e-6
    # a very wide strand centred on the pixel covers it fully
    pos, rgb, fl = _stream([(8.5, 2.0, 1.0), (8.5, -12.0, 1.0)], 20.0)
    out = _soft(O, pos, rgb, fl, vis, cam, W, H, rp)
    assert out[4, 8, 3] == pytest.approx(1.0, abs=1e-12)


def test_soft_shading_matches_deferred_shading(O):
    # two independent implementations of the shading (C binary64 and torch binary64)
    sc = scenes.config_tiny(width=96, height=96)
    t, soff, (_, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, t, ncp)
    vis = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height)
    rp = ResolveParams()
    _, cc = O.resolve(pos, rgb, fl, vis, sc.cams, sc.width, sc.height, rp, 2, want_center=True)
    import torch
    out = O.soft_forward(torch.as_tensor(pos.astype(np.float64)),
                         torch.as_tensor(rgb.astype(np.float64)), fl, vis, sc.cams, sc.width,
                         sc.height, rp).numpy()
    hitc = vis[:, 0] != EMPTY
    a = out[..., 3][hitc]
    ok = a > 1e-3
    S = out[..., :3][hitc][ok] / a[ok][:, None]
    assert np.abs(S - cc[hitc][ok]).max() < 1e-9


def test_soft_gradient_matches_central_differences(O):
    import torch
    sc = scenes.micro_scene(2, res=24, width=0.04)
    t, soff, (_, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, t, ncp)
    vis = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, 1.0)
    rp = ResolveParams()
    rng = np.random.default_rng(0)
    target = rng.uniform(0, 0.3, (1, sc.height, sc.width, 4))
    p64 = pos.astype(np.float64)
    c64 = rgb.astype(np.float64)

    def loss(p, c):
        o = O.soft_forward(torch.as_tensor(p), torch.as_tensor(c), fl, vis, sc.cams, sc.width,
                           sc.height, rp).numpy()
        return ((o - target) ** 2).sum()

    o = O.soft_forward(torch.as_tensor(p64), torch.as_tensor(c64), fl, vis, sc.cams, sc.width,
                       sc.height, rp).numpy()
    gp, gc = O.soft_grad(p64, c64, fl, vis, sc.cams, sc.width, sc.height, rp, 2 * (o - target))
    used = np.unique((vis[0].astype(np.uint64) & np.uint64((1 << 40) - 1)).astype(np.int64))
    used = used[used < ncp]
    checks = 0
    for v in rng.choice(used, 12, replace=False):
        for c, h in ((0, 1e-6), (1, 1e-6), (2, 1e-6), (3, 1e-7)):
            pp, pm = p64.copy(), p64.copy()
            pp[v, c] += h
            pm[v, c] -= h
            fd = (loss(pp, c64) - loss(pm, c64)) / (2 * h)
            assert abs(fd - gp[v, c]) <= 1e-6 * max(1.0, abs(gp[v, c])) + 1e-7
            checks += 1
        for c in range(3):
            cp, cm = c64.copy(), c64.copy()
            cp[v, c] += 1e-6
            cm[v, c] -= 1e-6
            fd = (loss(p64, cp) - loss(p64, cm)) / 2e-6
            assert abs(fd - gc[v, c]) <= 1e-6 * max(1.0, abs(gc[v, c])) + 1e-7
    assert checks == 48
    assert np.abs(gp).max() > 0 and np.abs(gc).max() > 0
