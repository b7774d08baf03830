"""Pins of the oracle's compressed G-buffer (Sec. 3.1.2, deferred atomic
shading: 24-bit depth + 40 bits of quantised shading inputs): the octahedral
tangent code against its inverse map and the closed-form codes of the axis
directions, the 6-bit colour codes, the invariant that the payload changes
no depth and no coverage, and the decoded shading against the shading of the
segment itself within the quantisation error."""
import math

import numpy as np
import pytest

from paper_2607_04230_amd import scenes
from paper_2607_04230_amd.scenes import ResolveParams

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
MASK40 = np.uint64((1 << 40) - 1)


def _oct_decode(code):
    """Inverse octahedral map (written from its definition: unfold the lower
    half across the diagonals, then normalise)."""
    u = ((code >> 8) & 255) / 255.0 * 2.0 - 1.0
    v = (code & 255) / 255.0 * 2.0 - 1.0
    z = 1.0 - abs(u) - abs(v)
    if z < 0.0:
        u, v = (1.0 - abs(v)) * math.copysign(1.0, u), (1.0 - abs(u)) * math.copysign(1.0, v)
    t = np.array([u, v, z])
    return t / np.linalg.norm(t)


def test_octahedral_axis_codes(O):
    # x, y map to the octahedron's corners, +z to the centre, -z (folded) to
    # the corner (1, 1); code = round((c + 1) / 2 * 255) per axis
    assert O.oct16([1, 0, 0]) == (255 << 8) | 128
    assert O.oct16([-1, 0, 0]) == (0 << 8) | 128
    assert O.oct16([0, 1, 0]) == (128 << 8) | 255
    assert O.oct16([0, -1, 0]) == (128 << 8) | 0
    assert O.oct16([0, 0, 1]) == (128 << 8) | 128
    assert O.oct16([0, 0, -1]) == (255 << 8) | 255
    assert O.oct16([0, 0, 0]) == (128 << 8) | 128
    # a direction and its scaled copy share the code (projection by the L1 norm)
    assert O.oct16([0.3, -0.5, 0.2]) == O.oct16([0.6, -1.0, 0.4])


def test_octahedral_round_trip_error(O):
    """Every unit vector comes back within 1 degree (8 bits per axis: a code
    step of 2/255 on the octahedron), on the right hemisphere."""
    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(4000):
        t = rng.normal(size=3)
        t = (t / np.linalg.norm(t)).astype(np.float32)
        d = _oct_decode(O.oct16(t))
        tt = t.astype(np.float64) / np.linalg.norm(t)
        worst = max(worst, math.degrees(math.acos(min(1.0, float(d @ tt)))))
        if abs(tt[2]) > 0.02:
            assert np.sign(d[2]) == np.sign(tt[2])
    assert 0.3 < worst <= 1.0


def _tiny(O, **kw):
    sc = scenes.config_tiny(**kw)
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, rgb, fl = O.generate(sc, table, ncp)
    return sc, soff, pos, rgb, fl


@pytest.mark.parametrize("r_min", [0.0, 0.5, 1.5])
def test_payload_changes_no_depth_and_no_coverage(O, r_min):
    sc, soff, pos, rgb, fl = _tiny(O)
    v1 = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, r_min, sc.scene_z)
    v2 = O.raster_gbuf(pos, rgb, fl, soff, sc.cams, sc.width, sc.height, r_min, sc.scene_z)
    assert np.array_equal(v1 >> np.uint64(40), v2 >> np.uint64(40))
    assert np.array_equal(v1 == EMPTY, v2 == EMPTY)
    opaque = np.uint64((1 << 40) - 2)
    assert np.array_equal((v1 & MASK40) == opaque, (v2 & MASK40) == opaque)
    hit = (v2 != EMPTY) & ((v2 & MASK40) != opaque)
    assert hit.sum() > 1000
    assert ((v2[hit] & np.uint64(63)) == np.uint64(63)).all()      # AO code: no baked AO


def test_colour_codes_of_a_constant_albedo(O):
    sc, soff, pos, rgb, fl = _tiny(O)
    c = np.array([0.2, 0.5, 0.9], np.float32)
    rgb = rgb.copy()
    rgb[:, :3] = c
    v = O.raster_gbuf(pos, rgb, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    hit = (v != EMPTY) & ((v & MASK40) != np.uint64((1 << 40) - 2))
    w = v[hit] & MASK40
    expect = [int(x * 63.0 + 0.5) for x in c]                       # 13, 32, 57
    assert expect == [13, 32, 57]
    assert ((w >> np.uint64(18)) & np.uint64(63) == expect[0]).all()
    assert ((w >> np.uint64(12)) & np.uint64(63) == expect[1]).all()
    assert ((w >> np.uint64(6)) & np.uint64(63) == expect[2]).all()


def test_decoded_shading_is_close_to_the_segment_shading(O):
    """The centre resolve from the compressed buffer against the centre
    resolve that gathers the segment: the same pixels are hair and
    background; colours differ by the quantisation (tangent within 1 degree,
    albedo within 1/126, position from the depth code at the pixel centre)."""
    sc, soff, pos, rgb, fl = _tiny(O)
    rp = ResolveParams()
    v1 = O.raster(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    v2 = O.raster_gbuf(pos, rgb, fl, soff, sc.cams, sc.width, sc.height, sc.r_min, sc.scene_z)
    a = O.resolve(pos, rgb, fl, v1, sc.cams, sc.width, sc.height, rp, 2, sc.bg)
    b = O.resolve_gbuf(v2, sc.cams, sc.width, sc.height, rp, sc.bg)
    assert np.array_equal(a[..., 3], b[..., 3])
    bgpx = a[..., 3] == 0
    assert np.array_equal(a[bgpx], b[bgpx])
    d = np.abs(a - b)[~bgpx]
    assert d.max() <= 0.03 and d.mean() <= 0.003
    assert d.max() > 0.0                                            # it is lossy
