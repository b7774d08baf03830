"""Seeded synthetic inputs: hair meshes, cameras, occluder depth and the five workloads.

This module only *builds inputs*.  It holds none of the method's arithmetic (no
hashing, interpolation, projection to pixels, coverage or shading) and imports
neither the HIP library nor the CPU oracle, so that both sides can consume the
same arrays.

Hair-mesh structure (bundles of L stacked quad layers, roots on the first
layer, tips on the last) follows the paper's background on hair meshes
(Sec. 2, "Background: Hair mesh rendering").  The concrete grooms are synthetic
stand-ins for the paper's two ~127k-strand grooms (Sec. 4), which are not
available: a unit-sphere head whose scalp is tiled by cube-sphere quads, with
layers extruded along the scalp normal.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Camera record layout shared by every consumer (18 float32):
#   R[9] (world->camera rotation, rows = right, up, forward), eye[3],
#   fx, fy, cx, cy, znear, zfar
CAM_FLOATS = 18

MODE_FILTER = 0
MODE_SOFT = 1
MODE_CENTER = 2   # plain 1-spp center shading, no reconstruction filter

LOD_OFF = 0
LOD_ON = 1


@dataclasses.dataclass
class ResolveParams:
    """Resolve constants as the paper states them (Sec. 3.3, 3.4); defaults
    are the paper's values where it gives one."""
    light_dir: tuple = (0.3, 0.8, 0.5)     # towards the light
    light_rgb: tuple = (1.0, 1.0, 1.0)
    ka: float = 0.1
    kd: float = 0.7
    ks: float = 0.3
    spec_squarings: int = 5                # specular (1 - (T.H)^2)^(2^5)
    filter_radius: int = 5                 # r = 5
    s_par: float = 0.4                     # sigma_par = r * s_par
    s_perp: float = 0.1                    # sigma_perp = r * s_perp
    sigma_c: float = 0.9
    iso_scale: float = 0.4                 # sigma_iso = 0.4 r
    depth_reject: float = 1.45e-3          # neighbour rejection (normalised depth)
    depth_mismatch: float = 5e-4           # centre/conservative mismatch
    strip_half: float = 0.5                # alpha strip half width (px)
    iso_len: float = 1e-6                  # screen tangent length below which the filter is isotropic
    soft_sigma: float = 0.28867513459481287  # 1/sqrt(12) px, soft-coverage pixel filter


@dataclasses.dataclass
class ShadowParams:
    """Deep-opacity-map shadows (Sec. 3.4; the paper cites Yuksel & Keyser
    2008 for the map and gives no constants, so these are choices): a pinhole
    light camera looking at the groom from the light direction, 4 layers of
    fixed thickness behind the nearest fragment, and a constant opacity per
    fragment."""
    width: int = 512
    height: int = 512
    distance: float = 4.0            # light camera eye = groom centre + distance * L
    vfov_deg: float = 45.0
    znear: float = 0.1
    zfar: float = 10.0
    n_layers: int = 4
    layer_world: float = 0.05        # layer thickness (world units along the light view)
    alpha: float = 0.05              # opacity of one fragment
    r_min: float = 0.5               # fragment coverage half width in the light view (px)

    def layer_codes(self) -> int:
        """Layer thickness in 24-bit depth-code units."""
        return max(1, int(self.layer_world / (self.zfar - self.znear) * 16777216.0))


def light_camera(sc: "Scene", sp: ShadowParams, rp: "ResolveParams" = None) -> np.ndarray:
    """Light camera record [1][18] for scene `sc`: a pinhole at the groom's
    bounding-box centre + distance * L looking back at that centre."""
    rp = rp or ResolveParams()
    L = np.asarray(rp.light_dir, np.float64)
    L /= np.linalg.norm(L)
    pts = np.asarray(sc.layer_pos, np.float64).reshape(-1, 3)
    centre = 0.5 * (pts.min(0) + pts.max(0))
    up = (0.0, 0.0, 1.0) if abs(L[1]) > 0.99 else (0.0, 1.0, 0.0)
    return look_at_camera(centre + sp.distance * L, centre, sp.width, sp.height,
                          vfov_deg=sp.vfov_deg, znear=sp.znear, zfar=sp.zfar, up=up)[None]


@dataclasses.dataclass
class Scene:
    """Everything one render call needs, as host numpy arrays."""
    name: str
    layer_pos: np.ndarray            # f32 [L][NV][3]
    quads: np.ndarray                # u32 [B][4]  (A, B, C, D counter-clockwise)
    bundle_key: np.ndarray           # u32 [B]     hash key of each bundle
    bundle_nstrands: np.ndarray      # u32 [B]     full strand count N_b
    bundle_cmax: np.ndarray          # u32 [B]     control points per strand (cap)
    bundle_scene: np.ndarray         # u32 [B]     scene (camera / image) of the bundle
    strand_base: np.ndarray          # u32 [B]     first full-strand record of the bundle
    strand_rgb: Optional[np.ndarray] # f32 [n_full][3] or None (use base_rgb)
    cams: np.ndarray                 # f32 [S][18]
    width: int
    height: int
    scene_z: Optional[np.ndarray]    # f32 [S][H][W] linear view depth of the opaque scene, inf = none
    seed: int = 1000
    strand_width: float = 0.002
    curl_amp: float = 0.02
    curl_turns: float = 3.0
    base_rgb: tuple = (0.30, 0.18, 0.10)
    lod_mode: int = LOD_OFF
    lod_lambda: float = 3.0
    r_min: float = 0.0
    mode: int = MODE_FILTER
    bg: tuple = (0.0, 0.0, 0.0)
    meta: dict = dataclasses.field(default_factory=dict)   # builder facts (e.g. head centres)

    @property
    def n_scenes(self) -> int:
        return int(self.cams.shape[0])

    @property
    def n_bundles(self) -> int:
        return int(self.quads.shape[0])

    @property
    def n_layers(self) -> int:
        return int(self.layer_pos.shape[0])

    @property
    def n_full_strands(self) -> int:
        return int(self.bundle_nstrands.astype(np.int64).sum())

    @property
    def n_cp_full(self) -> int:
        """Control points before any level of detail (upper bound for buffers);
        a count below 2 is taken as 2, as the library and the oracle do."""
        return int((self.bundle_nstrands.astype(np.int64) * self._cmax()).sum())

    @property
    def n_seg_full(self) -> int:
        return int((self.bundle_nstrands.astype(np.int64) * (self._cmax() - 1)).sum())

    def _cmax(self) -> np.ndarray:
        return np.maximum(self.bundle_cmax.astype(np.int64), 2)


# ----------------------------------------------------------------------------- cameras
def look_at_camera(eye, target, width, height, vfov_deg=40.0, znear=0.1, zfar=10.0,
                   up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """Pinhole camera record (float64 construction, stored as float32)."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    f = target - eye
    f /= np.linalg.norm(f)
    upw = np.asarray(up, np.float64)
    if abs(float(np.dot(f, upw))) > 0.999:
        upw = np.array([0.0, 0.0, 1.0])
    r = np.cross(f, upw)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    fy = (height / 2.0) / math.tan(math.radians(vfov_deg) / 2.0)
    rec = np.zeros(CAM_FLOATS, np.float64)
    rec[0:3], rec[3:6], rec[6:9] = r, u, f
    rec[9:12] = eye
    rec[12], rec[13] = fy, fy
    rec[14], rec[15] = width / 2.0, height / 2.0
    rec[16], rec[17] = znear, zfar
    return rec.astype(np.float32)


def sphere_depth(cams: np.ndarray, width: int, height: int, centers, radius=1.0) -> np.ndarray:
    """Linear view depth (camera-space z) of the nearest unit-sphere head per pixel centre.

    Analytic ray-sphere intersection in float64; pixels that miss every sphere get +inf.
    """
    centers = np.asarray(centers, np.float64).reshape(-1, 3)
    out = np.empty((cams.shape[0], height, width), np.float32)
    jj, ii = np.meshgrid(np.arange(height, dtype=np.float64) + 0.5,
                         np.arange(width, dtype=np.float64) + 0.5, indexing="ij")
    for s, c in enumerate(cams.astype(np.float64)):
        R = c[0:9].reshape(3, 3)
        eye = c[9:12]
        fx, fy, cx, cy = c[12], c[13], c[14], c[15]
        # camera-space ray with z = 1
        dc = np.stack([(ii - cx) / fx, -(jj - cy) / fy, np.ones_like(ii)], -1)
        dw = dc @ R            # world direction (R is orthonormal: R^T dc)
        zbest = np.full((height, width), np.inf)
        for cen in centers:
            oc = eye - cen
            a = np.einsum("hwk,hwk->hw", dw, dw)
            b = 2.0 * (dw @ oc)
            cc = float(oc @ oc) - radius * radius
            disc = b * b - 4 * a * cc
            hit = disc >= 0
            tq = np.where(hit, (-b - np.sqrt(np.where(hit, disc, 0))) / (2 * a), np.inf)
            tq = np.where(tq > 0, tq, np.inf)   # param along dc; dc has z = 1 so t == view z
            zbest = np.minimum(zbest, tq)
        out[s] = zbest.astype(np.float32)
    return out


# ----------------------------------------------------------------------------- grooms
def _face_grid(face: str, n: int, a_range=(-1.0, 1.0), b_range=(-1.0, 1.0)):
    """Cube-face grid points (n+1)^2 projected onto the unit sphere; returns (pts, quads)."""
    a = np.linspace(a_range[0], a_range[1], n + 1)
    b = np.linspace(b_range[0], b_range[1], n + 1)
    A, Bm = np.meshgrid(a, b, indexing="ij")
    if face == "top":      # +y, a along x, b along -z (counter-clockwise seen from +y)
        p = np.stack([A, np.ones_like(A), -Bm], -1)
    elif face == "front":  # +z, a along x, b along y
        p = np.stack([A, Bm, np.ones_like(A)], -1)
    elif face == "back":   # -z
        p = np.stack([-A, Bm, -np.ones_like(A)], -1)
    elif face == "right":  # +x
        p = np.stack([np.ones_like(A), Bm, -A], -1)
    elif face == "left":   # -x
        p = np.stack([-np.ones_like(A), Bm, A], -1)
    else:
        raise ValueError(face)
    p = p / np.linalg.norm(p, axis=-1, keepdims=True)
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    q = np.stack([idx[:-1, :-1], idx[1:, :-1], idx[1:, 1:], idx[:-1, 1:]], -1).reshape(-1, 4)
    return p.reshape(-1, 3), q


def scalp(kind: str):
    """Scalp vertices on the unit sphere and quads.  kind: 'cap64' or 'head2000'."""
    if kind == "cap64":
        return _face_grid("top", 8, (-0.5, 0.5), (-0.5, 0.5))
    if kind == "head2000":
        pts, quads = [], []
        base = 0
        for face in ("top", "front", "back", "right", "left"):
            br = (-1.0, 1.0) if face == "top" else (0.0, 1.0)
            p, q = _face_grid(face, 20, (-1.0, 1.0), br)
            pts.append(p)
            quads.append(q + base)
            base += p.shape[0]
        return np.concatenate(pts), np.concatenate(quads)
    raise ValueError(kind)


def extrude_layers(scalp_pts: np.ndarray, n_layers: int, height: float, offset=(0.0, 0.0, 0.0)):
    """Layer l = p + n * height * l / (L-1), n = p (unit sphere normal)."""
    ls = []
    for l in range(n_layers):
        ls.append(scalp_pts * (1.0 + height * l / (n_layers - 1)))
    lp = np.stack(ls, 0) + np.asarray(offset, np.float64)
    return lp.astype(np.float32)


def _bundle_arrays(B, nstrands, cmax, scene=None, key=None):
    ns = np.broadcast_to(np.asarray(nstrands, np.uint32), (B,)).copy()
    cm = np.broadcast_to(np.asarray(cmax, np.uint32), (B,)).copy()
    sc = np.zeros(B, np.uint32) if scene is None else np.asarray(scene, np.uint32)
    ky = np.arange(B, dtype=np.uint32) if key is None else np.asarray(key, np.uint32)
    base = np.zeros(B, np.uint32)
    if B > 1:
        base[1:] = np.cumsum(ns.astype(np.int64))[:-1].astype(np.uint32)
    return ns, cm, sc, ky, base


def _jitter_rgb(rng, n, base, sigma=0.05):
    rgb = np.asarray(base, np.float64)[None, :] + rng.normal(0.0, sigma, (n, 3))
    return np.clip(rgb, 0.0, 1.0).astype(np.float32)


# ----------------------------------------------------------------------------- workloads
def config_tiny(seed=1001, width=256, height=256) -> Scene:
    """64 quads on a unit-sphere cap, 4 layers, 16 strands/quad, 8 segments, 256x256."""
    pts, quads = scalp("cap64")
    lp = extrude_layers(pts, 4, 0.3)
    B = quads.shape[0]
    ns, cm, sc, ky, base = _bundle_arrays(B, 16, 9)
    cam = look_at_camera((0.0, 1.3, 2.6), (0.0, 1.0, 0.0), width, height, znear=0.1, zfar=10.0)
    return Scene("tiny", lp, quads.astype(np.uint32), ky, ns, cm, sc, base, None,
                 cam[None], width, height, None, seed=seed, strand_width=0.002,
                 curl_amp=0.02, mode=MODE_FILTER)


def config_head(seed=1002, width=1920, height=1080, strands_per_quad=64, n_cp=17,
                strand_width=0.0008, occluder=True, mode=MODE_FILTER,
                eye=(0.0, 0.4, 4.0), target=(0.0, 0.4, 0.0)) -> Scene:
    """Full head: 2000 quads x 6 layers, 64 strands/quad, 16 segments, 1080p."""
    rng = np.random.default_rng(seed)
    pts, quads = scalp("head2000")
    lp = extrude_layers(pts, 6, 0.5)
    B = quads.shape[0]
    ns, cm, sc, ky, base = _bundle_arrays(B, strands_per_quad, n_cp)
    rgb = _jitter_rgb(rng, int(ns.astype(np.int64).sum()), (0.30, 0.18, 0.10))
    cam = look_at_camera(eye, target, width, height, znear=0.1, zfar=10.0)[None]
    sz = sphere_depth(cam, width, height, [(0.0, 0.0, 0.0)]) if occluder else None
    return Scene("head", lp, quads.astype(np.uint32), ky, ns, cm, sc, base, rgb, cam,
                 width, height, sz, seed=seed, strand_width=strand_width, mode=mode)


def config_lod(seed=1003, width=2560, height=1440, n_heads=32, lod_lambda=3.0, d_near=2.0,
               d_far=60.0) -> Scene:
    """32 full-head characters at geometric distances 2..60 in one 1440p view, LOD on."""
    rng = np.random.default_rng(seed)
    pts, quads = scalp("head2000")
    B0 = quads.shape[0]
    nv = pts.shape[0]
    vfov = math.radians(40.0)
    hfov = 2.0 * math.atan(width / height * math.tan(vfov / 2))
    layers, qs, centers = [], [], []
    for k in range(n_heads):
        d = d_near * (d_far / d_near) ** (k / max(n_heads - 1, 1))
        frac = (0.618 * k) % 1.0
        a = (frac - 0.5) * 0.8 * hfov
        c = np.array([d * math.sin(a), -0.4, -d * math.cos(a)])
        centers.append(c)
        layers.append(extrude_layers(pts, 6, 0.5, offset=c))
        qs.append(quads + k * nv)
    lp = np.concatenate(layers, axis=1)
    quads_all = np.concatenate(qs).astype(np.uint32)
    B = quads_all.shape[0]
    key = (np.arange(B) % B0).astype(np.uint32)
    ns, cm, sc, ky, base = _bundle_arrays(B, 64, 17, key=key)
    # same groom on every head: colours repeat per head
    rgb1 = _jitter_rgb(rng, B0 * 64, (0.30, 0.18, 0.10))
    rgb = np.tile(rgb1, (n_heads, 1))
    cam = look_at_camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), width, height, znear=0.5, zfar=64.0)[None]
    sz = sphere_depth(cam, width, height, centers)
    return Scene("lod", lp, quads_all, ky, ns, cm, sc, base, rgb, cam, width, height, sz,
                 seed=seed, strand_width=0.0008, lod_mode=LOD_ON, lod_lambda=lod_lambda,
                 mode=MODE_FILTER, meta={"centers": np.array(centers)})


def config_batched(seed=1004, n_scenes=64, res=512, n_min=1e3, n_max=2e5) -> Scene:
    """64 independent 512x512 scenes, 1k..200k strands (log-uniform), 8..16 segments."""
    rng = np.random.default_rng(seed)
    pts, quads = scalp("head2000")
    lp = extrude_layers(pts, 6, 0.5)
    B0 = quads.shape[0]
    n_k = np.round(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_scenes))).astype(np.int64)
    c_k = rng.integers(9, 18, n_scenes)
    cams, ns_all, cm_all, sc_all = [], [], [], []
    for s in range(n_scenes):
        r = rng.uniform(3.0, 8.0)
        az = rng.uniform(0.0, 2 * math.pi)
        el = math.radians(rng.uniform(-10.0, 40.0))
        eye = (r * math.cos(el) * math.sin(az), 0.3 + r * math.sin(el), r * math.cos(el) * math.cos(az))
        cams.append(look_at_camera(eye, (0.0, 0.3, 0.0), res, res, znear=0.1, zfar=16.0))
        nb = np.full(B0, n_k[s] // B0, np.int64)
        nb[: n_k[s] % B0] += 1
        ns_all.append(nb)
        cm_all.append(np.full(B0, c_k[s], np.int64))
        sc_all.append(np.full(B0, s, np.int64))
    cams = np.stack(cams)
    quads_all = np.tile(quads, (n_scenes, 1)).astype(np.uint32)
    key = np.tile(np.arange(B0), n_scenes).astype(np.uint32)
    ns, cm, sc, ky, base = _bundle_arrays(quads_all.shape[0], np.concatenate(ns_all),
                                          np.concatenate(cm_all), np.concatenate(sc_all), key)
    rgb = _jitter_rgb(rng, int(ns.astype(np.int64).sum()), (0.30, 0.18, 0.10))
    sz = sphere_depth(cams, res, res, [(0.0, 0.0, 0.0)])
    return Scene("batched", lp, quads_all, ky, ns, cm, sc, base, rgb, cams, res, res, sz,
                 seed=seed, strand_width=0.0008, mode=MODE_FILTER)


def config_diff(seed=1005, res=512, strands_per_quad=16) -> Scene:
    """32k strands x 16 segments at 512x512, soft-coverage resolve.  The
    coverage tests use a 1 px minimum half width so the visibility buffer
    reaches the Gaussian footprint of the soft coverage (3.5 sigma)."""
    sc = config_head(seed=seed, width=res, height=res, strands_per_quad=strands_per_quad,
                     n_cp=17, strand_width=0.002, occluder=False, mode=MODE_SOFT)
    sc.r_min = 1.0
    return sc


def perturb_stream(pos_w: np.ndarray, rgb: np.ndarray, seed: int, sigma=0.01):
    """Target parameters for the differentiable workload: positions + N(0, s),
    widths * (1 + N(0, s)), colours + N(0, s).  Inputs are [n_cp][4] float32."""
    rng = np.random.default_rng(seed)
    p = pos_w.astype(np.float64).copy()
    c = rgb.astype(np.float64).copy()
    p[:, :3] += rng.normal(0.0, sigma, (p.shape[0], 3))
    p[:, 3] *= 1.0 + rng.normal(0.0, sigma, p.shape[0])
    c[:, :3] += rng.normal(0.0, sigma, (c.shape[0], 3))
    return p.astype(np.float32), c.astype(np.float32)


def select_scene(sc: Scene, s: int) -> Scene:
    """Scene s of a multi-scene frame as a frame of its own."""
    sel = np.nonzero(sc.bundle_scene == s)[0]
    ns = sc.bundle_nstrands[sel].copy()
    base = np.zeros(sel.size, np.uint32)
    if sel.size > 1:
        base[1:] = np.cumsum(ns.astype(np.int64))[:-1].astype(np.uint32)
    rgb = None
    if sc.strand_rgb is not None and sel.size:
        a = int(sc.strand_base[sel[0]])
        rgb = sc.strand_rgb[a:a + int(ns.astype(np.int64).sum())].copy()
    return dataclasses.replace(
        sc, name=f"{sc.name}[{s}]", quads=sc.quads[sel].copy(), bundle_key=sc.bundle_key[sel].copy(),
        bundle_nstrands=ns, bundle_cmax=sc.bundle_cmax[sel].copy(),
        bundle_scene=np.zeros(sel.size, np.uint32), strand_base=base, strand_rgb=rgb,
        cams=sc.cams[s:s + 1].copy(),
        scene_z=None if sc.scene_z is None else sc.scene_z[s:s + 1].copy(), meta={})


CONFIGS = {
    "tiny": config_tiny,
    "head": config_head,
    "lod": config_lod,
    "batched": config_batched,
    "diff": config_diff,
}


def build(name: str, **kw) -> Scene:
    return CONFIGS[name](**kw)


def micro_scene(seed: int, n_bundles=3, n_layers=3, strands=4, n_cp=5, res=32,
                width=0.05, curl=0.02) -> Scene:
    """A tiny random groom seen up close, for brute-force checks."""
    rng = np.random.default_rng(seed)
    B = n_bundles
    lp = np.zeros((n_layers, 4 * B, 3), np.float64)
    quads = np.arange(4 * B, dtype=np.uint32).reshape(B, 4)
    for b in range(B):
        c = rng.uniform(-0.3, 0.3, 3)
        c[2] = rng.uniform(-0.3, 0.3)
        s = rng.uniform(0.05, 0.2)
        corners = np.array([[-s, 0, -s], [s, 0, -s], [s, 0, s], [-s, 0, s]]) + c
        d = rng.normal(0, 1, 3)
        d /= np.linalg.norm(d)
        for l in range(n_layers):
            lp[l, 4 * b:4 * b + 4] = corners + d * 0.3 * l + rng.normal(0, 0.02, (4, 3))
    ns, cm, sc, ky, base = _bundle_arrays(B, strands, n_cp)
    cam = look_at_camera((0.2, 0.5, 2.0), (0.0, 0.1, 0.0), res, res, vfov_deg=40.0,
                         znear=0.1, zfar=10.0)[None]
    return Scene(f"micro{seed}", lp.astype(np.float32), quads, ky, ns, cm, sc, base, None, cam,
                 res, res, None, seed=seed, strand_width=width, curl_amp=curl)
