// Device-side building blocks of libhm (gfx950, wave64).
//
// Floating-point contract: the steps whose results decide integers (strand
// hash -> uv, LOD counts, generation, projection, coverage predicates,
// 24-bit depth code, filter strip decisions) use binary32 with the operation
// order spelled out here, compiled with -ffp-contract=off and correctly
// rounded division / square root, so they reproduce the same bits as any
// IEEE binary32 evaluation of the same expressions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hm.h"

#define HM_EMPTY 0xFFFFFFFFFFFFFFFFull
#define HM_ID_BITS 40
#define HM_ID_MASK ((1ull << HM_ID_BITS) - 1ull)
#define HM_ID_OPAQUE ((1ull << HM_ID_BITS) - 2ull)
#define HM_QMAX 16777215u
#define HM_ROOT 1u
#define HM_TIP 2u

namespace hm {

// ----------------------------------------------------------------- hashing
// PCG hash (Jarzynski & Olano 2020): LCG step + RXS-M-XS output permutation.
__device__ __forceinline__ uint32_t pcg(uint32_t v)
{
    uint32_t s = v * 747796405u + 2891336453u;
    uint32_t w = ((s >> ((s >> 28u) + 4u)) ^ s) * 277803737u;
    return (w >> 22u) ^ w;
}

// top 24 bits as a float in [0, 1)
__device__ __forceinline__ float unit24(uint32_t h) { return (float)(h >> 8) * 0x1p-24f; }

__device__ __forceinline__ uint32_t bundle_hash(uint32_t seed, uint32_t key)
{
    return pcg(pcg(seed) ^ key);
}

__device__ __forceinline__ float fminx(float a, float b) { return a < b ? a : b; }
__device__ __forceinline__ float fmaxx(float a, float b) { return a > b ? a : b; }

// ----------------------------------------------------------------- camera
struct Cam {
    float R[9];
    float ex, ey, ez;
    float fx, fy, cx, cy, zn, zf;
};

__device__ __forceinline__ Cam load_cam(const hm_camera *c)
{
    Cam k;
#pragma unroll
    for (int i = 0; i < 9; ++i) k.R[i] = c->R[i];
    k.ex = c->eye[0]; k.ey = c->eye[1]; k.ez = c->eye[2];
    k.fx = c->fx; k.fy = c->fy; k.cx = c->cx; k.cy = c->cy;
    k.zn = c->znear; k.zf = c->zfar;
    return k;
}

// Camera-space coordinates: rows of R dotted with (P - eye), summed left to right.
__device__ __forceinline__ void to_camera(const Cam &c, float px, float py, float pz,
                                         float &X, float &Y, float &Z)
{
    float dx = px - c.ex, dy = py - c.ey, dz = pz - c.ez;
    X = (c.R[0] * dx + c.R[1] * dy) + c.R[2] * dz;
    Y = (c.R[3] * dx + c.R[4] * dy) + c.R[5] * dz;
    Z = (c.R[6] * dx + c.R[7] * dy) + c.R[8] * dz;
}

// Screen record of a control point: (x_px, y_px, width_px, 1/z); 1/z = 0 marks
// a point outside the open depth range (znear, zfar).
__device__ __forceinline__ float4 project(const Cam &c, float4 p)
{
    float X, Y, Z;
    to_camera(c, p.x, p.y, p.z, X, Y, Z);
    if (!(Z > c.zn && Z < c.zf)) return make_float4(0.f, 0.f, 0.f, 0.f);
    float iz = 1.0f / Z;
    float4 o;
    o.x = c.cx + c.fx * (X * iz);
    o.y = c.cy - c.fy * (Y * iz);
    o.z = p.w * (c.fy * iz);
    o.w = iz;
    return o;
}

// 1 / x for x in [2^-126, 2^126): the hardware reciprocal (about 1 ulp)
// refined by one Newton step with fused multiply-adds, e = 1 - x y, y + e y.
// On gfx950 this equals the correctly rounded quotient 1.0f / x for every x in
// that range (hm_bench_reciprocal counts the exceptions over all of them).
__device__ __forceinline__ float rcp_refined(float x)
{
    const float y = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, y, 1.0f);
    return __builtin_fmaf(e, y, y);
}

// 24-bit normalised linear depth, truncated and clamped.
__device__ __forceinline__ uint32_t depth_code(float z, float zn, float inv_range)
{
    float d = (z - zn) * inv_range;
    float fq = d * 16777216.0f;
    // branch-free: truncation of min(fq, 2^24 - 1) for fq > 0, else 0
    const float c = fq < 16777215.0f ? fq : 16777215.0f;
    return fq > 0.0f ? (uint32_t)c : 0u;
}

// ----------------------------------------------------------------- coverage
// Per-segment constants of the two coverage tests.
struct Seg {
    float x0, y0, w0, iz0;
    float dx, dy, dw, diz;
    float len2, ilen2, ra;
    float sxmn, sxmx, symn, symx;
    float idy;              // 1/dy for candidate enumeration (0 when |dy| <= 1e-3)
    float e;                // slack of candidate enumeration against binary32 rounding
    float iz1;              // 1/z of the second endpoint (G-buffer payload parameter)
};

// Slack of candidate enumeration: 0.05 px, widened by ~8 ulp of the largest
// magnitude involved so that clips of far off-screen endpoints stay
// conservative.
__device__ __forceinline__ float seg_slack(const Seg &s)
{
    const float m = fmaxx(fmaxx(fmaxx(fabsf(s.sxmn), fabsf(s.sxmx)),
                                fmaxx(fabsf(s.symn), fabsf(s.symx))), s.ra);
    return 0.05f + 1e-6f * m;
}

__device__ __forceinline__ Seg make_seg(float4 a, float4 b, float r_min)
{
    Seg s;
    s.x0 = a.x; s.y0 = a.y; s.w0 = a.z; s.iz0 = a.w;
    s.dx = b.x - a.x;
    s.dy = b.y - a.y;
    s.dw = b.z - a.z;
    s.diz = b.w - a.w;
    s.len2 = s.dx * s.dx + s.dy * s.dy;
    s.ilen2 = s.len2 > 0.0f ? 1.0f / s.len2 : 0.0f;
    float ra = 0.5f * fmaxx(a.z, b.z);
    s.ra = fmaxx(ra, r_min);
    s.sxmn = fminx(a.x, b.x); s.sxmx = fmaxx(a.x, b.x);
    s.symn = fminx(a.y, b.y); s.symx = fmaxx(a.y, b.y);
    s.idy = fabsf(s.dy) > 1e-3f ? 1.0f / s.dy : 0.0f;
    s.e = seg_slack(s);
    s.iz1 = b.w;
    return s;
}

// Coverage of pixel (i, j): `centre` (centre sample) and `cons`
// (conservative); q gets the depth code at the clamped closest point.  Returns
// centre || cons.
__device__ __forceinline__ bool cover_tz(const Seg &s, int i, int j, float r_min, float zn,
                                         float inv_range, bool &centre, bool &cons, uint32_t &q,
                                         float &ts_out, float &z_out);

__device__ __forceinline__ bool cover(const Seg &s, int i, int j, float r_min, float zn,
                                      float inv_range, bool &centre, bool &cons, uint32_t &q)
{
    float ts, z;
    return cover_tz(s, i, j, r_min, zn, inv_range, centre, cons, q, ts, z);
}

// As cover; also returns the clamped closest-point parameter ts and the linear
// depth z of the depth code.
__device__ __forceinline__ bool cover_tz(const Seg &s, int i, int j, float r_min, float zn,
                                         float inv_range, bool &centre, bool &cons, uint32_t &q,
                                         float &ts_out, float &z_out)
{
    // Evaluated without branches except for the rare degenerate segment: the
    // two tests, the closest point and the depth code are computed for every
    // candidate pixel.  For a degenerate segment ilen2 = 0, so t = 0 and r is
    // the endpoint radius.  fminf / fmaxf (v_min / v_max) stand for the
    // ternary minimum and maximum where only the sign of a zero could differ,
    // which no comparison below can see (and a NaN radius from t = 0 * inf
    // yields r_min either way).
    const float fi = (float)i, fj = (float)j;
    const float ux = (fi + 0.5f) - s.x0;
    const float uy = (fj + 0.5f) - s.y0;
    const float tn = ux * s.dx + uy * s.dy;
    const float t = tn * s.ilen2;
    const float wt = s.w0 + t * s.dw;
    const float r = fmaxf(0.5f * wt, r_min);
    const float r2 = r * r;
    if (__builtin_expect(s.len2 > 0.0f, 1)) {
        const float cr = ux * s.dy - uy * s.dx;
        centre = (tn >= 0.0f) & (tn < s.len2) & (cr * cr <= r2 * s.len2);
    } else {
        centre = (ux * ux + uy * uy) <= r2;
    }
    const float bx0 = fi - s.ra, bx1 = (fi + 1.0f) + s.ra;
    const float by0 = fj - s.ra, by1 = (fj + 1.0f) + s.ra;
    const float fa = (bx0 - s.x0) * s.dy, fb = (bx1 - s.x0) * s.dy;
    const float ga = (by0 - s.y0) * s.dx, gb = (by1 - s.y0) * s.dx;
    const float lo = fminf(fa, fb) - fmaxf(ga, gb);
    const float hi = fmaxf(fa, fb) - fminf(ga, gb);
    cons = (s.sxmn <= bx1) & (s.sxmx >= bx0) & (s.symn <= by1) & (s.symx >= by0) &
           (lo <= 0.0f) & (hi >= 0.0f);
    float ts = t;
    ts = fmaxx(ts, 0.0f);
    ts = fminx(ts, 1.0f);
    const float iz = s.iz0 + ts * s.diz;
    const float z = 1.0f / iz;
    q = depth_code(z, zn, inv_range);
    ts_out = ts;
    z_out = z;
    return centre | cons;
}

// ----------------------------------------------------------------- compressed G-buffer
// The 64-bit deferred-shading word of Sec. 3.1.2: depth code << 40, then
// octahedral tangent (u, v: 8 bits each), albedo r, g, b (6 bits each) and
// ambient occlusion (6 bits, 63: none baked).  Quantisation rounds to
// nearest; every step is binary32 in the order written.
__device__ __forceinline__ uint32_t gb_q8(float x)
{
    float f = (x * 0.5f + 0.5f) * 255.0f + 0.5f;
    f = f > 0.0f ? f : 0.0f;
    f = f < 255.0f ? f : 255.0f;
    return (uint32_t)f;
}

__device__ __forceinline__ uint32_t gb_q6(float c)
{
    float f = c * 63.0f + 0.5f;
    f = f > 0.0f ? f : 0.0f;
    f = f < 63.0f ? f : 63.0f;
    return (uint32_t)f;
}

// Octahedral map: project onto |x| + |y| + |z| = 1, fold the lower half
// (z < 0) across the diagonals, keep (x, y); the zero vector maps to the centre.
__device__ __forceinline__ uint32_t gb_oct16(float tx, float ty, float tz)
{
    const float l1 = (fabsf(tx) + fabsf(ty)) + fabsf(tz);
    float px = 0.0f, py = 0.0f;
    if (l1 > 0.0f) {
        px = tx / l1;
        py = ty / l1;
        if (tz < 0.0f) {
            const float ax = fabsf(px), ay = fabsf(py);
            const float sx = px >= 0.0f ? 1.0f : -1.0f, sy = py >= 0.0f ? 1.0f : -1.0f;
            px = (1.0f - ay) * sx;
            py = (1.0f - ax) * sy;
        }
    }
    return (gb_q8(px) << 8) | gb_q8(py);
}

// Payload of segment v (stream point v) at closest-point parameter ts and
// linear depth z: the perspective-correct segment parameter
// t3 = ts * (1/z_1) * z, then tangent and albedo interpolated at t3.
__device__ __forceinline__ uint64_t gb_payload_of(float4 T0, float4 T1, float4 c0, float4 c1,
                                                  float ts, float z, float iz1)
{
    const float t3 = (ts * iz1) * z;
    const float tx = T0.x + t3 * (T1.x - T0.x);
    const float ty = T0.y + t3 * (T1.y - T0.y);
    const float tz = T0.z + t3 * (T1.z - T0.z);
    const float cr = c0.x + t3 * (c1.x - c0.x);
    const float cg = c0.y + t3 * (c1.y - c0.y);
    const float cb = c0.z + t3 * (c1.z - c0.z);
    return ((uint64_t)gb_oct16(tx, ty, tz) << 24) | ((uint64_t)gb_q6(cr) << 18) |
           ((uint64_t)gb_q6(cg) << 12) | ((uint64_t)gb_q6(cb) << 6) | 63u;
}

__device__ __forceinline__ uint64_t gb_payload(const float4 *tan, const float4 *rgb, uint32_t v,
                                               float ts, float z, float iz1)
{
    return gb_payload_of(tan[v], tan[v + 1], rgb[v], rgb[v + 1], ts, z, iz1);
}

// Unit tangent of a stream point for the G-buffer keys, as the resolve
// computes it: root -> next, tip <- previous, else the central difference
// b - a of its neighbours (a = previous or itself, b = next or itself); zero
// for a point that is both root and tip (no segment).
__device__ __forceinline__ float4 cp_unit_tangent(float4 a, float4 b, bool root_and_tip)
{
    float dx = 0.0f, dy = 0.0f, dz = 0.0f;
    if (!root_and_tip) {
        dx = b.x - a.x;
        dy = b.y - a.y;
        dz = b.z - a.z;
    }
    const float n2 = (dx * dx + dy * dy) + dz * dz;
    float4 t = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (n2 > 0.0f) {
        const float inv = 1.0f / sqrtf(n2);
        t = make_float4(dx * inv, dy * inv, dz * inv, 0.0f);
    }
    return t;
}

// Raster-side inputs of the G-buffer keys (null tan: segment-id keys).
struct GbK {
    const float4 *tan;      // unit tangent per control point
    const float4 *rgb;      // albedo per control point
};

// Candidate pixel box of a segment (superset of every pixel either predicate
// can accept), clipped to the image.  Returns false if empty.
__device__ __forceinline__ bool seg_box(const Seg &sg, uint32_t W, uint32_t H, int &i0, int &i1,
                                        int &j0, int &j1)
{
    const float xmn = sg.sxmn - sg.ra - 2.0f, xmx = sg.sxmx + sg.ra + 2.0f;
    const float ymn = sg.symn - sg.ra - 2.0f, ymx = sg.symx + sg.ra + 2.0f;
    if (!(xmx >= 0.0f && ymx >= 0.0f && xmn <= (float)W && ymn <= (float)H)) return false;
    i0 = xmn > 0.0f ? (int)xmn : 0;
    j0 = ymn > 0.0f ? (int)ymn : 0;
    i1 = xmx < (float)(W - 1) ? (int)xmx : (int)W - 1;
    j1 = ymx < (float)(H - 1) ? (int)ymx : (int)H - 1;
    return i0 <= i1 && j0 <= j1;
}

// Column range of candidate pixels in row j.  Pixel (i, j) can pass either
// test only if the segment has a point with y in [j - ra, j + 1 + ra] and x in
// [i - ra, i + 1 + ra] (the centre test's disc of radius r <= ra around the
// pixel centre lies inside that square).  So: clip the segment to the row band
// widened by ra, and take i in [x_lo - 1 - ra, x_hi + ra]; the slack sg.e
// (0.05 px plus ~8 ulp of the coordinates' magnitude) absorbs binary32
// rounding of the clip: an error of the clip parameter is bounded by the
// rounding of its numerator over |dy|, far below the band's widening e / |dy|.
__device__ __forceinline__ void row_span(const Seg &sg, int j, int &i0, int &i1)
{
    const float e = sg.e;
    const float ylo = ((float)j - sg.ra) - e, yhi = (((float)j + 1.0f) + sg.ra) + e;
    float xlo = sg.sxmn, xhi = sg.sxmx;
    if (sg.idy != 0.0f) {
        float ta = (ylo - sg.y0) * sg.idy, tb = (yhi - sg.y0) * sg.idy;
        float t0 = fmaxx(fminx(ta, tb), 0.0f), t1 = fminx(fmaxx(ta, tb), 1.0f);
        if (t0 > t1) { i0 = 1; i1 = 0; return; }
        float xa = sg.x0 + t0 * sg.dx, xb = sg.x0 + t1 * sg.dx;
        xlo = fminx(xa, xb);
        xhi = fmaxx(xa, xb);
    } else if (sg.symx < ylo || sg.symn > yhi) {
        i0 = 1; i1 = 0;
        return;
    }
    const float flo = ((xlo - 1.0f) - sg.ra) - e, fhi = (xhi + sg.ra) + e;
    i0 = flo > -1.0e9f ? (int)ceilf(flo) : -1000000000;
    i1 = fhi < 1.0e9f ? (int)floorf(fhi) : 1000000000;
}

// Scene of control point c: last s with scene_off[s] <= c (scene_off non-decreasing).
__device__ __forceinline__ uint32_t scene_of(const uint32_t *scene_off, uint32_t n_scenes,
                                             uint32_t c)
{
    uint32_t lo = 0, hi = n_scenes;      // invariant: scene_off[lo] <= c < scene_off[hi]
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (scene_off[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// ----------------------------------------------------------------- wave / block scans
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// 32-bit inclusive scan over the 64 lanes of a full wave with DPP moves:
// row_shr 1, 2, 4, 8 give the prefix inside each row of 16 lanes;
// row_bcast 15 adds the end of rows 0 / 2 to rows 1 / 3, and row_bcast 31 the
// end of row 1 to rows 2 and 3.  Every lane of the wave must be active.
template <>
__device__ __forceinline__ uint32_t wave_inclusive_scan<uint32_t>(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
    return x;
}

// Value of lane 63 (wave-uniform).
__device__ __forceinline__ uint32_t wave_last(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Exclusive scan over the block; lds must hold blockDim.x / 64 values.  Returns
// the exclusive prefix and writes the block total to `total`.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T *lds, T &total)
{
    const int lane = lane_id();
    const int wid = (int)(threadIdx.x >> 6);
    const int nw = (int)(blockDim.x >> 6);
    T inc = wave_inclusive_scan(x);
    if (lane == 63) lds[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        T v = lane < nw ? lds[lane] : (T)0;
        T vi = wave_inclusive_scan(v);
        if (lane < nw) lds[lane] = vi - v;
        if (lane == nw - 1) lds[nw] = vi;
    }
    __syncthreads();
    T res = inc - x + lds[wid];
    total = lds[nw];
    __syncthreads();
    return res;
}

}  // namespace hm
