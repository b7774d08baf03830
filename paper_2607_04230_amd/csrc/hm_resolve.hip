// Deferred resolve (Sec. 3.3, 3.4, Code 2) for gfx950.
//
//   k_shade       one thread per pixel: shades the centre-sample hit once
//                 (deferred, 1 spp) and writes a 16-byte record
//                 {r, g, b, word}: word = the centre hit's 24-bit depth code,
//                 REC_CONS_ONLY for a pixel with a conservative hit only,
//                 REC_EMPTY for no hit;
//   k_filter      16 x 16 pixel workgroups stage the records of their tile
//                 plus an r-pixel halo in LDS and run strand connection, the
//                 elliptical bilateral filter and alpha estimation out of LDS;
//   k_shade_gbuf  centre shading of compressed G-buffer keys (decode only);
//   k_soft        soft-coverage resolve (one thread per pixel), and
//   k_soft_bwd    its binary64 backward, summed per 16 x 16 tile in LDS;
//   k_dom_shadow  deep-opacity-map transmittance of each pixel's shaded point.
#include "hm_device.hpp"
#include "hm_internal.hpp"

namespace hm {

// Record words of pixels without a centre hit: above every depth code and
// further from it than any depth window of the filter (thresholds < 2^24 codes).
constexpr uint32_t REC_EMPTY = 0x40000000u;
constexpr uint32_t REC_CONS_ONLY = 0x60000000u;

struct V3 { float x, y, z; };
__device__ __forceinline__ V3 v3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 xyz(float4 p) { return {p.x, p.y, p.z}; }
__device__ __forceinline__ V3 nrm(V3 a)
{
    const float n2 = dot(a, a);
    if (!(n2 > 0.0f)) return {0.0f, 0.0f, 0.0f};
    return a * (1.0f / sqrtf(n2));
}

__device__ __forceinline__ bool is_hit(uint64_t k)
{
    return k != HM_EMPTY && (k & HM_ID_MASK) != HM_ID_OPAQUE;
}

// Everything the shading of one pixel needs about its segment.
struct SegShade {
    double ts;              // closest screen-space parameter
    float t3;               // matching segment parameter (perspective-correct)
    V3 X, T;                // shading point and unit tangent
    V3 alb;
};

// Screen position and 1/z in binary64.  Continuous resolve quantities (the
// closest-point parameter, pixel distance, screen tangent of the filter
// weights) are ill-conditioned for segments nearly parallel to the view ray:
// binary32 pixel coordinates around 10^3 px carry ~1e-4 px of rounding.
struct DProj { double x, y, iz; };

__device__ __forceinline__ DProj project_d(const Cam &c, float4 p)
{
    const double dx = (double)p.x - c.ex, dy = (double)p.y - c.ey, dz = (double)p.z - c.ez;
    const double X = (double)c.R[0] * dx + (double)c.R[1] * dy + (double)c.R[2] * dz;
    const double Y = (double)c.R[3] * dx + (double)c.R[4] * dy + (double)c.R[5] * dz;
    const double Z = (double)c.R[6] * dx + (double)c.R[7] * dy + (double)c.R[8] * dz;
    const double iz = 1.0 / Z;
    return {(double)c.cx + (double)c.fx * X * iz, (double)c.cy - (double)c.fy * Y * iz, iz};
}

// Closest screen-space parameter of pixel centre (px, py) on segment a -> b.
__device__ __forceinline__ double closest_t(DProj a, DProj b, double px, double py)
{
    const double dx = b.x - a.x, dy = b.y - a.y;
    const double len2 = dx * dx + dy * dy;
    if (!(len2 > 0.0)) return 0.0;
    const double t = ((px - a.x) * dx + (py - a.y) * dy) / len2;
    return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
}

// The stream values the shading of segment v reads: its points and colours,
// the flags of both points and the neighbours their tangents may need.
struct SegPts {
    float4 Pm, P0, P1, P2, C0, C1;
    uint8_t f0, f1;
};

// All of them loaded together (one round of gathers): a neighbour outside
// the stream (v = 0, or v + 2 >= n) is replaced by a point of the segment,
// which the flags then never use (v is a root, or v + 1 a tip).
__device__ __forceinline__ SegPts load_seg_pts(const float4 *pos, const float4 *rgb,
                                               const uint8_t *flags, uint32_t v, uint32_t n)
{
    SegPts q;
    q.f0 = flags[v];
    q.f1 = flags[v + 1];
    q.Pm = pos[v > 0 ? v - 1 : v];
    q.P0 = pos[v];
    q.P1 = pos[v + 1];
    q.P2 = pos[v + 2 < n ? v + 2 : v + 1];
    q.C0 = rgb[v];
    q.C1 = rgb[v + 1];
    return q;
}

// Unit tangents of the segment's two points from the loaded values: forward
// difference at a root, backward at a tip, central otherwise.
__device__ __forceinline__ void seg_tangents(const SegPts &q, V3 &T0, V3 &T1)
{
    V3 d0, d1;
    if (q.f0 & HM_ROOT) d0 = xyz(q.P1) - xyz(q.P0);
    else if (q.f0 & HM_TIP) d0 = xyz(q.P0) - xyz(q.Pm);
    else d0 = xyz(q.P1) - xyz(q.Pm);
    if (q.f1 & HM_ROOT) d1 = xyz(q.P2) - xyz(q.P1);
    else if (q.f1 & HM_TIP) d1 = xyz(q.P1) - xyz(q.P0);
    else d1 = xyz(q.P2) - xyz(q.P0);
    T0 = nrm(d0);
    T1 = nrm(d1);
}

__device__ __forceinline__ SegShade seg_shade_pts(const SegPts &q, DProj a, DProj b, double px,
                                                  double py)
{
    SegShade r;
    r.ts = closest_t(a, b, px, py);
    const double iz = a.iz + r.ts * (b.iz - a.iz);
    r.t3 = (float)(r.ts * b.iz / iz);
    const V3 P0 = xyz(q.P0), P1 = xyz(q.P1);
    r.X = P0 + (P1 - P0) * r.t3;
    V3 T0, T1;
    seg_tangents(q, T0, T1);
    r.T = nrm(T0 + (T1 - T0) * r.t3);
    const V3 c0 = xyz(q.C0), c1 = xyz(q.C1);
    r.alb = c0 + (c1 - c0) * r.t3;
    return r;
}

// Kajiya-Kay style diffuse sin(T, L) plus a specular lobe (1 - (T.H)^2)^(2^n);
// sh (the light's transmittance) scales both direct terms, not the ambient one.
__device__ __forceinline__ V3 shade(const SegShade &g, const Cam &c, const ShadeK &k,
                                    float sh = 1.0f, float ao = 1.0f)
{
    const V3 L = v3(k.Lx, k.Ly, k.Lz);
    const V3 V = nrm(v3(c.ex, c.ey, c.ez) - g.X);
    const V3 H = nrm(L + V);
    const float tl = dot(g.T, L), th = dot(g.T, H);
    const float sd = 1.0f - tl * tl;
    const float diff = sd > 0.0f ? sqrtf(sd) : 0.0f;
    float sp = fmaxx(1.0f - th * th, 0.0f);
    for (int i = 0; i < k.nsq; ++i) sp = sp * sp;
    const float dd = k.ka * ao + (sh * k.kd) * diff;
    const float ks = sh * k.ks;
    return v3(g.alb.x * k.Er * dd + ks * k.Er * sp, g.alb.y * k.Eg * dd + ks * k.Eg * sp,
              g.alb.z * k.Eb * dd + ks * k.Eb * sp);
}

// ------------------------------------------------------------------ centre shading
__global__ __launch_bounds__(256) void k_shade(const float4 *pos, const float4 *rgb,
                                               const uint8_t *flags, uint32_t n_cp,
                                               const uint64_t *vis, const hm_camera *cams,
                                               uint32_t S, uint32_t W, uint32_t H, ShadeK k,
                                               float4 *rec, float4 *out)
{
    const size_t hw = (size_t)W * H;
    const size_t n = hw * S;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n;
         p += (size_t)gridDim.x * blockDim.x) {
        const uint32_t s = (uint32_t)(p / hw);
        const size_t loc = p - (size_t)s * hw;
        const uint64_t kc = vis[(size_t)s * 2 * hw + loc], ka = vis[(size_t)s * 2 * hw + hw + loc];
        const bool hc = is_hit(kc), ha = is_hit(ka);
        V3 col = v3(0.f, 0.f, 0.f);
        if (hc) {
            const Cam c = load_cam(cams + s);
            const uint32_t v = (uint32_t)(kc & HM_ID_MASK);
            const SegPts q = load_seg_pts(pos, rgb, flags, v, n_cp);
            const DProj a = project_d(c, q.P0), b = project_d(c, q.P1);
            const uint32_t j = (uint32_t)(loc / W), i = (uint32_t)(loc - (size_t)j * W);
            const SegShade g = seg_shade_pts(q, a, b, (double)i + 0.5, (double)j + 0.5);
            col = shade(g, c, k, k.shadow ? k.shadow[p] : 1.0f);
        }
        const uint32_t bits = hc ? (uint32_t)(kc >> HM_ID_BITS)
                                 : (ha ? REC_CONS_ONLY : REC_EMPTY);
        if (rec) rec[p] = make_float4(col.x, col.y, col.z, __uint_as_float(bits));
        if (out) {
            out[p] = hc ? make_float4(col.x, col.y, col.z, 1.0f)
                        : make_float4(k.bgr, k.bgg, k.bgb, 0.0f);
        }
    }
}

// ------------------------------------------------------------------ G-buffer shading
// Centre resolve of a buffer of compressed keys: each centre-hit pixel is
// shaded from its key alone (no stream read): position rebuilt at the pixel
// centre from the middle of its depth code's interval (binary64), unit
// tangent from the octahedral code (unfold the lower half, normalise),
// albedo and occlusion from their 6-bit codes.
__global__ __launch_bounds__(256) void k_shade_gbuf(const uint64_t *vis, const hm_camera *cams,
                                                    uint32_t S, uint32_t W, uint32_t H, ShadeK k,
                                                    float4 *out)
{
    const size_t hw = (size_t)W * H;
    const size_t n = hw * S;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n;
         p += (size_t)gridDim.x * blockDim.x) {
        const uint32_t s = (uint32_t)(p / hw);
        const size_t loc = p - (size_t)s * hw;
        const uint64_t kc = vis[(size_t)s * 2 * hw + loc];
        float4 o = make_float4(k.bgr, k.bgg, k.bgb, 0.0f);
        if (is_hit(kc)) {
            const hm_camera *cp = cams + s;
            const Cam c = load_cam(cp);
            const uint64_t w = kc & HM_ID_MASK;
            const uint32_t j = (uint32_t)(loc / W), i = (uint32_t)(loc - (size_t)j * W);
            const double px = (double)i + 0.5, py = (double)j + 0.5;
            const double zn = cp->znear, zf = cp->zfar;
            const double z = zn + ((double)(kc >> HM_ID_BITS) + 0.5) / 16777216.0 * (zf - zn);
            const double xc = (px - (double)cp->cx) * z / (double)cp->fx;
            const double yc = -(py - (double)cp->cy) * z / (double)cp->fy;
            const double R[9] = {cp->R[0], cp->R[1], cp->R[2], cp->R[3], cp->R[4],
                                 cp->R[5], cp->R[6], cp->R[7], cp->R[8]};
            SegShade g;
            g.X = v3((float)((double)cp->eye[0] + (R[0] * xc + R[3] * yc + R[6] * z)),
                     (float)((double)cp->eye[1] + (R[1] * xc + R[4] * yc + R[7] * z)),
                     (float)((double)cp->eye[2] + (R[2] * xc + R[5] * yc + R[8] * z)));
            float u = (float)((w >> 32) & 0xFFu) / 255.0f * 2.0f - 1.0f;
            float v = (float)((w >> 24) & 0xFFu) / 255.0f * 2.0f - 1.0f;
            const float tz = (1.0f - fabsf(u)) - fabsf(v);
            if (tz < 0.0f) {
                const float au = fabsf(u), av = fabsf(v);
                u = (1.0f - av) * (u >= 0.0f ? 1.0f : -1.0f);
                v = (1.0f - au) * (v >= 0.0f ? 1.0f : -1.0f);
            }
            g.T = nrm(v3(u, v, tz));
            g.alb = v3((float)((w >> 18) & 63u) / 63.0f, (float)((w >> 12) & 63u) / 63.0f,
                       (float)((w >> 6) & 63u) / 63.0f);
            const float ao = (float)(w & 63u) / 63.0f;
            const V3 col = shade(g, c, k, 1.0f, ao);
            o = make_float4(col.x, col.y, col.z, 1.0f);
        }
        out[p] = o;
    }
}

// ------------------------------------------------------------------ filter
constexpr int FT = 16;          // output tile edge
constexpr int RMAX = 8;         // largest supported radius
constexpr int HALO_MAX = FT + 2 * RMAX;

// Weighted colour sum of one output pixel, exponent-shifted.
struct FilterAcc {
    float Sx, Sy, Sz, Wsum, emax;
};

// Per-pixel constants of the weight taps.  Exponents are in log2 units: a
// tap's weight is 2^(e - emax) with
//   e = -(pw^2 A + cw^2 B) - |C_P - C_Q|^2 Csc,
// pw, cw the offset's components along / across the weight tangent (the
// isotropic fallback has A = B).  The spatial part is the quadratic form
//   qa fx^2 + qb fx fy + qc fy^2,
// evaluated per row as fx (qa fx + qb fy) + qc fy^2.  The colour part is
// expanded as Csc |C_P|^2 + Csc |C_Q|^2 - 2 Csc C_P . C_Q, with |C_Q|^2 staged
// beside each record and Csc |C_P|^2 folded into the row constant: four fused
// multiply-adds per tap (the expansion's rounding, a few 1e-7 of the exponent,
// is far inside the tolerance).  When the centre sample is a hit whose colour
// the filter compares against, the centre tap has e = 0 >= every other e (up
// to that rounding), so emax = 0 from the start; otherwise emax follows the
// running maximum (a far-off strand would underflow every weight), and the
// tap at the maximum adds exactly 1 to Wsum, so Wsum > 0 iff some neighbour
// was accepted.
struct FilterPix {
    float qa, qb, qc;
    float Csc;
    float gx, gy, gz;       // -2 Csc C_P
    uint32_t q_lo, q_span;  // accepted depth codes: (q - q_lo) mod 2^32 <= q_span
    bool track_max;
};

__device__ __forceinline__ void filter_tap(const FilterPix &f, FilterAcc &a, float fx, float r1,
                                           float r0, float4 Q, uint32_t word)
{
    // centre-sample hit within the depth window [qP - rej, qP + rej]: a
    // centre hit's word is its depth code, every other word lies above 2^29,
    // beyond any window
    const bool take = (word - f.q_lo) <= f.q_span;
    // continuous weight (tolerance-compared): fused multiply-adds are fine
    // here; Q.w = |C_Q|^2, r0 holds Csc |C_P|^2
    float g = fmaf(fx, fmaf(f.qa, fx, r1), r0);
    g = fmaf(Q.w, f.Csc, g);
    g = fmaf(f.gx, Q.x, g);
    g = fmaf(f.gy, Q.y, g);
    g = fmaf(f.gz, Q.z, g);
    const float e = -g;
    if (f.track_max && take && e > a.emax) {
        const float sc = __builtin_amdgcn_exp2f(a.emax - e);
        a.Sx *= sc; a.Sy *= sc; a.Sz *= sc; a.Wsum *= sc;
        a.emax = e;
    }
    const float w = take ? __builtin_amdgcn_exp2f(e - a.emax) : 0.0f;
    a.Sx = fmaf(w, Q.x, a.Sx);
    a.Sy = fmaf(w, Q.y, a.Sy);
    a.Sz = fmaf(w, Q.z, a.Sz);
    a.Wsum += w;
}

// Strip counts for alpha (Sec. 3.3): over the window taps whose distance to
// the strand's screen line through the pixel is within the strip half width
// h, count those with any hit (Ha) and with a centre hit (Hc; hcode holds 1 +
// 2^16 for a centre hit, 1 for a conservative hit only, 0 for none).
// Membership is decided in binary32 exactly as perp2 = |o - (o.T) T|^2 <= h^2
// (a zero tangent, the isotropic case, gives |o|^2).  Only taps near the line are
// tested: along the line's major axis every offset a in [-r, r] has its
// minor-axis candidates b in an interval of width 2h / |major component|
// around the line, widened by 0.05 against rounding (an error of perp2 of a
// few ulp of r^2 moves the boundary by far less).  With (P, Q) the tangent's
// components along the major and minor axis, o.T = a P + b Q and the two
// components of o - (o.T) T are a - (o.T) P and b - (o.T) Q: the same
// products and sums as the (x, y) form, only added in the other order for a
// steep tangent, which leaves every binary32 result unchanged.
__device__ __forceinline__ void strip_counts(const uint32_t *hcode, int E, int cx, int cy, int r,
                                             float Tx, float Ty, float h, float h2, int &Hc,
                                             int &Ha)
{
    uint32_t cnt = 0;       // Ha + 2^16 Hc
    const bool steep = fabsf(Ty) >= fabsf(Tx);      // iso (0, 0) counts as steep
    const float P = steep ? Ty : Tx, Q = steep ? Tx : Ty;
    const float aM = fabsf(P);
    const float slope = aM > 0.0f ? Q / P : 0.0f;
    const float half = (aM > 0.0f ? h / aM : h) + 0.05f;
    // word index steps along a and b
    const int sa = steep ? E : 1, sb = steep ? 1 : E;
    const int centre = cy * E + cx;
    for (int a = -r; a <= r; ++a) {
        const float fa = (float)a;
        const float c = fa * slope;
        const int b0 = max(-r, (int)ceilf(c - half)), b1 = min(r, (int)floorf(c + half));
        const float pa = fa * P;
        int idx = centre + a * sa + b0 * sb;
        float fb = (float)b0;
        for (int b = b0; b <= b1; ++b, fb += 1.0f, idx += sb) {
            const float par = pa + fb * Q;
            const float u = fa - par * P, v = fb - par * Q;
            const bool in = u * u + v * v <= h2;
            cnt += in ? hcode[idx] : 0u;
        }
    }
    Ha = (int)(cnt & 0xFFFFu);
    Hc = (int)(cnt >> 16);
}

// R > 0: the radius is a compile-time constant (each row of taps unrolls into
// LDS reads at fixed offsets); R = 0: any radius up to RMAX, read from k.r.
template <int R>
__global__ __launch_bounds__(256) void k_filter(const float4 *pos, const uint64_t *vis,
                                                const hm_camera *cams, uint32_t W, uint32_t H,
                                                ShadeK k, const float4 *rec, float4 *out)
{
    constexpr int EMAX = R > 0 ? FT + 2 * R : HALO_MAX;
    // colours with |C|^2, the record words apart, and per record the strip's
    // counts: 1 for any hit plus 2^16 for a centre hit (the strip reads
    // consecutive addresses)
    __shared__ float4 tile[EMAX * EMAX];
    __shared__ uint32_t words[EMAX * EMAX];
    __shared__ uint32_t hcode[EMAX * EMAX];
    const int r = R > 0 ? R : k.r;
    const int E = R > 0 ? EMAX : FT + 2 * r;
    const uint32_t tiles_x = (W + FT - 1) / FT;
    const uint32_t tiles_y = (H + FT - 1) / FT;
    const uint32_t s = blockIdx.x / (tiles_x * tiles_y);
    const uint32_t tr = blockIdx.x - s * tiles_x * tiles_y;
    const int ty = (int)(tr / tiles_x), tx = (int)(tr - (uint32_t)ty * tiles_x);
    const int ox0 = tx * FT - r, oy0 = ty * FT - r;
    const size_t hw = (size_t)W * H;
    const float4 *recs = rec + (size_t)s * hw;
    const int li = (int)(threadIdx.x % FT), lj = (int)(threadIdx.x / FT);
    const int i = tx * FT + li, j = ty * FT + lj;
    const bool inb = i < (int)W && j < (int)H;
    const size_t loc = (size_t)j * W + i;
    uint64_t kc = HM_EMPTY, ka = HM_EMPTY;
    if (inb) {
        kc = vis[(size_t)s * 2 * hw + loc];
        ka = vis[(size_t)s * 2 * hw + hw + loc];
    }
    const bool hc = is_hit(kc), ha = is_hit(ka);
    float4 *o = out + (size_t)s * hw + loc;
    // a tile without hair pixels needs no records
    if (!__syncthreads_or(hc || ha)) {
        if (inb) *o = make_float4(k.bgr, k.bgg, k.bgb, 0.0f);
        return;
    }
    // the pixel's segment (the conservative one on a depth mismatch), its
    // control points loaded while the tile is staged
    const uint32_t qc = (uint32_t)(kc >> HM_ID_BITS), qa = (uint32_t)(ka >> HM_ID_BITS);
    const bool mism = hc && ha && qc > qa && (qc - qa) >= k.dq_mis;
    const uint64_t src = (hc && !mism) ? kc : ka;
    const uint32_t vs = (uint32_t)(src & HM_ID_MASK);
    float4 P0 = make_float4(0.f, 0.f, 0.f, 0.f), P1 = P0;
    if (hc || ha) {
        P0 = pos[vs];
        P1 = pos[vs + 1];
    }
    for (int x = threadIdx.x; x < E * E; x += blockDim.x) {
        const int ly = x / E, lx = x - ly * E;
        const int gi = ox0 + lx, gj = oy0 + ly;
        float4 v = make_float4(0.f, 0.f, 0.f, __uint_as_float(REC_EMPTY));
        if (gi >= 0 && gj >= 0 && gi < (int)W && gj < (int)H) v = recs[(size_t)gj * W + gi];
        tile[ly * E + lx] = make_float4(v.x, v.y, v.z, fmaf(v.x, v.x, fmaf(v.y, v.y, v.z * v.z)));
        const uint32_t wd = __float_as_uint(v.w);
        words[ly * E + lx] = wd;
        hcode[ly * E + lx] = (wd != REC_EMPTY ? 1u : 0u) + (wd <= HM_QMAX ? 0x10000u : 0u);
    }
    __syncthreads();
    if (!inb) return;
    if (!hc && !ha) {
        *o = make_float4(k.bgr, k.bgg, k.bgb, 0.0f);
        return;
    }
    const Cam c = load_cam(cams + s);
    const float4 pa = project(c, P0), pb = project(c, P1);
    const float tdx = pb.x - pa.x, tdy = pb.y - pa.y;
    const float tlen = sqrtf(tdx * tdx + tdy * tdy);
    const bool iso = !(tlen >= k.iso_len);
    const float4 CP = tile[(lj + r) * E + (li + r)];
    const bool colour_sim = hc && !mism;
    constexpr double LOG2E = 1.4426950408889634074;
    // binary32 tangent: strip membership decision (same bits as any IEEE
    // evaluation); binary64 tangent: the continuous filter weights
    float Tx = 0.0f, Ty = 0.0f;
    double A = k.inv_siso2 * LOG2E, B = A, Tw0 = 1.0, Tw1 = 0.0;
    if (!iso) {
        const float il = 1.0f / tlen;
        Tx = tdx * il;
        Ty = tdy * il;
        const DProj da = project_d(c, P0), db = project_d(c, P1);
        const double ddx = db.x - da.x, ddy = db.y - da.y;
        const double dl = sqrt(ddx * ddx + ddy * ddy);
        Tw0 = ddx / dl;
        Tw1 = ddy / dl;
        A = k.inv_spar2 * LOG2E;
        B = k.inv_sperp2 * LOG2E;
    }
    FilterPix f;
    f.qa = (float)(A * Tw0 * Tw0 + B * Tw1 * Tw1);
    f.qb = (float)(2.0 * Tw0 * Tw1 * (A - B));
    f.qc = (float)(A * Tw1 * Tw1 + B * Tw0 * Tw0);
    f.Csc = colour_sim ? (float)(k.inv_sc2 * LOG2E) : 0.0f;
    f.gx = -2.0f * f.Csc * CP.x;
    f.gy = -2.0f * f.Csc * CP.y;
    f.gz = -2.0f * f.Csc * CP.z;
    const float K0 = f.Csc * CP.w;          // Csc |C_P|^2
    const uint32_t qP = (uint32_t)(src >> HM_ID_BITS);
    f.q_lo = qP - k.dq_rej;
    f.q_span = 2u * k.dq_rej;
    f.track_max = !colour_sim;
    FilterAcc a;
    a.Sx = a.Sy = a.Sz = a.Wsum = 0.0f;
    a.emax = colour_sim ? 0.0f : -INFINITY;
    const float4 *ctr = tile + (lj + r) * E + (li + r);
    if (R > 0) {
        // the window's top-left record: every tap at a fixed non-negative
        // offset from it (an immediate of the LDS read)
        const float4 *win = tile + lj * EMAX + li;
        const uint32_t *wwin = words + lj * EMAX + li;
        // taps from the centre outwards (offsets 0, -1, 1, -2, 2, ...), so
        // that a running maximum meets its final value early and rescales
        // rarely
#pragma unroll 1
        for (int ky = 0; ky <= 2 * R; ++ky) {
            const int oy = (ky & 1) ? -((ky + 1) >> 1) : (ky >> 1);
            const float4 *row = win + (oy + R) * EMAX;
            const uint32_t *wrow = wwin + (oy + R) * EMAX;
            const float fy = (float)oy;
            const float r1 = f.qb * fy, r0 = fmaf(f.qc, fy * fy, K0);
#pragma unroll
            for (int kx = 0; kx <= 2 * R; ++kx) {
                const int ox = (kx & 1) ? -((kx + 1) >> 1) : (kx >> 1);
                filter_tap(f, a, (float)ox, r1, r0, row[ox + R], wrow[ox + R]);
            }
        }
    } else {
        const uint32_t *wctr = words + (lj + r) * E + (li + r);
        for (int oy = -r; oy <= r; ++oy) {
            const float fy = (float)oy;
            const float r1 = f.qb * fy, r0 = fmaf(f.qc, fy * fy, K0);
            for (int ox = -r; ox <= r; ++ox)
                filter_tap(f, a, (float)ox, r1, r0, ctr[oy * E + ox], wctr[oy * E + ox]);
        }
    }
    int Hc, Ha;
    strip_counts(hcode, E, li + r, lj + r, r, Tx, Ty, k.strip_half, k.strip2, Hc, Ha);
    const float aP = Ha > 0 ? (float)Hc / (float)Ha : 1.0f;
    float rr = 0.f, gg = 0.f, bb = 0.f, alpha = 0.f;
    if (hc && !mism) {
        rr = a.Sx / a.Wsum; gg = a.Sy / a.Wsum; bb = a.Sz / a.Wsum;
        alpha = aP;
    } else if (mism) {
        float cr = CP.x, cg = CP.y, cb = CP.z;
        if (a.Wsum > 0.0f) {
            cr = a.Sx / a.Wsum; cg = a.Sy / a.Wsum; cb = a.Sz / a.Wsum;
        }
        rr = aP * cr + (1.0f - aP) * CP.x;
        gg = aP * cg + (1.0f - aP) * CP.y;
        bb = aP * cb + (1.0f - aP) * CP.z;
        alpha = 1.0f;
    } else if (a.Wsum > 0.0f) {
        rr = a.Sx / a.Wsum; gg = a.Sy / a.Wsum; bb = a.Sz / a.Wsum;
        alpha = aP;
    }
    *o = make_float4(alpha * rr + (1.0f - alpha) * k.bgr, alpha * gg + (1.0f - alpha) * k.bgg,
                     alpha * bb + (1.0f - alpha) * k.bgb, alpha);
}

// ------------------------------------------------------------------ soft coverage
__device__ __forceinline__ uint64_t soft_source(uint64_t kc, uint64_t ka)
{
    return is_hit(kc) ? kc : (is_hit(ka) ? ka : HM_EMPTY);
}

__global__ __launch_bounds__(256) void k_soft(const float4 *pos, const float4 *rgb,
                                              const uint8_t *flags, uint32_t n_cp,
                                              const uint64_t *vis, const hm_camera *cams,
                                              uint32_t S, uint32_t W, uint32_t H, ShadeK k,
                                              float4 *out)
{
    const size_t hw = (size_t)W * H;
    const size_t n = hw * S;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n;
         p += (size_t)gridDim.x * blockDim.x) {
        const uint32_t s = (uint32_t)(p / hw);
        const size_t loc = p - (size_t)s * hw;
        const uint64_t src = soft_source(vis[(size_t)s * 2 * hw + loc],
                                         vis[(size_t)s * 2 * hw + hw + loc]);
        if (src == HM_EMPTY) {
            out[p] = make_float4(k.bgr, k.bgg, k.bgb, 0.0f);
            continue;
        }
        const Cam c = load_cam(cams + s);
        const uint32_t v = (uint32_t)(src & HM_ID_MASK);
        const SegPts q = load_seg_pts(pos, rgb, flags, v, n_cp);
        const float4 P0 = q.P0, P1 = q.P1;
        const DProj a = project_d(c, P0), b = project_d(c, P1);
        const uint32_t j = (uint32_t)(loc / W), i = (uint32_t)(loc - (size_t)j * W);
        const double px = (double)i + 0.5, py = (double)j + 0.5;
        const SegShade g = seg_shade_pts(q, a, b, px, py);
        const double ex = px - (a.x + g.ts * (b.x - a.x)), ey = py - (a.y + g.ts * (b.y - a.y));
        const float d = (float)sqrt(ex * ex + ey * ey);
        const double w0 = (double)P0.w * c.fy * a.iz, w1 = (double)P1.w * c.fy * b.iz;
        const float wt = (float)(w0 + g.ts * (w1 - w0));
        const float alpha = 0.5f * (erff((d + 0.5f * wt) * k.soft_k) - erff((d - 0.5f * wt) * k.soft_k));
        const V3 Sc = shade(g, c, k);
        out[p] = make_float4(alpha * Sc.x + (1.0f - alpha) * k.bgr,
                             alpha * Sc.y + (1.0f - alpha) * k.bgg,
                             alpha * Sc.z + (1.0f - alpha) * k.bgb, alpha);
    }
}

// ------------------------------------------------------------------ host side
size_t resolve_workspace(const hm_frame &f)
{
    return align_up(sizeof(float4) * (size_t)f.width * f.height * f.n_scenes);
}

void launch_resolve(const hm_strands &s, const uint64_t *vis, const hm_camera *cams,
                    const hm_frame &f, const ShadeK &k, float *out, void *ws, hipStream_t st)
{
    const float4 *pos = reinterpret_cast<const float4 *>(s.pos_w);
    const float4 *rgb = reinterpret_cast<const float4 *>(s.rgb);
    float4 *o = reinterpret_cast<float4 *>(out);
    const size_t npix = (size_t)f.width * f.height * f.n_scenes;
    if (k.mode == HM_RESOLVE_SOFT) {
        hipLaunchKernelGGL(k_soft, dim3(stride_grid(npix, 256)), dim3(256), 0, st, pos, rgb,
                           (const uint8_t *)s.flags, s.cap, vis, cams, f.n_scenes, f.width,
                           f.height, k, o);
        return;
    }
    if (k.payload == HM_PAYLOAD_GBUFFER) {
        hipLaunchKernelGGL(k_shade_gbuf, dim3(stride_grid(npix, 256)), dim3(256), 0, st, vis,
                           cams, f.n_scenes, f.width, f.height, k, o);
        return;
    }
    if (k.mode == HM_RESOLVE_CENTER) {
        hipLaunchKernelGGL(k_shade, dim3(full_grid(npix, 256)), dim3(256), 0, st, pos, rgb,
                           (const uint8_t *)s.flags, s.cap, vis, cams, f.n_scenes, f.width,
                           f.height, k, (float4 *)nullptr, o);
        return;
    }
    float4 *rec = reinterpret_cast<float4 *>(ws);
    hipLaunchKernelGGL(k_shade, dim3(full_grid(npix, 256)), dim3(256), 0, st, pos, rgb,
                       (const uint8_t *)s.flags, s.cap, vis, cams, f.n_scenes, f.width,
                       f.height, k, rec, (float4 *)nullptr);
    const uint32_t tiles = ((f.width + FT - 1) / FT) * ((f.height + FT - 1) / FT) * f.n_scenes;
    if (k.r == 5) {             // the paper's radius: unrolled taps
        hipLaunchKernelGGL(k_filter<5>, dim3(tiles), dim3(FT * FT), 0, st, pos, vis, cams,
                           f.width, f.height, k, (const float4 *)rec, o);
    } else {
        hipLaunchKernelGGL(k_filter<0>, dim3(tiles), dim3(FT * FT), 0, st, pos, vis, cams,
                           f.width, f.height, k, (const float4 *)rec, o);
    }
}

// ------------------------------------------------------------------ soft backward
// Reverse-mode derivative of the soft resolve of one pixel with respect to the
// control points v-1 .. v+2 (tangent stencil), the widths of v, v+1 and the
// colours of v, v+1, visibility held fixed.  Evaluated in binary64.
struct D3 { double x, y, z; };
__device__ __forceinline__ D3 d3(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(D3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dotd(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 dl(float4 p) { return {(double)p.x, (double)p.y, (double)p.z}; }
__device__ __forceinline__ double lend(D3 a) { return sqrt(dotd(a, a)); }
// gradient through u = a / |a|: (g - u (u.g)) / |a|
__device__ __forceinline__ D3 nrm_back(D3 u, double n, D3 g)
{
    if (!(n > 0.0)) return d3(0, 0, 0);
    return (g - u * dotd(u, g)) * (1.0 / n);
}

struct DCam {
    double R[9], e[3], fx, fy, cx, cy;
};

__device__ __forceinline__ DCam load_dcam(const hm_camera *c)
{
    DCam d;
#pragma unroll
    for (int i = 0; i < 9; ++i) d.R[i] = c->R[i];
    d.e[0] = c->eye[0]; d.e[1] = c->eye[1]; d.e[2] = c->eye[2];
    d.fx = c->fx; d.fy = c->fy; d.cx = c->cx; d.cy = c->cy;
    return d;
}

struct DPt { double x, y, iz, X, Y; };

__device__ __forceinline__ DPt proj_pt(const DCam &c, D3 P)
{
    const double dx = P.x - c.e[0], dy = P.y - c.e[1], dz = P.z - c.e[2];
    const double X = c.R[0] * dx + c.R[1] * dy + c.R[2] * dz;
    const double Y = c.R[3] * dx + c.R[4] * dy + c.R[5] * dz;
    const double Z = c.R[6] * dx + c.R[7] * dy + c.R[8] * dz;
    const double iz = 1.0 / Z;
    return {c.cx + c.fx * X * iz, c.cy - c.fy * Y * iz, iz, X, Y};
}

// gx dx/dP + gy dy/dP + giz d(1/z)/dP
__device__ __forceinline__ D3 proj_back(const DCam &c, const DPt &p, double gx, double gy,
                                        double giz)
{
    const double a0 = gx * c.fx * p.iz, a1 = -gy * c.fy * p.iz;
    const double a2 = -(gx * c.fx * p.X - gy * c.fy * p.Y + giz) * p.iz * p.iz;
    return d3(a0 * c.R[0] + a1 * c.R[3] + a2 * c.R[6], a0 * c.R[1] + a1 * c.R[4] + a2 * c.R[7],
              a0 * c.R[2] + a1 * c.R[5] + a2 * c.R[8]);
}

__device__ __forceinline__ void atomic_add3(float *base, D3 g)
{
    atomicAdd(base + 0, (float)g.x);
    atomicAdd(base + 1, (float)g.y);
    atomicAdd(base + 2, (float)g.z);
}

// Gradient contributions of one pixel of the soft resolve (binary64), or
// false when the pixel has no visible segment or a zero output gradient.
struct SoftGrad {
    uint32_t v;
    bool root, tip;
    float3 gP0, gP1, gPm, gPp;    // positions of v, v + 1, v - 1, v + 2
    float g_ww0, g_ww1;           // widths of v, v + 1
    float3 gc0, gc1;              // colours of v, v + 1
};

__device__ __forceinline__ float3 f3of(D3 a) { return make_float3((float)a.x, (float)a.y, (float)a.z); }

__device__ __forceinline__ bool soft_bwd_pixel(const float4 *pos, const float4 *rgb,
                                               const uint8_t *flags, const uint64_t *vis,
                                               const DCam &c, uint32_t s, uint32_t W,
                                               size_t hw, uint32_t i, uint32_t j, const ShadeK &k,
                                               const float4 *dout, SoftGrad &o)
{
    const double kk = k.soft_k, isp = 0.5641895835477563;   // 1/sqrt(pi)
    const size_t loc = (size_t)j * W + i;
    const size_t p = (size_t)s * hw + loc;
    const uint64_t src = soft_source(vis[(size_t)s * 2 * hw + loc],
                                     vis[(size_t)s * 2 * hw + hw + loc]);
    if (src == HM_EMPTY) return false;
    const float4 go = dout[p];
    if (go.x == 0.0f && go.y == 0.0f && go.z == 0.0f && go.w == 0.0f) return false;
    const uint32_t v = (uint32_t)(src & HM_ID_MASK);
    const uint8_t f0 = flags[v], f1 = flags[v + 1];
    const bool root = f0 & HM_ROOT, tip = f1 & HM_TIP;
    const float4 Q0 = pos[v], Q1 = pos[v + 1];
    const D3 P0 = dl(Q0), P1 = dl(Q1);
    const D3 Pm = root ? P0 : dl(pos[v - 1]);
    const D3 Pp = tip ? P1 : dl(pos[v + 2]);
    const double px = (double)i + 0.5, py = (double)j + 0.5;

    // ---- forward (binary64)
    const DPt a = proj_pt(c, P0), b = proj_pt(c, P1);
    const double w0 = (double)Q0.w * c.fy * a.iz, w1 = (double)Q1.w * c.fy * b.iz;
    const double dx = b.x - a.x, dy = b.y - a.y, len2 = dx * dx + dy * dy;
    const double ux = px - a.x, uy = py - a.y;
    double traw = len2 > 0.0 ? (ux * dx + uy * dy) / len2 : 0.0;
    const bool interior = len2 > 0.0 && traw > 0.0 && traw < 1.0;
    const double ts = traw < 0.0 ? 0.0 : (traw > 1.0 ? 1.0 : traw);
    const double ex = ux - ts * dx, ey = uy - ts * dy;
    const double d = sqrt(ex * ex + ey * ey);
    const double wt = w0 + ts * (w1 - w0);
    const double za = (d + 0.5 * wt) * kk, zb = (d - 0.5 * wt) * kk;
    const double alpha = 0.5 * (erf(za) - erf(zb));
    const double ga2 = exp(-za * za), gb2 = exp(-zb * zb);
    const double iz = a.iz + ts * (b.iz - a.iz);
    const double t3 = ts * b.iz / iz;
    const D3 X = P0 + (P1 - P0) * t3;
    const D3 D0 = root ? (P1 - P0) : (P1 - Pm);
    const D3 D1 = tip ? (P1 - P0) : (Pp - P0);
    const double n0 = lend(D0), n1 = lend(D1);
    const D3 T0 = n0 > 0 ? D0 * (1.0 / n0) : d3(0, 0, 0);
    const D3 T1 = n1 > 0 ? D1 * (1.0 / n1) : d3(0, 0, 0);
    const D3 Tm = T0 + (T1 - T0) * t3;
    const double nm = lend(Tm);
    const D3 T = nm > 0 ? Tm * (1.0 / nm) : d3(0, 0, 0);
    const D3 c0 = dl(rgb[v]), c1 = dl(rgb[v + 1]);
    const D3 alb = c0 + (c1 - c0) * t3;
    const D3 EV = d3(c.e[0], c.e[1], c.e[2]) - X;
    const double nv = lend(EV);
    const D3 V = EV * (1.0 / nv);
    const D3 L = d3(k.Lx, k.Ly, k.Lz);
    const D3 LV = L + V;
    const double nh = lend(LV);
    const D3 Hh = LV * (1.0 / nh);
    const double tl = dotd(T, L), th = dotd(T, Hh);
    const double sd = 1.0 - tl * tl;
    const double diff = sd > 0.0 ? sqrt(sd) : 0.0;
    const double sh0 = 1.0 - th * th;
    const double sh = sh0 > 0.0 ? sh0 : 0.0;
    double q = sh, shp = 1.0;                    // shp = sh^(2^n - 1)
    for (int it = 0; it < k.nsq; ++it) { shp *= q; q = q * q; }
    const double spec = q;
    const double E[3] = {k.Er, k.Eg, k.Eb}, bgc[3] = {k.bgr, k.bgg, k.bgb};
    const double albv[3] = {alb.x, alb.y, alb.z};
    const double gI[3] = {go.x, go.y, go.z};
    double Sv[3];
    const double dd = k.ka + k.kd * diff;
    for (int ch = 0; ch < 3; ++ch) Sv[ch] = albv[ch] * E[ch] * dd + k.ks * E[ch] * spec;

    // ---- backward
    double g_alpha = go.w;
    double galb[3], g_diff = 0.0, g_spec = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        g_alpha += gI[ch] * (Sv[ch] - bgc[ch]);
        const double gS = gI[ch] * alpha;
        galb[ch] = gS * E[ch] * dd;
        g_diff += gS * albv[ch] * E[ch] * k.kd;
        g_spec += gS * k.ks * E[ch];
    }
    const double g_sh = sh0 > 0.0 ? g_spec * (double)(1 << k.nsq) * shp : 0.0;
    const double g_th = -2.0 * th * g_sh;
    const double g_tl = sd > 0.0 ? -tl / diff * g_diff : 0.0;
    const D3 gT = L * g_tl + Hh * g_th;
    const D3 gH = T * g_th;
    const D3 gV = nrm_back(Hh, nh, gH);
    const D3 gX = nrm_back(V, nv, gV) * -1.0;
    const D3 gAlb = d3(galb[0], galb[1], galb[2]);
    double g_t3 = dotd(gAlb, c1 - c0);
    const D3 gc0 = gAlb * (1.0 - t3), gc1 = gAlb * t3;
    const D3 gTm = nrm_back(T, nm, gT);
    g_t3 += dotd(gTm, T1 - T0);
    const D3 gT0 = gTm * (1.0 - t3), gT1 = gTm * t3;
    const D3 gD0 = nrm_back(T0, n0, gT0), gD1 = nrm_back(T1, n1, gT1);
    D3 gP0 = gX * (1.0 - t3), gP1 = gX * t3, gPm = d3(0, 0, 0), gPp = d3(0, 0, 0);
    g_t3 += dotd(gX, P1 - P0);
    if (root) { gP1 = gP1 + gD0; gP0 = gP0 - gD0; } else { gP1 = gP1 + gD0; gPm = gPm - gD0; }
    if (tip) { gP1 = gP1 + gD1; gP0 = gP0 - gD1; } else { gPp = gPp + gD1; gP0 = gP0 - gD1; }
    // t3 = ts iz1 / iz(ts)
    const double iz2 = iz * iz;
    double g_ts = g_t3 * a.iz * b.iz / iz2;
    double g_iz0 = -g_t3 * ts * b.iz * (1.0 - ts) / iz2;
    double g_iz1 = g_t3 * ts * a.iz * (1.0 - ts) / iz2;
    // alpha(d, wt)
    const double g_d = g_alpha * kk * isp * (ga2 - gb2);
    const double g_wt = g_alpha * 0.5 * kk * isp * (ga2 + gb2);
    double g_w0 = g_wt * (1.0 - ts), g_w1 = g_wt * ts;
    g_ts += g_wt * (w1 - w0);
    double g_x0 = 0, g_y0 = 0, g_x1 = 0, g_y1 = 0;
    if (d > 0.0) {
        const double gex = g_d * ex / d, gey = g_d * ey / d;
        g_x0 += gex * (ts - 1.0); g_x1 += -gex * ts;
        g_y0 += gey * (ts - 1.0); g_y1 += -gey * ts;
        g_ts += -(gex * dx + gey * dy);
    }
    if (interior) {
        const double il = 1.0 / len2;
        g_x0 += g_ts * (-dx - ux + 2.0 * traw * dx) * il;
        g_x1 += g_ts * (ux - 2.0 * traw * dx) * il;
        g_y0 += g_ts * (-dy - uy + 2.0 * traw * dy) * il;
        g_y1 += g_ts * (uy - 2.0 * traw * dy) * il;
    }
    // pixel widths w = width fy / z
    g_iz0 += g_w0 * (double)Q0.w * c.fy;
    g_iz1 += g_w1 * (double)Q1.w * c.fy;
    const double g_ww0 = g_w0 * c.fy * a.iz, g_ww1 = g_w1 * c.fy * b.iz;
    gP0 = gP0 + proj_back(c, a, g_x0, g_y0, g_iz0);
    gP1 = gP1 + proj_back(c, b, g_x1, g_y1, g_iz1);

    o.v = v;
    o.root = root;
    o.tip = tip;
    o.gP0 = f3of(gP0); o.gP1 = f3of(gP1); o.gPm = f3of(gPm); o.gPp = f3of(gPp);
    o.g_ww0 = (float)g_ww0; o.g_ww1 = (float)g_ww1;
    o.gc0 = f3of(gc0); o.gc1 = f3of(gc1);
    return true;
}

// Per-workgroup gradient table: control point -> {d pos xyz, d width, d rgb},
// LDS adds, flushed with one global add per nonzero component and point.
constexpr uint32_t BWD_SLOTS = 1024;      // >= 4 points x 256 pixels: never full
constexpr uint32_t BWD_FREE = 0xFFFFFFFFu;

__device__ __forceinline__ void bwd_add(uint32_t *keys, float *vals, uint32_t cp, float3 gp,
                                        float gw, float3 gc)
{
    uint32_t sl = (cp * 2654435761u) >> 22;
    for (;;) {
        const uint32_t prev = atomicCAS(&keys[sl], BWD_FREE, cp);
        if (prev == BWD_FREE || prev == cp) break;
        sl = (sl + 1u) & (BWD_SLOTS - 1u);
    }
    float *o = vals + sl * 8u;
    const float g[7] = {gp.x, gp.y, gp.z, gw, gc.x, gc.y, gc.z};
#pragma unroll
    for (int q = 0; q < 7; ++q)
        if (g[q] != 0.0f) atomicAdd(o + q, g[q]);
}

// One 16 x 16 pixel tile per workgroup iteration: every pixel's contributions
// to the control points v - 1 .. v + 2 are summed in LDS (neighbouring pixels
// mostly share segments), then added to the global gradients.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_soft_bwd(const float4 *pos, const float4 *rgb,
                                                  const uint8_t *flags, const uint64_t *vis,
                                                  const hm_camera *cams, uint32_t S, uint32_t W,
                                                  uint32_t H, ShadeK k, const float4 *dout,
                                                  float *gpos, float *grgb)
{
    __shared__ uint32_t keys[BWD_SLOTS];
    __shared__ float vals[BWD_SLOTS * 8];
    const size_t hw = (size_t)W * H;
    const uint32_t ntx = (W + 15u) / 16u, nty = (H + 15u) / 16u;
    const uint32_t per = ntx * nty, ntiles = per * S;
    const uint32_t tid = threadIdx.x;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (uint32_t x = tid; x < BWD_SLOTS; x += blockDim.x) keys[x] = BWD_FREE;
        for (uint32_t x = tid; x < BWD_SLOTS * 8u; x += blockDim.x) vals[x] = 0.0f;
        __syncthreads();
        const uint32_t s = t / per, r = t - s * per;
        const uint32_t ty = r / ntx, tx = r - ty * ntx;
        const uint32_t i = tx * 16u + (tid & 15u), j = ty * 16u + (tid >> 4);
        SoftGrad g;
        if (i < W && j < H &&
            soft_bwd_pixel(pos, rgb, flags, vis, load_dcam(cams + s), s, W, hw, i, j, k, dout,
                           g)) {
            bwd_add(keys, vals, g.v, g.gP0, g.g_ww0, g.gc0);
            bwd_add(keys, vals, g.v + 1u, g.gP1, g.g_ww1, g.gc1);
            const float3 z3 = make_float3(0.0f, 0.0f, 0.0f);
            if (!g.root) bwd_add(keys, vals, g.v - 1u, g.gPm, 0.0f, z3);
            if (!g.tip) bwd_add(keys, vals, g.v + 2u, g.gPp, 0.0f, z3);
        }
        __syncthreads();
        for (uint32_t x = tid; x < BWD_SLOTS; x += blockDim.x) {
            const uint32_t cp = keys[x];
            if (cp == BWD_FREE) continue;
            const float *o = vals + x * 8u;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (o[q] != 0.0f) atomicAdd(gpos + 4 * (size_t)cp + q, o[q]);
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (o[4 + q] != 0.0f) atomicAdd(grgb + 4 * (size_t)cp + q, o[4 + q]);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ deep-opacity lookup
// Transmittance towards the light at the shaded point of every pixel with a
// centre hit, everything in binary64 in the order the host-side definition
// uses: screen projection as (f X) / Z, the closest screen parameter, the
// perspective-correct segment parameter, the point X, its light-view
// coordinates, light pixel and 24-bit depth code.  The LOD-corrected code
// q' = q0 + (uint32)((float)(q - q0) * beta) is a binary32 product; the
// opacity in front of q' sums whole layers and the interpolated part of the
// layer holding q' (the last layer taken whole once passed).
struct DomQ {
    uint32_t W, H, LW, LH;
    uint32_t layer_codes, n_layers, n_bundles;
    double alpha;
};

__device__ __forceinline__ void dom_proj(const DCam &c, D3 P, double &x, double &y, double &iz)
{
    const double dx = P.x - c.e[0], dy = P.y - c.e[1], dz = P.z - c.e[2];
    const double X = c.R[0] * dx + c.R[1] * dy + c.R[2] * dz;
    const double Y = c.R[3] * dx + c.R[4] * dy + c.R[5] * dz;
    const double Z = c.R[6] * dx + c.R[7] * dy + c.R[8] * dz;
    x = c.cx + c.fx * X / Z;
    y = c.cy - c.fy * Y / Z;
    iz = 1.0 / Z;
}

__global__ __launch_bounds__(256) void k_dom_shadow(const float4 *pos, const uint64_t *vis,
                                                    const hm_camera *cam, const hm_camera *light,
                                                    const uint64_t *light_vis,
                                                    const uint32_t *counts, const uint32_t *table,
                                                    const uint32_t *nstr, DomQ d, float *shadow)
{
    const size_t hw = (size_t)d.W * d.H, lhw = (size_t)d.LW * d.LH;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < hw;
         p += (size_t)gridDim.x * blockDim.x) {
        float T = 1.0f;
        const uint64_t kc = vis[p];
        if (is_hit(kc)) {
            const uint32_t v = (uint32_t)(kc & HM_ID_MASK);
            const DCam c = load_dcam(cam);
            const uint32_t j = (uint32_t)(p / d.W), i = (uint32_t)(p - (size_t)j * d.W);
            const D3 P0 = dl(pos[v]), P1 = dl(pos[v + 1]);
            double ax, ay, aiz, bx, by, biz;
            dom_proj(c, P0, ax, ay, aiz);
            dom_proj(c, P1, bx, by, biz);
            const double dx = bx - ax, dy = by - ay;
            const double len2 = dx * dx + dy * dy;
            double ts = 0.0;
            if (len2 > 0.0) {
                ts = (((double)i + 0.5 - ax) * dx + ((double)j + 0.5 - ay) * dy) / len2;
                ts = ts < 0.0 ? 0.0 : (ts > 1.0 ? 1.0 : ts);
            }
            const double iz = aiz + ts * (biz - aiz);
            const double t3 = ts * biz / iz;
            const D3 X = P0 + (P1 - P0) * t3;
            const DCam lc = load_dcam(light);
            const double zn = light->znear, zf = light->zfar;
            const double ex = X.x - lc.e[0], ey = X.y - lc.e[1], ez = X.z - lc.e[2];
            const double LX = lc.R[0] * ex + lc.R[1] * ey + lc.R[2] * ez;
            const double LY = lc.R[3] * ex + lc.R[4] * ey + lc.R[5] * ez;
            const double LZ = lc.R[6] * ex + lc.R[7] * ey + lc.R[8] * ez;
            const double lx = lc.cx + lc.fx * LX / LZ, ly = lc.cy - lc.fy * LY / LZ;
            if (LZ > zn && LZ < zf && lx >= 0.0 && ly >= 0.0 && lx < (double)d.LW &&
                ly < (double)d.LH) {
                const size_t lp = (size_t)floor(ly) * d.LW + (size_t)floor(lx);
                const uint64_t k0 = light_vis[lhw + lp];
                const double dq = (LZ - zn) / (zf - zn) * 16777216.0;
                const uint32_t q =
                    dq > 0.0 ? (dq >= 16777215.0 ? 16777215u : (uint32_t)dq) : 0u;
                const uint32_t q0 = (uint32_t)(k0 >> HM_ID_BITS);
                if (k0 != HM_EMPTY && q > q0) {
                    // bundle of segment v: last b with first CP table[4b+3] <= v
                    uint32_t lo = 0, hi = d.n_bundles;
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (table[4 * (size_t)mid + 3] <= v) lo = mid; else hi = mid;
                    }
                    const float beta = (float)table[4 * (size_t)lo] / (float)nstr[lo];
                    const uint32_t dd = (uint32_t)((float)(q - q0) * beta);
                    uint32_t kq = dd / d.layer_codes;
                    double f;
                    if (kq >= d.n_layers - 1) {
                        kq = d.n_layers - 1;
                        f = (double)(dd - kq * d.layer_codes) / d.layer_codes;
                        f = f < 1.0 ? f : 1.0;
                    } else {
                        f = (double)(dd - kq * d.layer_codes) / d.layer_codes;
                    }
                    double o = 0.0;
                    for (uint32_t k = 0; k < kq; ++k) o += counts[(size_t)k * lhw + lp];
                    o += f * counts[(size_t)kq * lhw + lp];
                    T = (float)exp(-d.alpha * o);
                }
            }
        }
        shadow[p] = T;
    }
}

void launch_dom_shadow(const hm_strands &s, const uint64_t *vis, const hm_camera *cam,
                       const hm_frame &f, const hm_camera *light, const hm_dom_params &p,
                       const uint64_t *light_vis, const uint32_t *counts, const uint32_t *table,
                       const uint32_t *nstr, uint32_t n_bundles, float *shadow, hipStream_t st)
{
    DomQ d;
    d.W = f.width; d.H = f.height; d.LW = p.width; d.LH = p.height;
    d.layer_codes = p.layer_codes; d.n_layers = p.n_layers; d.n_bundles = n_bundles;
    d.alpha = p.alpha;
    const size_t npix = (size_t)f.width * f.height;
    hipLaunchKernelGGL(k_dom_shadow, dim3(stride_grid(npix, 256)), dim3(256), 0, st,
                       reinterpret_cast<const float4 *>(s.pos_w), vis, cam, light, light_vis,
                       counts, table, nstr, d, shadow);
}

void launch_resolve_bwd(const hm_strands &s, const uint64_t *vis, const hm_camera *cams,
                        const hm_frame &f, const ShadeK &k, const float *d_out, float *gpos,
                        float *grgb, hipStream_t st)
{
    const size_t ntiles = (size_t)((f.width + 15) / 16) * ((f.height + 15) / 16) * f.n_scenes;
    hipLaunchKernelGGL(k_soft_bwd, dim3(stride_grid(ntiles * 256, 256)), dim3(256), 0, st,
                       reinterpret_cast<const float4 *>(s.pos_w),
                       reinterpret_cast<const float4 *>(s.rgb), (const uint8_t *)s.flags, vis,
                       cams, f.n_scenes, f.width, f.height, k,
                       reinterpret_cast<const float4 *>(d_out), gpos, grgb);
}

}  // namespace hm
