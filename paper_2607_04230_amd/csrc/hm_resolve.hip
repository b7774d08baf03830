// Deferred resolve (Sec. 3.3, 3.4, Code 2) for gfx950.
//
//   k_shade   one thread per pixel: shades the centre-sample hit once
//             (deferred, 1 spp) and writes a 16-byte record
//             {r, g, b, bits(depth24 | centre-hit << 24 | any-hit << 25)};
//   k_filter  16 x 16 pixel workgroups stage the records of their tile plus
//             an r-pixel halo in LDS and run strand connection, the elliptical
//             bilateral filter and alpha estimation out of LDS;
//   k_soft    soft-coverage resolve (one thread per pixel).
#include "hm_device.hpp"
#include "hm_internal.hpp"

namespace hm {

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

__device__ __forceinline__ V3 cp_tangent(const float4 *pos, const uint8_t *flags, uint32_t v)
{
    const uint8_t f = flags[v];
    V3 d;
    if (f & HM_ROOT) d = xyz(pos[v + 1]) - xyz(pos[v]);
    else if (f & HM_TIP) d = xyz(pos[v]) - xyz(pos[v - 1]);
    else d = xyz(pos[v + 1]) - xyz(pos[v - 1]);
    return nrm(d);
}

__device__ __forceinline__ SegShade seg_shade_point(const float4 *pos, const float4 *rgb,
                                                    const uint8_t *flags, DProj a, DProj b,
                                                    uint32_t v, double px, double py)
{
    SegShade r;
    r.ts = closest_t(a, b, px, py);
    const double iz = a.iz + r.ts * (b.iz - a.iz);
    r.t3 = (float)(r.ts * b.iz / iz);
    const V3 P0 = xyz(pos[v]), P1 = xyz(pos[v + 1]);
    r.X = P0 + (P1 - P0) * r.t3;
    const V3 T0 = cp_tangent(pos, flags, v), T1 = cp_tangent(pos, flags, v + 1);
    r.T = nrm(T0 + (T1 - T0) * r.t3);
    const V3 c0 = xyz(rgb[v]), c1 = xyz(rgb[v + 1]);
    r.alb = c0 + (c1 - c0) * r.t3;
    return r;
}

// Kajiya-Kay style diffuse sin(T, L) plus a specular lobe (1 - (T.H)^2)^(2^n).
__device__ __forceinline__ V3 shade(const SegShade &g, const Cam &c, const ShadeK &k)
{
    const V3 L = v3(k.Lx, k.Ly, k.Lz);
    const V3 V = nrm(v3(c.ex, c.ey, c.ez) - g.X);
    const V3 H = nrm(L + V);
    const float tl = dot(g.T, L), th = dot(g.T, H);
    const float sd = 1.0f - tl * tl;
    const float diff = sd > 0.0f ? sqrtf(sd) : 0.0f;
    float sp = fmaxx(1.0f - th * th, 0.0f);
    for (int i = 0; i < k.nsq; ++i) sp = sp * sp;
    const float dd = k.ka + k.kd * diff;
    return v3(g.alb.x * k.Er * dd + k.ks * k.Er * sp, g.alb.y * k.Eg * dd + k.ks * k.Eg * sp,
              g.alb.z * k.Eb * dd + k.ks * k.Eb * sp);
}

// ------------------------------------------------------------------ centre shading
__global__ __launch_bounds__(256) void k_shade(const float4 *pos, const float4 *rgb,
                                               const uint8_t *flags, const uint64_t *vis,
                                               const hm_camera *cams, uint32_t S, uint32_t W,
                                               uint32_t H, ShadeK k, float4 *rec, float4 *out)
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
            const DProj a = project_d(c, pos[v]), b = project_d(c, pos[v + 1]);
            const uint32_t j = (uint32_t)(loc / W), i = (uint32_t)(loc - (size_t)j * W);
            const SegShade g = seg_shade_point(pos, rgb, flags, a, b, v, (double)i + 0.5,
                                               (double)j + 0.5);
            col = shade(g, c, k);
        }
        const uint32_t bits = (hc ? (uint32_t)(kc >> HM_ID_BITS) : 0u) | (hc ? 1u << 24 : 0u) |
                              ((hc || ha) ? 1u << 25 : 0u);
        if (rec) rec[p] = make_float4(col.x, col.y, col.z, __uint_as_float(bits));
        if (out) {
            out[p] = hc ? make_float4(col.x, col.y, col.z, 1.0f)
                        : make_float4(k.bgr, k.bgg, k.bgb, 0.0f);
        }
    }
}

// ------------------------------------------------------------------ filter
constexpr int FT = 16;          // output tile edge
constexpr int RMAX = 8;         // largest supported radius
constexpr int HALO_MAX = FT + 2 * RMAX;

__global__ __launch_bounds__(256) void k_filter(const float4 *pos, const uint64_t *vis,
                                                const hm_camera *cams, uint32_t W, uint32_t H,
                                                ShadeK k, const float4 *rec, float4 *out)
{
    __shared__ float4 tile[HALO_MAX * HALO_MAX];
    const int r = k.r;
    const int E = FT + 2 * r;
    const uint32_t tiles_x = (W + FT - 1) / FT;
    const uint32_t tiles_y = (H + FT - 1) / FT;
    const uint32_t s = blockIdx.x / (tiles_x * tiles_y);
    const uint32_t tr = blockIdx.x - s * tiles_x * tiles_y;
    const int ty = (int)(tr / tiles_x), tx = (int)(tr - (uint32_t)ty * tiles_x);
    const int ox0 = tx * FT - r, oy0 = ty * FT - r;
    const size_t hw = (size_t)W * H;
    const float4 *recs = rec + (size_t)s * hw;
    for (int x = threadIdx.x; x < E * E; x += blockDim.x) {
        const int ly = x / E, lx = x - ly * E;
        const int gi = ox0 + lx, gj = oy0 + ly;
        float4 v = make_float4(0.f, 0.f, 0.f, __uint_as_float(0u));
        if (gi >= 0 && gj >= 0 && gi < (int)W && gj < (int)H) v = recs[(size_t)gj * W + gi];
        tile[ly * E + lx] = v;
    }
    __syncthreads();
    const int li = (int)(threadIdx.x % FT), lj = (int)(threadIdx.x / FT);
    const int i = tx * FT + li, j = ty * FT + lj;
    if (i >= (int)W || j >= (int)H) return;
    const size_t loc = (size_t)j * W + i;
    const uint64_t kc = vis[(size_t)s * 2 * hw + loc], ka = vis[(size_t)s * 2 * hw + hw + loc];
    const bool hc = is_hit(kc), ha = is_hit(ka);
    float4 *o = out + (size_t)s * hw + loc;
    if (!hc && !ha) {
        *o = make_float4(k.bgr, k.bgg, k.bgb, 0.0f);
        return;
    }
    const uint32_t qc = (uint32_t)(kc >> HM_ID_BITS), qa = (uint32_t)(ka >> HM_ID_BITS);
    const bool mism = hc && ha && qc > qa && (qc - qa) >= k.dq_mis;
    const uint64_t src = (hc && !mism) ? kc : ka;
    const uint32_t vs = (uint32_t)(src & HM_ID_MASK);
    const uint32_t qP = (uint32_t)(src >> HM_ID_BITS);
    const Cam c = load_cam(cams + s);
    const float4 pa = project(c, pos[vs]), pb = project(c, pos[vs + 1]);
    const float tdx = pb.x - pa.x, tdy = pb.y - pa.y;
    const float tlen = sqrtf(tdx * tdx + tdy * tdy);
    const bool iso = !(tlen >= k.iso_len);
    // binary32 tangent: strip membership decision (same bits as any IEEE
    // evaluation); binary64 tangent: the continuous filter weights
    float Tx = 0.0f, Ty = 0.0f, Twx = 0.0f, Twy = 0.0f;
    if (!iso) {
        const float il = 1.0f / tlen;
        Tx = tdx * il;
        Ty = tdy * il;
        const DProj da = project_d(c, pos[vs]), db = project_d(c, pos[vs + 1]);
        const double ddx = db.x - da.x, ddy = db.y - da.y;
        const double dl = sqrt(ddx * ddx + ddy * ddy);
        Twx = (float)(ddx / dl);
        Twy = (float)(ddy / dl);
    }
    const float4 CP = tile[(lj + r) * E + (li + r)];
    const bool colour_sim = hc && !mism;
    // normalised sum with a running exponent shift: sum_q exp(e_q - m) C_q /
    // sum_q exp(e_q - m), m = max e_q so far (no underflow of the weight sum)
    float Sx = 0.f, Sy = 0.f, Sz = 0.f, Wsum = 0.f, emax = -INFINITY;
    int Hc = 0, Ha = 0, nacc = 0;
    for (int oy = -r; oy <= r; ++oy) {
        const float4 *row = tile + (lj + r + oy) * E + (li + r);
        const float fy = (float)oy;
        for (int ox = -r; ox <= r; ++ox) {
            const float4 Q = row[ox];
            const uint32_t bits = __float_as_uint(Q.w);
            const bool qh = (bits >> 24) & 1u, qany = (bits >> 25) & 1u;
            const float fx = (float)ox;
            float par, perp2;
            if (iso) {
                par = 0.0f;
                perp2 = fx * fx + fy * fy;
            } else {
                par = fx * Tx + fy * Ty;
                const float ex = fx - par * Tx, ey = fy - par * Ty;
                perp2 = ex * ex + ey * ey;
            }
            if (perp2 <= k.strip2) {
                Ha += qany ? 1 : 0;
                Hc += qh ? 1 : 0;
            }
            if (!qh) continue;
            const uint32_t qq = bits & 0xFFFFFFu;
            const uint32_t dq = qq > qP ? qq - qP : qP - qq;
            if (dq > k.dq_rej) continue;
            float e;
            if (iso) {
                e = -(perp2 * k.inv_siso2);
            } else {
                const float pw = fx * Twx + fy * Twy;        // d_par with the accurate tangent
                const float cw = fx * Twy - fy * Twx;        // signed d_perp
                e = -(pw * pw * k.inv_spar2) - cw * cw * k.inv_sperp2;
            }
            if (colour_sim) {
                const float d0 = CP.x - Q.x, d1 = CP.y - Q.y, d2 = CP.z - Q.z;
                e -= (d0 * d0 + d1 * d1 + d2 * d2) * k.inv_sc2;
            }
            if (e > emax) {
                const float sc = expf(emax - e);
                Sx *= sc; Sy *= sc; Sz *= sc; Wsum *= sc;
                emax = e;
            }
            const float w = expf(e - emax);
            Sx += w * Q.x;
            Sy += w * Q.y;
            Sz += w * Q.z;
            Wsum += w;
            ++nacc;
        }
    }
    const float aP = Ha > 0 ? (float)Hc / (float)Ha : 1.0f;
    float rr = 0.f, gg = 0.f, bb = 0.f, alpha = 0.f;
    if (hc && !mism) {
        rr = Sx / Wsum; gg = Sy / Wsum; bb = Sz / Wsum;
        alpha = aP;
    } else if (mism) {
        float cr = CP.x, cg = CP.y, cb = CP.z;
        if (nacc > 0) {
            cr = Sx / Wsum; cg = Sy / Wsum; cb = Sz / Wsum;
        }
        rr = aP * cr + (1.0f - aP) * CP.x;
        gg = aP * cg + (1.0f - aP) * CP.y;
        bb = aP * cb + (1.0f - aP) * CP.z;
        alpha = 1.0f;
    } else if (nacc > 0) {
        rr = Sx / Wsum; gg = Sy / Wsum; bb = Sz / Wsum;
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
                                              const uint8_t *flags, const uint64_t *vis,
                                              const hm_camera *cams, uint32_t S, uint32_t W,
                                              uint32_t H, ShadeK k, float4 *out)
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
        const float4 P0 = pos[v], P1 = pos[v + 1];
        const DProj a = project_d(c, P0), b = project_d(c, P1);
        const uint32_t j = (uint32_t)(loc / W), i = (uint32_t)(loc - (size_t)j * W);
        const double px = (double)i + 0.5, py = (double)j + 0.5;
        const SegShade g = seg_shade_point(pos, rgb, flags, a, b, v, px, py);
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
                           (const uint8_t *)s.flags, vis, cams, f.n_scenes, f.width, f.height, k,
                           o);
        return;
    }
    if (k.mode == HM_RESOLVE_CENTER) {
        hipLaunchKernelGGL(k_shade, dim3(stride_grid(npix, 256)), dim3(256), 0, st, pos, rgb,
                           (const uint8_t *)s.flags, vis, cams, f.n_scenes, f.width, f.height, k,
                           (float4 *)nullptr, o);
        return;
    }
    float4 *rec = reinterpret_cast<float4 *>(ws);
    hipLaunchKernelGGL(k_shade, dim3(stride_grid(npix, 256)), dim3(256), 0, st, pos, rgb,
                       (const uint8_t *)s.flags, vis, cams, f.n_scenes, f.width, f.height, k, rec,
                       (float4 *)nullptr);
    const uint32_t tiles = ((f.width + FT - 1) / FT) * ((f.height + FT - 1) / FT) * f.n_scenes;
    hipLaunchKernelGGL(k_filter, dim3(tiles), dim3(FT * FT), 0, st, pos, vis, cams, f.width,
                       f.height, k, (const float4 *)rec, o);
}

void launch_resolve_bwd(const hm_strands &s, const uint64_t *vis, const hm_camera *cams,
                        const hm_frame &f, const ShadeK &k, const float *d_out, float *gpos,
                        float *grgb, hipStream_t st)
{
    (void)s; (void)vis; (void)cams; (void)f; (void)k; (void)d_out; (void)gpos; (void)grgb;
    (void)st;
}

}  // namespace hm
