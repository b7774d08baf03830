// LOD pre-pass (Sec. 3.2) and strand generation (Sec. 3.1.1) for gfx950.
//
// The paper dispatches one workgroup per strand indirectly from the LOD
// buffer.  HIP has no indirect dispatch, so the LOD pass writes the per-bundle
// counts and a device prefix sum turns them into offsets (the table of
// {N_LOD, C, first strand, first CP}); generation then gives each bundle a
// workgroup, or one wave of one when there are many or small bundles, that
// reads its (possibly zero) row of the table.  A bundle's strand parameters, bilinear layer points and
// finite-difference layer tangents are computed once into LDS per chunk of
// strands; lanes then evaluate consecutive control points (Hermite + curl)
// and store them coalesced.  The fused variant also projects each control
// point and rasterizes the chunk's segments from LDS (the paper's
// assembly-and-raster in one pass); the binning variant projects each control
// point and bins the chunk's segments into screen tiles where they are
// generated, in place of the tile raster's first binning pass.
#include "hm_bin.hpp"
#include "hm_device.hpp"
#include "hm_internal.hpp"
#include "hm_scan.hpp"

namespace hm {

// ------------------------------------------------------------------ LOD
__device__ __forceinline__ void lod_counts(float L, uint32_t N, float delta, uint32_t cmax,
                                           uint32_t n_layers, uint32_t &n_lod, uint32_t &cps)
{
    int n = (int)ceilf(L * ((float)N + delta));
    n = n < 1 ? 1 : n;
    n = n > (int)N ? (int)N : n;
    n_lod = (uint32_t)n;
    int craw = (int)floorf(sqrtf(L) * (float)cmax);
    craw = craw < (int)n_layers ? (int)n_layers : craw;
    uint32_t p2 = 1u << (31 - __clz((uint32_t)(craw - 1)));   // 2^floor(log2(craw - 1))
    uint32_t c = p2 + 1u;
    cps = c > cmax ? cmax : c;
}

// Strand and control-point counts of bundle b (0 strands = culled).
__device__ __forceinline__ void lod_entry(const hm_hair_mesh &m, const hm_camera *cams, uint32_t W,
                                          uint32_t H, int mode, float lambda, uint32_t seed,
                                          uint32_t b, uint32_t &n_out, uint32_t &cp_out)
{
    const uint32_t N = m.bundle_nstrands[b];
    const uint32_t cmax = m.bundle_cmax[b] < 2u ? 2u : m.bundle_cmax[b];   // C >= 2 always
    uint32_t n = N, cp = cmax;
    if (mode == HM_LOD_ON && N > 0) {
        const Cam c = load_cam(cams + m.bundle_scene[b]);
        const uint4 q = reinterpret_cast<const uint4 *>(m.quads)[b];
        const uint32_t qi[4] = {q.x, q.y, q.z, q.w};
        float xmn = INFINITY, xmx = -INFINITY, ymn = INFINITY, ymx = -INFINITY;
        uint32_t n_near = 0;
        auto vertex = [&](float px, float py, float pz) {
            float X, Y, Z;
            to_camera(c, px, py, pz, X, Y, Z);
            if (Z <= c.zn) { n_near++; return; }
            float iz = 1.0f / Z;
            float x = c.cx + c.fx * (X * iz);
            float y = c.cy - c.fy * (Y * iz);
            xmn = fminx(x, xmn); xmx = fmaxx(x, xmx);
            ymn = fminx(y, ymn); ymx = fmaxx(y, ymx);
        };
        constexpr uint32_t LPRE = 6;          // layers whose vertices are loaded up front
        if (m.n_layers <= LPRE) {
            // all loads first (one memory latency per bundle), then the projections
            float P[LPRE][4][3];
#pragma unroll
            for (uint32_t l = 0; l < LPRE; ++l) {
                const float *lay = m.layer_pos + (size_t)(l < m.n_layers ? l : 0) * m.n_verts * 3;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float *q3 = lay + (size_t)qi[k] * 3;
                    P[l][k][0] = q3[0]; P[l][k][1] = q3[1]; P[l][k][2] = q3[2];
                }
            }
#pragma unroll
            for (uint32_t l = 0; l < LPRE; ++l) {
                if (l < m.n_layers) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) vertex(P[l][k][0], P[l][k][1], P[l][k][2]);
                }
            }
        } else {
            for (uint32_t l = 0; l < m.n_layers; ++l) {
                const float *lay = m.layer_pos + (size_t)l * m.n_verts * 3;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float *q3 = lay + (size_t)qi[k] * 3;
                    vertex(q3[0], q3[1], q3[2]);
                }
            }
        }
        bool keep = true;
        float L = 1.0f;
        if (n_near == 4u * m.n_layers) {
            keep = false;
        } else if (n_near == 0) {
            if (xmx < 0.0f || xmn > (float)W || ymx < 0.0f || ymn > (float)H) {
                keep = false;
            } else {
                float ex = xmx - xmn, ey = ymx - ymn;
                float diag = sqrtf(ex * ex + ey * ey);
                L = (diag / (float)H) * lambda;
                L = fmaxx(L, 0.0f);
                L = fminx(L, 1.0f);
            }
        }
        if (!keep) {
            n = 0;
        } else {
            const float delta =
                unit24(pcg(bundle_hash(seed, m.bundle_key[b]) ^ 0xA511E9B3u));
            lod_counts(L, N, delta, cmax, m.n_layers, n, cp);
        }
    }
    if (n == 0) cp = 0;
    n_out = n;
    cp_out = cp;
}

__global__ __launch_bounds__(256) void k_lod(hm_hair_mesh m, const hm_camera *cams, uint32_t W,
                                             uint32_t H, int mode, float lambda, uint32_t seed,
                                             uint32_t *table, uint64_t *cnt_s, uint64_t *cnt_c)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m.n_bundles) return;
    uint32_t n, cp;
    lod_entry(m, cams, W, H, mode, lambda, seed, b, n, cp);
    table[4 * (size_t)b + 0] = n;
    table[4 * (size_t)b + 1] = cp;
    cnt_s[b] = n;
    cnt_c[b] = (uint64_t)n * cp;
}

// scene_off[t] is the first CP of the first bundle whose scene is >= t (the
// total when there is none).  bundle_scene is non-decreasing, so bundle b
// starts the scenes t in (bundle_scene[b - 1], bundle_scene[b]] (t from 0 for
// b = 0): each bundle writes those entries from its neighbour's scene, one
// coalesced load instead of a binary search of dependent loads per scene.
// Entries stay below S + 1 for any input.
__device__ __forceinline__ void scene_starts(const uint32_t *bundle_scene, uint32_t b, uint32_t S,
                                             uint32_t off, uint32_t *scene_off)
{
    const uint32_t sb = bundle_scene[b];
    const uint32_t t0 = b == 0 ? 0u : bundle_scene[b - 1] + 1u;
    const uint32_t t1 = sb < S ? sb : S;
    for (uint32_t t = t0; t <= t1; ++t) scene_off[t] = off;
}

// Whole LOD pass in one workgroup (meshes of up to LOD_SMALL bundles): counts,
// both exclusive prefix sums, scene offsets and totals in a single launch.
constexpr uint32_t LOD_SMALL = 8192;

__global__ __launch_bounds__(1024) void k_lod_small(hm_hair_mesh m, const hm_camera *cams,
                                                    uint32_t W, uint32_t H, int mode, float lambda,
                                                    uint32_t seed, uint32_t S, uint32_t *table,
                                                    uint32_t *scene_off, uint64_t *totals)
{
    __shared__ uint64_t lds_s[1024 / 64 + 1], lds_c[1024 / 64 + 1];
    const uint32_t B = m.n_bundles;
    const uint64_t lim = 0xFFFFFFFFull;
    uint64_t carry_s = 0, carry_c = 0;
    for (uint32_t base = 0; base < B; base += blockDim.x) {
        const uint32_t b = base + threadIdx.x;
        uint32_t n = 0, cp = 0;
        if (b < B) lod_entry(m, cams, W, H, mode, lambda, seed, b, n, cp);
        uint64_t ts, tc;
        const uint64_t os = block_exclusive_scan<uint64_t>(n, lds_s, ts) + carry_s;
        const uint64_t oc = block_exclusive_scan<uint64_t>((uint64_t)n * cp, lds_c, tc) + carry_c;
        if (b < B) {
            const uint32_t oc32 = (uint32_t)(oc < lim ? oc : lim);
            table[4 * (size_t)b + 0] = n;
            table[4 * (size_t)b + 1] = cp;
            table[4 * (size_t)b + 2] = (uint32_t)(os < lim ? os : lim);
            table[4 * (size_t)b + 3] = oc32;
            scene_starts(m.bundle_scene, b, S, oc32, scene_off);
        }
        carry_s += ts;
        carry_c += tc;
    }
    // scenes after the last bundle's start at the total
    const uint32_t tot32 = (uint32_t)(carry_c < lim ? carry_c : lim);
    for (uint32_t t = m.bundle_scene[B - 1] + 1u + threadIdx.x; t <= S; t += blockDim.x)
        scene_off[t] = tot32;
    if (threadIdx.x == 0) {
        totals[0] = carry_s;
        totals[1] = carry_c;
    }
}

__global__ __launch_bounds__(256) void k_lod_finish(uint32_t *table, const uint64_t *off_s,
                                                    const uint64_t *off_c, uint32_t B,
                                                    const uint32_t *bundle_scene, uint32_t S,
                                                    uint32_t *scene_off, uint64_t *totals)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t lim = 0xFFFFFFFFull;
    if (t < B) {
        const uint32_t oc32 = (uint32_t)(off_c[t] < lim ? off_c[t] : lim);
        table[4 * (size_t)t + 2] = (uint32_t)(off_s[t] < lim ? off_s[t] : lim);
        table[4 * (size_t)t + 3] = oc32;
        scene_starts(bundle_scene, t, S, oc32, scene_off);
    }
    if (t <= S && t > bundle_scene[B - 1])       // after the last bundle's scene: the total
        scene_off[t] = (uint32_t)(off_c[B] < lim ? off_c[B] : lim);
    if (t == 0) {
        totals[0] = off_s[B];
        totals[1] = off_c[B];
    }
}

size_t lod_workspace(uint32_t B)
{
    size_t nb = scan_blocks(B) + 1;
    return 2 * align_up(sizeof(uint64_t) * ((size_t)B + 1)) + 2 * align_up(sizeof(uint64_t) * nb);
}

void launch_lod(const hm_hair_mesh &m, const hm_camera *cams, const hm_frame &f,
                const hm_lod_params &p, uint32_t *table, uint32_t *scene_off, uint64_t *totals,
                void *ws, hipStream_t st)
{
    const uint32_t B = m.n_bundles;
    if (B <= LOD_SMALL) {
        hipLaunchKernelGGL(k_lod_small, dim3(1), dim3(1024), 0, st, m, cams, f.width, f.height,
                           (int)p.mode, p.lambda, p.seed, f.n_scenes, table, scene_off, totals);
        return;
    }
    char *w = (char *)ws;
    uint64_t *cs = (uint64_t *)w;
    w += align_up(sizeof(uint64_t) * ((size_t)B + 1));
    uint64_t *cc = (uint64_t *)w;
    w += align_up(sizeof(uint64_t) * ((size_t)B + 1));
    const size_t nb = scan_blocks(B) + 1;
    uint64_t *ps = (uint64_t *)w;
    w += align_up(sizeof(uint64_t) * nb);
    uint64_t *pc = (uint64_t *)w;
    hipLaunchKernelGGL(k_lod, dim3((B + 255) / 256), dim3(256), 0, st, m, cams, f.width,
                       f.height, (int)p.mode, p.lambda, p.seed, table, cs, cc);
    scan_exclusive<uint64_t>(cs, cs, B, ps, st);
    scan_exclusive<uint64_t>(cc, cc, B, pc, st);
    const uint32_t n = (B > f.n_scenes + 1 ? B : f.n_scenes + 1);
    hipLaunchKernelGGL(k_lod_finish, dim3((n + 255) / 256), dim3(256), 0, st, table,
                       (const uint64_t *)cs, (const uint64_t *)cc, B, m.bundle_scene,
                       f.n_scenes, scene_off, totals);
}

// ------------------------------------------------------------------ generation
// Taylor polynomials of sin (degree 17) and cos (degree 16) about 0 in Horner
// form in a^2, coefficients = binary32 nearest 1/n!; argument in [-pi, pi).
__device__ __forceinline__ float tsin(float a)
{
    const float s = a * a;
    float p = 0x1.952c78p-49f;
    p = -0x1.ae7f3ep-41f + s * p;
    p = 0x1.612462p-33f + s * p;
    p = -0x1.ae6456p-26f + s * p;
    p = 0x1.71de3ap-19f + s * p;
    p = -0x1.a01a02p-13f + s * p;
    p = 0x1.111112p-7f + s * p;
    p = -0x1.555556p-3f + s * p;
    return a + (a * s) * p;
}

__device__ __forceinline__ float tcos(float a)
{
    const float s = a * a;
    float p = 0x1.ae7f3ep-45f;
    p = -0x1.93974ap-37f + s * p;
    p = 0x1.1eed8ep-29f + s * p;
    p = -0x1.27e4fcp-22f + s * p;
    p = 0x1.a01a02p-16f + s * p;
    p = -0x1.6c16c2p-10f + s * p;
    p = 0x1.555556p-5f + s * p;
    p = -0x1.0p-1f + s * p;
    return 1.0f + s * p;
}

struct F3 { float x, y, z; };

__device__ __forceinline__ F3 f3sub(F3 a, F3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ F3 f3norm(F3 a)
{
    float n2 = (a.x * a.x + a.y * a.y) + a.z * a.z;
    if (n2 > 0.0f) {
        float inv = 1.0f / sqrtf(n2);
        return {a.x * inv, a.y * inv, a.z * inv};
    }
    return {0.0f, 0.0f, 0.0f};
}
__device__ __forceinline__ F3 f3cross(F3 a, F3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ F3 ld3(const float *p) { return {p[0], p[1], p[2]}; }

// Base point of layer l at bilinear coordinates (u, v): lerp along AB and DC
// by u, then between the two by v.
__device__ __forceinline__ F3 layer_point(const float *layer_pos, uint32_t n_verts, uint32_t l,
                                          const uint32_t q[4], float u, float v)
{
    const float *L0 = layer_pos + (size_t)l * n_verts * 3;
    F3 A = ld3(L0 + 3 * (size_t)q[0]), B = ld3(L0 + 3 * (size_t)q[1]);
    F3 C = ld3(L0 + 3 * (size_t)q[2]), D = ld3(L0 + 3 * (size_t)q[3]);
    F3 ab = {A.x + u * (B.x - A.x), A.y + u * (B.y - A.y), A.z + u * (B.z - A.z)};
    F3 dc = {D.x + u * (C.x - D.x), D.y + u * (C.y - D.y), D.z + u * (C.z - D.z)};
    return {ab.x + v * (dc.x - ab.x), ab.y + v * (dc.y - ab.y), ab.z + v * (dc.z - ab.z)};
}

struct GenK {
    uint32_t seed;
    float width, curl_amp, curl_turns;
    float br, bg, bb;
};

// Cooperative assembly, one workgroup of four waves per bundle (the paper
// assigns a subgroup per strand and shares control points through shuffles;
// here the workgroup shares a bundle's strands through LDS): the strands'
// (u, v, phase), base layer points and layer tangents are computed once into
// LDS, then every lane evaluates control points (Hermite + curl) from LDS and
// stores them coalesced.  Strands are processed in chunks that fit the LDS
// budget.
constexpr uint32_t GEN_LDS_FLOATS = 4096;   // 16 KB: ten workgroups fit a CU

// Raster side of the fused generate + raster kernel.
struct FuseK {
    const hm_camera *cams;
    uint64_t *vis;        // [S][2][H][W], prefilled
    uint32_t W, H;
    float r_min;
};
constexpr uint32_t FUSE_CPS = 1024;        // screen records of strand chunks in LDS (16 KB)
constexpr uint32_t GEN_WAVES = 4;          // waves of a generation workgroup

// Orders the LDS and global accesses of the threads that share a bundle
// around a hand-off between stages: its one wave (WAVE), else the workgroup.
template <bool WAVE>
__device__ __forceinline__ void gen_sync()
{
    if (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        __syncthreads();
    }
}

// WAVE: one wave per bundle, four bundles per workgroup (each wave works in
// its own quarter of the LDS and synchronises only its own lanes, so a bundle
// left with a few short strands by the LOD does not hold a whole workgroup).
// Otherwise one workgroup per bundle: all 256 threads share its work, which
// keeps the chip busy when there are few bundles with many strands each.
// The two shapes compute the same values.  FUSED: every control point is
// also projected where it is generated (screen record in LDS, as the raster's projection
// computes it), and once a chunk of strands is complete each of its segments
// is rasterized from LDS by one thread with global atomic minima on both
// layers -- the paper's assembly-and-raster in one pass, with the same
// coverage tests, depth codes and keys as the raster call.  GB (fused only):
// the keys carry the compressed G-buffer payload, built from the points'
// unit tangents (computed in LDS from their neighbours, as the resolve does)
// and the strand's colour, and nothing of the stream is written (the paper's
// register-only assembly); strands longer than the LDS chunk recompute the
// points a segment needs.  BIN (plain stream only): every control point is
// also projected where it is generated and its screen record written, and
// once a chunk is complete each segment's tile box and accepted tiles are
// found and counted in the workgroup's LDS table (the tile raster's first
// binning pass, with the same record per unit); at the end the table is
// flushed to the tile counts and its occupied slots saved for the scatter
// pass, which walks the workgroup's span of the stream.
template <bool FUSED, bool WAVE, bool GB, bool BIN>
__global__ __launch_bounds__(256) void k_generate_bundle(hm_hair_mesh m, const uint32_t *table,
                                                        const uint32_t *strand_base,
                                                        const float *strand_rgb, GenK g,
                                                        float4 *pos_w, float4 *rgb,
                                                        uint8_t *flags, const uint32_t *scene_off,
                                                        uint32_t S, uint32_t cap, FuseK fk,
                                                        BinK bk)
{
    static_assert(!(BIN && (FUSED || GB)), "binning goes with the plain stream");
    constexpr uint32_t NB = WAVE ? GEN_WAVES : 1u;      // bundles per workgroup
    constexpr uint32_t NT = 256u / NB;                  // threads per bundle
    constexpr uint32_t SM_FLOATS = GEN_LDS_FLOATS / NB, PR_CPS = FUSE_CPS / NB;
    __shared__ float sm_all[GEN_LDS_FLOATS];
    __shared__ float4 pr_all[FUSED || BIN ? FUSE_CPS : GEN_WAVES];
    __shared__ float4 tn_all[GB ? FUSE_CPS : 1];        // world points, then unit tangents
    __shared__ uint32_t bkeys[BIN ? BIN_SLOTS : 1], bcnt[BIN ? BIN_SLOTS : 1];
    __shared__ uint32_t bsave;
    if (BIN) {
        // the workgroup's (segment, tile) table
        for (uint32_t x = threadIdx.x; x < BIN_SLOTS; x += blockDim.x) {
            bkeys[x] = BIN_FREE;
            bcnt[x] = 0u;
        }
        if (threadIdx.x == 0) bsave = 0u;
        __syncthreads();
    }
    const uint32_t wv = WAVE ? threadIdx.x >> 6 : 0u;
    const uint32_t lane = WAVE ? threadIdx.x & 63u : threadIdx.x;
    const uint32_t b = blockIdx.x * NB + wv;
    // one bundle's work (a return leaves the bundle, not the workgroup)
    auto bundle = [&]() {
        if (b >= m.n_bundles) return;                  // the whole wave / workgroup
        float *sm = sm_all + wv * SM_FLOATS;
        float4 *pr = pr_all + (FUSED || BIN ? wv * PR_CPS : 0u);
        float4 *tn = tn_all + (GB ? wv * PR_CPS : 0u);
        const uint4 tb = reinterpret_cast<const uint4 *>(table)[b];
        const uint32_t n = tb.x, C = tb.y, cp0 = tb.w;
        if (n == 0) return;
        const uint32_t total = scene_off[S];
        const uint32_t limit = total < cap ? total : cap;
        const uint32_t NL = m.n_layers;
        const uint32_t stride = 6u * NL + 3u;                 // P[L], T[L], u, v, phase
        uint32_t chunk = SM_FLOATS / stride;     // >= 2 (WAVE) / 10 strands for L <= 64
        // screen records of a chunk stay in LDS when a strand fits (C <= 256
        // (WAVE) / 1024); longer strands are projected again from the stream
        // they were just written to (same bits, no LDS limit)
        const bool in_lds = C <= PR_CPS;
        if ((FUSED || BIN) && in_lds) chunk = min(chunk, PR_CPS / C);   // >= 2 strands for C <= 127
        Cam cam;
        uint32_t sc = 0;
        if (FUSED || BIN) {
            sc = m.bundle_scene[b];
            cam = load_cam((FUSED ? fk.cams : bk.cams) + sc);
        }
        const uint4 q4 = reinterpret_cast<const uint4 *>(m.quads)[b];
        const uint32_t q[4] = {q4.x, q4.y, q4.z, q4.w};
        const uint32_t hb = bundle_hash(g.seed, m.bundle_key[b]);

        // bundle styling frame from the first layer interval
        F3 s0 = {0.0f, 0.0f, 0.0f};
    #pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            const F3 a0 = ld3(m.layer_pos + 3 * (size_t)q[k2]);
            const F3 a1 = ld3(m.layer_pos + ((size_t)m.n_verts + q[k2]) * 3);
            const F3 d = f3sub(a1, a0);
            s0.x = s0.x + d.x; s0.y = s0.y + d.y; s0.z = s0.z + d.z;
        }
        const F3 nb = f3norm(s0);
        F3 ax = {0.0f, 0.0f, 1.0f};
        if (fabsf(nb.z) > 0.9f) { ax.x = 1.0f; ax.z = 0.0f; }
        const F3 e1 = f3norm(f3cross(nb, ax));
        const F3 e2 = f3cross(nb, e1);

        for (uint32_t k0 = 0; k0 < n; k0 += chunk) {
            const uint32_t nk = (n - k0) < chunk ? (n - k0) : chunk;
            // base layer points; the strand's (u, v) and curl phase come from its
            // hash, recomputed by each of its layers' threads (no separate stage)
            for (uint32_t x = lane; x < nk * NL; x += NT) {
                const uint32_t kk = x / NL, l = x - kk * NL;
                float *o = sm + kk * stride;
                const uint32_t h1 = pcg(hb + (k0 + kk));
                const uint32_t h2 = pcg(h1);
                const float u = unit24(h1), v = unit24(h2);
                if (l == 0) {
                    o[6u * NL] = u;
                    o[6u * NL + 1] = v;
                    o[6u * NL + 2] = unit24(pcg(h2));
                }
                const F3 P = layer_point(m.layer_pos, m.n_verts, l, q, u, v);
                o[6 * l + 0] = P.x; o[6 * l + 1] = P.y; o[6 * l + 2] = P.z;
            }
            gen_sync<WAVE>();
            // finite-difference layer tangents
            for (uint32_t x = lane; x < nk * NL; x += NT) {
                const uint32_t kk = x / NL, l = x - kk * NL;
                float *o = sm + kk * stride;
                const uint32_t la = l == 0 ? 1u : (l == NL - 1 ? l : l + 1);
                const uint32_t lb = l == 0 ? 0u : l - 1;
                const F3 T = f3norm(f3sub(ld3(o + 6 * la), ld3(o + 6 * lb)));
                o[6 * l + 3] = T.x; o[6 * l + 4] = T.y; o[6 * l + 5] = T.z;
            }
            gen_sync<WAVE>();
            // styled control point j of chunk strand kk: chord-scaled Hermite
            // between the layer points, then the curl about the bundle axis
            auto styled_cp = [&](uint32_t kk, uint32_t j) -> float4 {
                const float *o = sm + kk * stride;
                const float w = (float)j / (float)(C - 1u);
                const float x = w * (float)(NL - 1u);
                int i = (int)x;
                i = i > (int)NL - 2 ? (int)NL - 2 : i;
                const float t = x - (float)i;
                const F3 Pi = ld3(o + 6 * i), Pj = ld3(o + 6 * (i + 1));
                const F3 Ti = ld3(o + 6 * i + 3), Tj = ld3(o + 6 * (i + 1) + 3);
                const F3 ch = f3sub(Pj, Pi);
                const float chord = sqrtf((ch.x * ch.x + ch.y * ch.y) + ch.z * ch.z);
                const float t2 = t * t, t3 = t2 * t;
                const float h00 = (2.0f * t3 - 3.0f * t2) + 1.0f;
                const float h10 = (t3 - 2.0f * t2) + t;
                const float h01 = 3.0f * t2 - 2.0f * t3;
                const float h11 = t3 - t2;
                const float pi3[3] = {Pi.x, Pi.y, Pi.z}, pj3[3] = {Pj.x, Pj.y, Pj.z};
                const float ti3[3] = {Ti.x, Ti.y, Ti.z}, tj3[3] = {Tj.x, Tj.y, Tj.z};
                float X[3];
    #pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const float m0 = chord * ti3[d], m1 = chord * tj3[d];
                    X[d] = ((h00 * pi3[d] + h10 * m0) + h01 * pj3[d]) + h11 * m1;
                }
                float f = g.curl_turns * w + o[6u * NL + 2];
                f = f - floorf(f);
                const float a = (f - 0.5f) * 0x1.921fb6p+2f;
                const float cth = -tcos(a), sth = -tsin(a);
                const float amp = g.curl_amp * w;
                float4 pw;
                pw.x = X[0] + amp * (cth * e1.x + sth * e2.x);
                pw.y = X[1] + amp * (cth * e1.y + sth * e2.y);
                pw.z = X[2] + amp * (cth * e1.z + sth * e2.z);
                pw.w = g.width;
                return pw;
            };
            auto strand_col = [&](uint32_t kk) -> float4 {
                if (strand_rgb) {
                    const float *sr = strand_rgb + 3 * ((size_t)strand_base[b] + k0 + kk);
                    return make_float4(sr[0], sr[1], sr[2], 1.0f);
                }
                return make_float4(g.br, g.bg, g.bb, 1.0f);
            };
            // control points of strands k0 .. k0+nk-1 (contiguous in the stream)
            for (uint32_t r = lane; r < nk * C; r += NT) {
                const uint32_t kk = r / C, j = r - kk * C;
                const uint32_t c = cp0 + (k0 + kk) * C + j;
                if (c >= limit) continue;
                const float4 pw = styled_cp(kk, j);
                if (GB) {
                    if (in_lds) tn[r] = pw;
                    continue;
                }
                pos_w[c] = pw;
                if (FUSED && in_lds) pr[r] = project(cam, pw);
                if (BIN) {
                    // the point's screen record, as the binning pass projects it
                    const float4 a = project(cam, pw);
                    bk.proj[c] = a;
                    if (in_lds) pr[r] = a;
                }
                rgb[c] = strand_col(kk);
                uint8_t fl = 0;
                if (j == 0) fl |= (uint8_t)HM_ROOT;
                // the last CP of a stream truncated to the capacity ends its strand
                if (j == C - 1u || c == limit - 1u) fl |= (uint8_t)HM_TIP;
                flags[c] = fl;
            }
            if (GB && in_lds) {
                // screen records and unit tangents of the chunk's points (the
                // tangents replace the world points once every lane has read its
                // neighbours)
                // a chunk holds at most PR_CPS = 4 NT points: four per lane
                static_assert(PR_CPS == 4u * NT, "four chunk points per lane");
                gen_sync<WAVE>();
                float4 tr[4];
    #pragma unroll
                for (uint32_t it = 0; it < 4u; ++it) {
                    const uint32_t r = lane + it * NT;
                    const uint32_t kk = r / C, j = r - kk * C;
                    const uint32_t c = cp0 + (k0 + kk) * C + j;
                    tr[it] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (r >= nk * C || c >= limit) continue;
                    const float4 P = tn[r];
                    pr[r] = project(cam, P);
                    const bool root = j == 0, tip = j == C - 1u || c == limit - 1u;
                    tr[it] = cp_unit_tangent(root ? P : tn[r - 1], tip ? P : tn[r + 1], root && tip);
                }
                gen_sync<WAVE>();
    #pragma unroll
                for (uint32_t it = 0; it < 4u; ++it) {
                    const uint32_t r = lane + it * NT;
                    const uint32_t kk = r / C, j = r - kk * C;
                    if (r < nk * C && cp0 + (k0 + kk) * C + j < limit) tn[r] = tr[it];
                }
            }
            gen_sync<WAVE>();
            if (FUSED) {
                // segments of the chunk: CP j of strand kk joins j + 1 unless j
                // is a tip (last CP of its strand, or of a truncated stream)
                const size_t hw = (size_t)fk.W * fk.H;
                uint64_t *vc = fk.vis + (size_t)sc * 2 * hw, *va = vc + hw;
                const float zn = cam.zn, inv_range = 1.0f / (cam.zf - zn);
                for (uint32_t r = lane; r < nk * C; r += NT) {
                    const uint32_t kk = r / C, j = r - kk * C;
                    const uint32_t c = cp0 + (k0 + kk) * C + j;
                    if (j + 1u >= C || c + 1u >= limit) continue;
                    float4 pa, pb, T0, T1;
                    if (in_lds) {
                        pa = pr[r];
                        pb = pr[r + 1];
                        if (GB) {
                            T0 = tn[r];
                            T1 = tn[r + 1];
                        }
                    } else if (GB) {
                        // no stream to read back: the segment's points again
                        const float4 P0 = styled_cp(kk, j), P1 = styled_cp(kk, j + 1u);
                        const bool root = j == 0, tip1 = j + 2u >= C || c + 2u >= limit;
                        const float4 Pm = root ? P0 : styled_cp(kk, j - 1u);
                        const float4 P2 = tip1 ? P1 : styled_cp(kk, j + 2u);
                        pa = project(cam, P0);
                        pb = project(cam, P1);
                        T0 = cp_unit_tangent(Pm, P1, false);
                        T1 = cp_unit_tangent(P0, P2, false);
                    } else {
                        pa = project(cam, pos_w[c]);
                        pb = project(cam, pos_w[c + 1]);
                    }
                    if (pa.w == 0.0f || pb.w == 0.0f) continue;
                    const Seg sg = make_seg(pa, pb, fk.r_min);
                    const float4 col = GB ? strand_col(kk) : make_float4(0.f, 0.f, 0.f, 0.f);
                    int i0, i1, j0, j1;
                    if (!seg_box(sg, fk.W, fk.H, i0, i1, j0, j1)) continue;
                    for (int y = j0; y <= j1; ++y) {
                        int a0, a1;
                        row_span(sg, y, a0, a1);
                        a0 = a0 > i0 ? a0 : i0;
                        a1 = a1 < i1 ? a1 : i1;
                        for (int x = a0; x <= a1; ++x) {
                            uint32_t q;
                            bool cc, ca;
                            float ts, z;
                            if (!cover_tz(sg, x, y, fk.r_min, zn, inv_range, cc, ca, q, ts, z))
                                continue;
                            const uint64_t low =
                                GB ? gb_payload_of(T0, T1, col, col, ts, z, pb.w) : (uint64_t)c;
                            const unsigned long long key = ((unsigned long long)q << HM_ID_BITS) | low;
                            const size_t px = (size_t)y * fk.W + x;
                            if (cc) atomicMin((unsigned long long *)(vc + px), key);
                            if (ca) atomicMin((unsigned long long *)(va + px), key);
                        }
                    }
                }
                // pr is rewritten only after the next chunk's two barriers
            }
            if (BIN) {
                // each control point's unit: the tile box and tiles of the
                // segment it starts (none for a tip), counted in the table
                for (uint32_t r = lane; r < nk * C; r += NT) {
                    const uint32_t kk = r / C, j = r - kk * C;
                    const uint32_t c = cp0 + (k0 + kk) * C + j;
                    if (c >= limit) continue;
                    SegTiles st;
                    st.nt = 0;
                    bool ok = false;
                    if (j + 1u < C && c + 1u < limit) {
                        float4 pa, pb;
                        if (in_lds) {
                            pa = pr[r];
                            pb = pr[r + 1];
                        } else {
                            pa = project(cam, pos_w[c]);
                            pb = project(cam, pos_w[c + 1]);
                        }
                        ok = seg_tiles_of(pa, pb, sc, bk.rk, st);
                    }
                    bk.segrec[c] = bin_count(st, ok, c, bk.rk, bk.kmax, bkeys, bcnt, bk.tile_cnt,
                                             bk.long_list, bk.counters);
                }
            }
        }
    };
    bundle();
    if (BIN) {
        // flush the table: one global add per (workgroup, tile), and save
        // its occupied slots (slot, tile, count) for the scatter pass
        __syncthreads();
        uint32_t *sv = bk.saved + (size_t)blockIdx.x * BIN_SAVE_WORDS;
        for (uint32_t x = threadIdx.x; x < BIN_SLOTS; x += blockDim.x) {
            const uint32_t t = bkeys[x];
            if (t == BIN_FREE) continue;
            const uint32_t c = bcnt[x];
            atomicAdd(&bk.tile_cnt[t], c);
            const uint32_t i = atomicAdd(&bsave, 1u);
            sv[1 + 3 * i] = x;
            sv[2 + 3 * i] = t;
            sv[3 + 3 * i] = c;
        }
        __syncthreads();
        if (threadIdx.x == 0) sv[0] = bsave;
    }
}

// Launch shape of the generator: one wave per bundle when the bundles alone
// give every SIMD of the chip (256 CUs x 4) several waves, or when a bundle
// at full detail averages at most two control points per thread of a
// workgroup (a workgroup would idle); otherwise one workgroup per bundle.
// cap bounds the stream, so cap / n_bundles bounds the average bundle.
static bool gen_wave(uint32_t n_bundles, uint32_t cap)
{
    return n_bundles >= 4096u || (uint64_t)cap <= 512ull * n_bundles;
}

uint32_t gen_bundles_per_group(uint32_t n_bundles, uint32_t cap)
{
    return gen_wave(n_bundles, cap) ? GEN_WAVES : 1u;
}

uint32_t gen_grid(uint32_t n_bundles, uint32_t cap)
{
    const uint32_t nb = gen_bundles_per_group(n_bundles, cap);
    return (n_bundles + nb - 1) / nb;
}

template <bool FUSED, bool GB, bool BIN = false>
static void launch_gen_kernel(const hm_hair_mesh &m, const uint32_t *table,
                              const uint32_t *strand_base, const float *strand_rgb, GenK g,
                              const hm_strands &s, FuseK fk, hipStream_t st,
                              BinK bk = BinK{})
{
    const bool wave = gen_wave(m.n_bundles, s.cap);
    const uint32_t grid = gen_grid(m.n_bundles, s.cap);
#define HM_GEN_LAUNCH(W)                                                                    \
    hipLaunchKernelGGL((k_generate_bundle<FUSED, W, GB, BIN>), dim3(grid), dim3(256), 0, st,  \
                       m, table,                                                             \
                       strand_base, strand_rgb, g, reinterpret_cast<float4 *>(s.pos_w),        \
                       reinterpret_cast<float4 *>(s.rgb), s.flags, s.scene_off, s.n_scenes,    \
                       s.cap, fk, bk)
    if (wave)
        HM_GEN_LAUNCH(true);
    else
        HM_GEN_LAUNCH(false);
#undef HM_GEN_LAUNCH
}

void launch_generate(const hm_hair_mesh &m, const uint32_t *table, const uint32_t *strand_base,
                     const float *strand_rgb, const hm_gen_params &p, const hm_strands &s,
                     hipStream_t st)
{
    GenK g{p.seed, p.width, p.curl_amp, p.curl_turns, p.base_rgb[0], p.base_rgb[1],
           p.base_rgb[2]};
    launch_gen_kernel<false, false>(m, table, strand_base, strand_rgb, g, s,
                                    FuseK{nullptr, nullptr, 0u, 0u, 0.0f}, st);
}

void launch_generate_raster(const hm_hair_mesh &m, const uint32_t *table,
                            const uint32_t *strand_base, const float *strand_rgb,
                            const hm_gen_params &p, const hm_strands &s, const hm_camera *cams,
                            const hm_frame &f, float r_min, int payload, const float *scene_z,
                            uint64_t *vis, hipStream_t st)
{
    launch_prefill(vis, scene_z, cams, f, st);
    GenK g{p.seed, p.width, p.curl_amp, p.curl_turns, p.base_rgb[0], p.base_rgb[1],
           p.base_rgb[2]};
    const FuseK fk{cams, vis, f.width, f.height, r_min};
    if (payload == HM_PAYLOAD_GBUFFER)
        launch_gen_kernel<true, true>(m, table, strand_base, strand_rgb, g, s, fk, st);
    else
        launch_gen_kernel<true, false>(m, table, strand_base, strand_rgb, g, s, fk, st);
}

void launch_generate_bin(const hm_hair_mesh &m, const uint32_t *table, const uint32_t *strand_base,
                         const float *strand_rgb, const hm_gen_params &p, const hm_strands &s,
                         const BinK &bk, hipStream_t st)
{
    GenK g{p.seed, p.width, p.curl_amp, p.curl_turns, p.base_rgb[0], p.base_rgb[1],
           p.base_rgb[2]};
    launch_gen_kernel<false, false, true>(m, table, strand_base, strand_rgb, g, s,
                                          FuseK{nullptr, nullptr, 0u, 0u, 0.0f}, st, bk);
}

}  // namespace hm

namespace hm {

// Depth correction of the LOD (Beer-Lambert): delta = -log(N_LOD / N_b).
__global__ __launch_bounds__(256) void k_lod_delta(const uint32_t *table, const uint32_t *nstr,
                                                   uint32_t B, float *delta)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const uint32_t n = table[4 * (size_t)b], N = nstr[b];
    float d = 0.0f;
    if (N > 0) d = n == 0 ? INFINITY : -logf((float)n / (float)N);
    delta[b] = d;
}

void launch_lod_delta(const uint32_t *table, const uint32_t *nstr, uint32_t B, float *delta,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_lod_delta, dim3((B + 255) / 256), dim3(256), 0, st, table, nstr, B,
                       delta);
}

}  // namespace hm
