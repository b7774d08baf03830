/*
 * hm_oracle.c -- plain, slow, single-threaded CPU oracle for deferred software
 * rasterization of strand hair (Lipp, Jarabo, Wimmer, Bode: "Deferred Software
 * Rasterization for Efficient Real-time Hair Rendering").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it is used by the test-suite, by the smoke check and by the
 * benchmark's CPU-baseline leg.  It shares no source with the HIP library.
 *
 * Precision contract.
 *   - Steps whose floating-point results decide integers (strand hash -> uv,
 *     LOD counts, strand generation, projection, the two coverage predicates,
 *     the 24-bit depth code, and the reconstruction filter's strip / depth
 *     decisions) are evaluated in binary32 with the operation order written
 *     below; this file must be compiled with -ffp-contract=off and without
 *     fast-math, so every operation is one correctly rounded IEEE op.
 *   - Continuous outputs (shading, filter weights, colours, composite) are
 *     evaluated in binary64 from the binary32 inputs.
 *
 * Conventions (all arrays row-major, caller-owned host memory):
 *   camera record (18 float): R[9] rows = camera right/up/forward, eye[3],
 *     fx, fy, cx, cy, znear, zfar.  Camera space: +z forward, +y up; pixel
 *     x = cx + fx*X/Z, y = cy - fy*Y/Z; pixel (i,j) has its centre at
 *     (i+0.5, j+0.5).
 *   strand stream: pos_w[n_cp][4] = (x, y, z, width), rgb[n_cp][4] =
 *     (r, g, b, ao), flags[n_cp] bit0 = root CP, bit1 = tip CP.
 *   LOD table [B][4] u32 = {strands, control points per strand, first strand,
 *     first control point} -- one uint4 per bundle as in Sec. 3.2.2.
 *   visibility [S][2][H][W] u64: layer 0 = centre sample, layer 1 =
 *     conservative; key = depth24 << 40 | segment id (the CP index of the
 *     segment's first endpoint); empty = all ones; opaque scene depth uses the
 *     id 2^40 - 2.
 *
 * Parity unpinned: the exact output bits of orc_pcg (the published PCG hash,
 *   pinned only by bijectivity, avalanche and uniformity) and the curl styling
 *   of orc_generate (the paper leaves the styling function unstated; pinned as
 *   a helix of the stated radius and phase).  Every other function is pinned
 *   by the tests/test_oracle_*.py checks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EMPTY 0xFFFFFFFFFFFFFFFFull
#define ORC_ID_BITS 40
#define ORC_ID_MASK ((1ull << ORC_ID_BITS) - 1ull)
#define ORC_ID_OPAQUE ((1ull << ORC_ID_BITS) - 2ull)
#define ORC_QMAX 16777215u
#define ORC_ROOT 1u
#define ORC_TIP 2u

typedef struct {
    float R[9];
    float eye[3];
    float fx, fy, cx, cy, znear, zfar;
} orc_cam;

/* Threads of the raster's segment loop and of the resolve's pixel rows (1 =
 * the plain sequential loops).  Neither result depends on it: the resolve's
 * pixels are independent, and the raster keeps each pixel's minimum with a
 * compare-and-swap, so the order in which threads meet a pixel is invisible. */
static int orc_nthreads = 1;
void orc_set_threads(int n) { orc_nthreads = n > 1 ? n : 1; }
int orc_get_threads(void) { return orc_nthreads; }

/* ------------------------------------------------------------------ hashing
 * Per-strand uv "from a PCG generator seeded by the strand index" (Sec. 3.1.1,
 * Code 1).  The PCG hash of Jarzynski and Olano (JCGT 2020, "Hash functions
 * for GPU rendering"): one LCG step followed by the PCG-RXS-M-XS output
 * permutation. */
uint32_t orc_pcg(uint32_t v)
{
    uint32_t s = v * 747796405u + 2891336453u;
    uint32_t w = ((s >> ((s >> 28u) + 4u)) ^ s) * 277803737u;
    return (w >> 22u) ^ w;
}

static float orc_unit24(uint32_t h) { return (float)(h >> 8) * 0x1p-24f; }

uint32_t orc_bundle_hash(uint32_t seed, uint32_t key) { return orc_pcg(orc_pcg(seed) ^ key); }

/* (u, v, curl phase) of strand k of the bundle with hash key `key`. */
void orc_strand_rand(uint32_t seed, uint32_t key, uint32_t k, float out[3])
{
    uint32_t h1 = orc_pcg(orc_bundle_hash(seed, key) + k);
    uint32_t h2 = orc_pcg(h1);
    uint32_t h3 = orc_pcg(h2);
    out[0] = orc_unit24(h1);
    out[1] = orc_unit24(h2);
    out[2] = orc_unit24(h3);
}

/* Per-bundle stochastic offset delta ~ U[0,1) of eq. (strand-lod). */
float orc_lod_delta(uint32_t seed, uint32_t key)
{
    return orc_unit24(orc_pcg(orc_bundle_hash(seed, key) ^ 0xA511E9B3u));
}

/* ------------------------------------------------------------ LOD (Sec. 3.2) */

/* Strand count (eq. strand-lod) and control-point count (eqs. cp-lod, cp-snap)
 * for LOD value L.  floor(log2(x)) is taken by repeated doubling so the
 * definition can be read directly. */
void orc_lod_counts(float L, uint32_t N, float delta, uint32_t cmax, uint32_t n_layers,
                    uint32_t *n_lod, uint32_t *cps)
{
    int n = (int)ceilf(L * ((float)N + delta));
    if (n < 1) n = 1;
    if (n > (int)N) n = (int)N;
    *n_lod = (uint32_t)n;

    int craw = (int)floorf(sqrtf(L) * (float)cmax);
    if (craw < (int)n_layers) craw = (int)n_layers;
    uint32_t p = 1;                       /* 2^floor(log2(craw - 1)) */
    while (2u * p <= (uint32_t)(craw - 1)) p *= 2u;
    uint32_t c = p + 1u;
    if (c > cmax) c = cmax;
    *cps = c;
}

/* LOD value of one bundle: projected AABB over all layers and corners
 * (the AABB equation and eq. lod-factor).  Returns 0 if the bundle is culled
 * (AABB outside the viewport, or every vertex at or behind the near plane),
 * else 1 and *L. */
int orc_lod_value(const orc_cam *c, int width, int height, float lambda,
                  const float *layer_pos, uint32_t n_layers, uint32_t n_verts,
                  const uint32_t quad[4], float *L)
{
    float xmn = INFINITY, xmx = -INFINITY, ymn = INFINITY, ymx = -INFINITY;
    uint32_t n_near = 0;
    for (uint32_t l = 0; l < n_layers; ++l) {
        for (int q = 0; q < 4; ++q) {
            const float *P = layer_pos + ((size_t)l * n_verts + quad[q]) * 3;
            float dx = P[0] - c->eye[0], dy = P[1] - c->eye[1], dz = P[2] - c->eye[2];
            float X = (c->R[0] * dx + c->R[1] * dy) + c->R[2] * dz;
            float Y = (c->R[3] * dx + c->R[4] * dy) + c->R[5] * dz;
            float Z = (c->R[6] * dx + c->R[7] * dy) + c->R[8] * dz;
            if (Z <= c->znear) { n_near++; continue; }
            float iz = 1.0f / Z;
            float x = c->cx + c->fx * (X * iz);
            float y = c->cy - c->fy * (Y * iz);
            xmn = x < xmn ? x : xmn;
            xmx = x > xmx ? x : xmx;
            ymn = y < ymn ? y : ymn;
            ymx = y > ymx ? y : ymx;
        }
    }
    if (n_near == 4u * n_layers) return 0;
    if (n_near > 0) { *L = 1.0f; return 1; }
    if (xmx < 0.0f || xmn > (float)width || ymx < 0.0f || ymn > (float)height) return 0;
    float ex = xmx - xmn, ey = ymx - ymn;
    float diag = sqrtf(ex * ex + ey * ey);
    float v = (diag / (float)height) * lambda;
    v = v < 0.0f ? 0.0f : v;
    v = v > 1.0f ? 1.0f : v;
    *L = v;
    return 1;
}

/* Per-bundle table + exclusive prefix sums.  mode 0 = LOD off (N_b strands,
 * C = cmax_b control points, no culling); mode 1 = Sec. 3.2 LOD.
 * scene_off[S+1] receives the first control point of every scene (bundles
 * must be sorted by scene).  Returns 0, or -1 if a count overflows 32 bits. */
int orc_lod_select(const float *layer_pos, const uint32_t *quads, uint32_t n_bundles,
                   uint32_t n_layers, uint32_t n_verts, const uint32_t *bundle_key,
                   const uint32_t *bundle_nstrands, const uint32_t *bundle_cmax,
                   const uint32_t *bundle_scene, const float *cams, uint32_t n_scenes,
                   int width, int height, int mode, float lambda, uint32_t seed,
                   uint32_t *table, uint32_t *scene_off, uint64_t *totals)
{
    uint64_t s_off = 0, c_off = 0;
    for (uint32_t b = 0; b < n_bundles; ++b) {
        /* a strand has at least one segment: fewer than two control points per
         * strand are taken as two */
        uint32_t N = bundle_nstrands[b], cmax = bundle_cmax[b] < 2u ? 2u : bundle_cmax[b];
        uint32_t n = N, cp = cmax;
        if (mode == 1 && N > 0) {
            const orc_cam *c = (const orc_cam *)(cams + 18 * (size_t)bundle_scene[b]);
            float L = 0.0f;
            if (!orc_lod_value(c, width, height, lambda, layer_pos, n_layers, n_verts,
                               quads + 4 * (size_t)b, &L)) {
                n = 0;
                cp = 0;
            } else {
                orc_lod_counts(L, N, orc_lod_delta(seed, bundle_key[b]), cmax, n_layers, &n, &cp);
            }
        }
        if (n == 0) cp = 0;
        if (s_off > 0xFFFFFFFFull || c_off > 0xFFFFFFFFull) return -1;
        table[4 * (size_t)b + 0] = n;
        table[4 * (size_t)b + 1] = cp;
        table[4 * (size_t)b + 2] = (uint32_t)s_off;
        table[4 * (size_t)b + 3] = (uint32_t)c_off;
        s_off += n;
        c_off += (uint64_t)n * cp;
    }
    if (c_off >= 0xFFFFFFFFull) return -1;
    totals[0] = s_off;
    totals[1] = c_off;
    for (uint32_t s = 0; s <= n_scenes; ++s) {
        uint32_t off = (uint32_t)c_off;
        for (uint32_t b = 0; b < n_bundles; ++b)
            if (bundle_scene[b] >= s) { off = table[4 * (size_t)b + 3]; break; }
        scene_off[s] = off;
    }
    return 0;
}

/* ------------------------------------------------- strand generation (Sec. 3.1.1)
 * Taylor polynomials of sine (degree 17) and cosine (degree 16) about 0,
 * Horner form in a^2; coefficients are the binary32 values nearest 1/n!.
 * Valid on the reduced range [-pi, pi). */
static float orc_sin(float a)
{
    float s = a * a;
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

static float orc_cos(float a)
{
    float s = a * a;
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

float orc_sin_export(float a) { return orc_sin(a); }
float orc_cos_export(float a) { return orc_cos(a); }

typedef struct { float x, y, z; } v3f;

static v3f v3_sub(v3f a, v3f b) { v3f r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static v3f v3_lerp(v3f a, v3f b, float t)
{
    v3f r = {a.x + t * (b.x - a.x), a.y + t * (b.y - a.y), a.z + t * (b.z - a.z)};
    return r;
}
static v3f v3_norm(v3f a)
{
    float n2 = (a.x * a.x + a.y * a.y) + a.z * a.z;
    v3f r = {0.0f, 0.0f, 0.0f};
    if (n2 > 0.0f) {
        float inv = 1.0f / sqrtf(n2);
        r.x = a.x * inv; r.y = a.y * inv; r.z = a.z * inv;
    }
    return r;
}
static v3f v3_cross(v3f a, v3f b)
{
    v3f r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
static v3f v3_load(const float *p) { v3f r = {p[0], p[1], p[2]}; return r; }

/* Generate the styled control points of strand k of bundle b.  Returns the
 * number of control points written at out index base. */
static void orc_gen_strand(const float *layer_pos, const uint32_t *quad, uint32_t n_layers,
                           uint32_t n_verts, uint32_t seed, uint32_t key, uint32_t k,
                           uint32_t C, float width, float curl_amp, float curl_turns,
                           const float rgb_s[3], float *pos_w, float *rgb, uint8_t *flags)
{
    float r3[3];
    orc_strand_rand(seed, key, k, r3);
    float u = r3[0], v = r3[1], ph = r3[2];
    v3f P[64], T[64];   /* n_layers <= 64 checked by the caller */

    /* base layer points: bilinear interpolation of each layer quad at (u, v) */
    for (uint32_t l = 0; l < n_layers; ++l) {
        const float *L0 = layer_pos + (size_t)l * n_verts * 3;
        v3f A = v3_load(L0 + 3 * (size_t)quad[0]), B = v3_load(L0 + 3 * (size_t)quad[1]);
        v3f Cq = v3_load(L0 + 3 * (size_t)quad[2]), D = v3_load(L0 + 3 * (size_t)quad[3]);
        v3f ab = v3_lerp(A, B, u), dc = v3_lerp(D, Cq, u);
        P[l] = v3_lerp(ab, dc, v);
    }
    /* finite-difference tangents (calcTangent of Code 1) */
    for (uint32_t l = 0; l < n_layers; ++l) {
        v3f d;
        if (l == 0) d = v3_sub(P[1], P[0]);
        else if (l == n_layers - 1) d = v3_sub(P[l], P[l - 1]);
        else d = v3_sub(P[l + 1], P[l - 1]);
        T[l] = v3_norm(d);
    }
    /* styling frame of the bundle: axis along the first layer interval */
    v3f s0 = {0, 0, 0};
    for (int q = 0; q < 4; ++q) {
        v3f a0 = v3_load(layer_pos + 3 * (size_t)quad[q]);
        v3f a1 = v3_load(layer_pos + ((size_t)n_verts + quad[q]) * 3);
        v3f d = v3_sub(a1, a0);
        s0.x = s0.x + d.x; s0.y = s0.y + d.y; s0.z = s0.z + d.z;
    }
    v3f nb = v3_norm(s0);
    v3f ax = {0.0f, 0.0f, 1.0f};
    if (fabsf(nb.z) > 0.9f) { ax.x = 1.0f; ax.z = 0.0f; }
    v3f e1 = v3_norm(v3_cross(nb, ax));
    v3f e2 = v3_cross(nb, e1);

    for (uint32_t j = 0; j < C; ++j) {
        float w = (float)j / (float)(C - 1u);
        float x = w * (float)(n_layers - 1u);
        int i = (int)x;
        if (i > (int)n_layers - 2) i = (int)n_layers - 2;
        float t = x - (float)i;
        v3f ch = v3_sub(P[i + 1], P[i]);
        float chord = sqrtf((ch.x * ch.x + ch.y * ch.y) + ch.z * ch.z);
        float t2 = t * t, t3 = t2 * t;
        /* cubic Hermite basis */
        float h00 = (2.0f * t3 - 3.0f * t2) + 1.0f;
        float h10 = (t3 - 2.0f * t2) + t;
        float h01 = 3.0f * t2 - 2.0f * t3;
        float h11 = t3 - t2;
        float Xb[3];
        const float *pa = &P[i].x, *pb = &P[i + 1].x, *ta = &T[i].x, *tb = &T[i + 1].x;
        for (int c = 0; c < 3; ++c) {
            float m0 = chord * ta[c], m1 = chord * tb[c];
            Xb[c] = ((h00 * pa[c] + h10 * m0) + h01 * pb[c]) + h11 * m1;
        }
        /* styling f(x): sinusoidal curl around the bundle axis, growing with w */
        float f = curl_turns * w + ph;
        f = f - floorf(f);
        float a = (f - 0.5f) * 0x1.921fb6p+2f;
        float cth = -orc_cos(a), sth = -orc_sin(a);
        float amp = curl_amp * w;
        const float *E1 = &e1.x, *E2 = &e2.x;
        float *o = pos_w + 4 * (size_t)j;
        for (int c = 0; c < 3; ++c) o[c] = Xb[c] + amp * (cth * E1[c] + sth * E2[c]);
        o[3] = width;
        float *oc = rgb + 4 * (size_t)j;
        oc[0] = rgb_s[0]; oc[1] = rgb_s[1]; oc[2] = rgb_s[2]; oc[3] = 1.0f;
        uint8_t fl = 0;
        if (j == 0) fl |= ORC_ROOT;
        if (j == C - 1u) fl |= ORC_TIP;
        flags[j] = fl;
    }
}

int orc_generate(const float *layer_pos, const uint32_t *quads, uint32_t n_bundles,
                 uint32_t n_layers, uint32_t n_verts, const uint32_t *bundle_key,
                 const uint32_t *table, const uint32_t *strand_base, const float *strand_rgb,
                 uint32_t seed, float width, float curl_amp, float curl_turns,
                 const float base_rgb[3], float *pos_w, float *rgb, uint8_t *flags)
{
    if (n_layers < 2 || n_layers > 64) return -1;
    for (uint32_t b = 0; b < n_bundles; ++b) {
        uint32_t n = table[4 * (size_t)b], C = table[4 * (size_t)b + 1];
        uint64_t cp0 = table[4 * (size_t)b + 3];
        for (uint32_t k = 0; k < n; ++k) {
            float rs[3] = {base_rgb[0], base_rgb[1], base_rgb[2]};
            if (strand_rgb) {
                const float *sr = strand_rgb + 3 * ((size_t)strand_base[b] + k);
                rs[0] = sr[0]; rs[1] = sr[1]; rs[2] = sr[2];
            }
            uint64_t o = cp0 + (uint64_t)k * C;
            orc_gen_strand(layer_pos, quads + 4 * (size_t)b, n_layers, n_verts, seed,
                           bundle_key[b], k, C, width, curl_amp, curl_turns, rs,
                           pos_w + 4 * o, rgb + 4 * o, flags + o);
        }
    }
    return 0;
}

/* ------------------------------------------------------------ rasterization
 * Projection of one control point (binary32).  Returns 0 when the point is
 * not strictly between the near and far planes. */
static int orc_proj(const orc_cam *c, const float *p, float o[4])
{
    float dx = p[0] - c->eye[0], dy = p[1] - c->eye[1], dz = p[2] - c->eye[2];
    float X = (c->R[0] * dx + c->R[1] * dy) + c->R[2] * dz;
    float Y = (c->R[3] * dx + c->R[4] * dy) + c->R[5] * dz;
    float Z = (c->R[6] * dx + c->R[7] * dy) + c->R[8] * dz;
    if (!(Z > c->znear && Z < c->zfar)) return 0;
    float iz = 1.0f / Z;
    o[0] = c->cx + c->fx * (X * iz);
    o[1] = c->cy - c->fy * (Y * iz);
    o[2] = p[3] * (c->fy * iz);
    o[3] = iz;
    return 1;
}

int orc_project_export(const float *cam, const float *p, float o[4])
{
    return orc_proj((const orc_cam *)cam, p, o);
}

/* 24-bit normalised linear depth code: truncation of d * 2^24, clamped. */
static uint32_t orc_qdepth(float z, float znear, float inv_range)
{
    float d = (z - znear) * inv_range;
    float fq = d * 16777216.0f;
    if (!(fq > 0.0f)) return 0u;
    if (fq >= 16777215.0f) return ORC_QMAX;
    return (uint32_t)fq;
}

uint32_t orc_qdepth_export(float z, float znear, float zfar)
{
    return orc_qdepth(z, znear, 1.0f / (zfar - znear));
}

/* Centre-sample and conservative coverage of pixel (i, j) by the projected
 * segment a -> b (each (x, y, pixel width, 1/z)).  Writes the key depth code
 * when either test passes.  Returns bit0 = centre, bit1 = conservative. */
static int orc_cover_tz(const float a[4], const float b[4], int i, int j, float r_min,
                        float znear, float inv_range, uint32_t *q, float *ts_out, float *z_out);

static int orc_cover(const float a[4], const float b[4], int i, int j, float r_min,
                     float znear, float inv_range, uint32_t *q)
{
    return orc_cover_tz(a, b, i, j, r_min, znear, inv_range, q, NULL, NULL);
}

/* As orc_cover; also returns the clamped closest-point parameter ts and the
 * linear depth z the depth code is taken from (binary32). */
static int orc_cover_tz(const float a[4], const float b[4], int i, int j, float r_min,
                        float znear, float inv_range, uint32_t *q, float *ts_out, float *z_out)
{
    float x0 = a[0], y0 = a[1], w0 = a[2], iz0 = a[3];
    float x1 = b[0], y1 = b[1], w1 = b[2], iz1 = b[3];
    float dx = x1 - x0, dy = y1 - y0;
    float len2 = dx * dx + dy * dy;
    float ilen2 = len2 > 0.0f ? 1.0f / len2 : 0.0f;
    float wmax = w0 > w1 ? w0 : w1;
    float ra = 0.5f * wmax;
    ra = ra > r_min ? ra : r_min;

    float px = (float)i + 0.5f, py = (float)j + 0.5f;
    float ux = px - x0, uy = py - y0;
    float tn = ux * dx + uy * dy;

    /* centre sample: distance from the pixel centre to the segment (flat caps,
     * half-open in t) within the local half width */
    int center;
    if (len2 > 0.0f) {
        float t = tn * ilen2;
        float wt = w0 + t * (w1 - w0);
        float r = 0.5f * wt;
        r = r > r_min ? r : r_min;
        float cr = ux * dy - uy * dx;
        center = (tn >= 0.0f) && (tn < len2) && (cr * cr <= (r * r) * len2);
    } else {
        float r = 0.5f * w0;
        r = r > r_min ? r : r_min;
        center = (ux * ux + uy * uy) <= r * r;
    }

    /* conservative: the segment meets the pixel square dilated by ra
     * (separating-axis test on x, y and the segment normal) */
    float bx0 = (float)i - ra, bx1 = ((float)i + 1.0f) + ra;
    float by0 = (float)j - ra, by1 = ((float)j + 1.0f) + ra;
    float sxmn = x0 < x1 ? x0 : x1, sxmx = x0 > x1 ? x0 : x1;
    float symn = y0 < y1 ? y0 : y1, symx = y0 > y1 ? y0 : y1;
    int cons = (sxmn <= bx1) && (sxmx >= bx0) && (symn <= by1) && (symx >= by0);
    if (cons) {
        float fa = (bx0 - x0) * dy, fb = (bx1 - x0) * dy;
        float ga = (by0 - y0) * dx, gb = (by1 - y0) * dx;
        float fmn = (fa < fb ? fa : fb) - (ga > gb ? ga : gb);
        float fmx = (fa > fb ? fa : fb) - (ga < gb ? ga : gb);
        cons = (fmn <= 0.0f) && (fmx >= 0.0f);
    }
    if (!center && !cons) return 0;

    /* depth at the closest point, perspective-correct through 1/z */
    float ts = tn * ilen2;
    ts = ts > 0.0f ? ts : 0.0f;
    ts = ts < 1.0f ? ts : 1.0f;
    float iz = iz0 + ts * (iz1 - iz0);
    float z = 1.0f / iz;
    *q = orc_qdepth(z, znear, inv_range);
    if (ts_out) *ts_out = ts;
    if (z_out) *z_out = z;
    return (center ? 1 : 0) | (cons ? 2 : 0);
}

int orc_cover_export(const float a[4], const float b[4], int i, int j, float r_min,
                     float znear, float zfar, uint32_t *q)
{
    return orc_cover(a, b, i, j, r_min, znear, 1.0f / (zfar - znear), q);
}

/* Visibility buffer: vis[s][l][p] = min over the prefill and over all
 * segments of scene s covering p in layer l of key(s, p) (Sec. 3.1.2, with the
 * 64-bit atomic-min replaced by its definition).  brute != 0 tests every
 * pixel against every segment; otherwise only the segment's dilated bounding
 * box.  `order`, if given, is a permutation of segment ids to visit. */
/* vis = min(vis, key) as one atomic step: compare-and-swap until the stored
 * key is not larger (threaded raster only). */
static void orc_atomic_min(uint64_t *p, uint64_t key)
{
    uint64_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (key < cur &&
           !__atomic_compare_exchange_n(p, &cur, key, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
    }
}

/* Scene of stream point v: the s with scene_off[s] <= v < scene_off[s + 1]. */
static uint32_t orc_scene_of(const uint32_t *scene_off, uint32_t n_scenes, uint64_t v)
{
    uint32_t lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) / 2;
        if (v >= scene_off[mid]) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Segment v of scene s into the two layers over its dilated bounding box
 * (optionally clipped to window win); atomic != 0 takes each minimum with
 * orc_atomic_min. */
static void orc_raster_seg(const float *pos_w, uint64_t v, const orc_cam *c, int width,
                           int height, float r_min, const int *win, uint64_t *v0, uint64_t *v1,
                           int atomic)
{
    float inv_range = 1.0f / (c->zfar - c->znear);
    float a[4], b[4];
    if (!orc_proj(c, pos_w + 4 * v, a) || !orc_proj(c, pos_w + 4 * (v + 1), b)) return;
    int i0 = 0, i1 = width - 1, j0 = 0, j1 = height - 1;
    float ra = 0.5f * (a[2] > b[2] ? a[2] : b[2]);
    ra = ra > r_min ? ra : r_min;
    float xmn = (a[0] < b[0] ? a[0] : b[0]) - ra - 2.0f;
    float xmx = (a[0] > b[0] ? a[0] : b[0]) + ra + 2.0f;
    float ymn = (a[1] < b[1] ? a[1] : b[1]) - ra - 2.0f;
    float ymx = (a[1] > b[1] ? a[1] : b[1]) + ra + 2.0f;
    if (xmx < 0.0f || ymx < 0.0f || xmn > (float)width || ymn > (float)height) return;
    if (xmn > 0.0f) i0 = (int)xmn;
    if (ymn > 0.0f) j0 = (int)ymn;
    if (xmx < (float)(width - 1)) i1 = (int)xmx;
    if (ymx < (float)(height - 1)) j1 = (int)ymx;
    if (win) {
        i0 = i0 > win[0] ? i0 : win[0];
        j0 = j0 > win[1] ? j0 : win[1];
        i1 = i1 < win[2] ? i1 : win[2];
        j1 = j1 < win[3] ? j1 : win[3];
    }
    for (int j = j0; j <= j1; ++j) {
        for (int i = i0; i <= i1; ++i) {
            uint32_t q;
            int m = orc_cover(a, b, i, j, r_min, c->znear, inv_range, &q);
            if (!m) continue;
            uint64_t key = ((uint64_t)q << ORC_ID_BITS) | (uint64_t)v;
            size_t p = (size_t)j * width + i;
            if (atomic) {
                if (m & 1) orc_atomic_min(v0 + p, key);
                if (m & 2) orc_atomic_min(v1 + p, key);
            } else {
                if ((m & 1) && key < v0[p]) v0[p] = key;
                if ((m & 2) && key < v1[p]) v1[p] = key;
            }
        }
    }
}

int orc_raster(const float *pos_w, const uint8_t *flags, const uint32_t *scene_off,
               const float *cams, uint32_t n_scenes, int width, int height, float r_min,
               const float *scene_z, int brute, const uint32_t *order, uint64_t n_order,
               const int *win, uint64_t *vis)
{
    size_t npix = (size_t)width * (size_t)height;
    for (uint32_t s = 0; s < n_scenes; ++s) {
        const orc_cam *c = (const orc_cam *)(cams + 18 * (size_t)s);
        float inv_range = 1.0f / (c->zfar - c->znear);
        uint64_t *v0 = vis + (size_t)s * 2 * npix, *v1 = v0 + npix;
        for (size_t p = 0; p < npix; ++p) {
            uint64_t k = ORC_EMPTY;
            if (scene_z) {
                float z = scene_z[(size_t)s * npix + p];
                if (z > c->znear && z < c->zfar)
                    k = ((uint64_t)orc_qdepth(z, c->znear, inv_range) << ORC_ID_BITS) | ORC_ID_OPAQUE;
            }
            v0[p] = k;
            v1[p] = k;
        }
    }
    uint64_t n_cp = scene_off[n_scenes];
    if (orc_nthreads > 1 && !brute && !order) {
        /* the same segments, spread over threads */
        int64_t n_seg = n_cp > 0 ? (int64_t)n_cp - 1 : 0;
#pragma omp parallel for schedule(dynamic, 1024) num_threads(orc_nthreads)
        for (int64_t it = 0; it < n_seg; ++it) {
            uint64_t v = (uint64_t)it;
            if (flags[v] & ORC_TIP) continue;
            uint32_t sv = orc_scene_of(scene_off, n_scenes, v);
            const orc_cam *c = (const orc_cam *)(cams + 18 * (size_t)sv);
            uint64_t *v0 = vis + (size_t)sv * 2 * npix;
            orc_raster_seg(pos_w, v, c, width, height, r_min, win, v0, v0 + npix, 1);
        }
        return 0;
    }
    uint64_t n_visit = order ? n_order : n_cp;
    uint32_t s = 0;
    for (uint64_t it = 0; it < n_visit; ++it) {
        uint64_t v = order ? order[it] : it;
        if (v + 1 >= n_cp || (flags[v] & ORC_TIP)) continue;
        if (order) {
            s = 0;
            while (s + 1 < n_scenes && v >= scene_off[s + 1]) s++;
        } else {
            while (s + 1 < n_scenes && v >= scene_off[s + 1]) s++;
        }
        const orc_cam *c = (const orc_cam *)(cams + 18 * (size_t)s);
        uint64_t *v0 = vis + (size_t)s * 2 * npix, *v1 = v0 + npix;
        if (!brute) {
            orc_raster_seg(pos_w, v, c, width, height, r_min, win, v0, v1, 0);
            continue;
        }
        /* brute force: every pixel (of the window) against the segment */
        float inv_range = 1.0f / (c->zfar - c->znear);
        float a[4], b[4];
        if (!orc_proj(c, pos_w + 4 * v, a) || !orc_proj(c, pos_w + 4 * (v + 1), b)) continue;
        int i0 = 0, i1 = width - 1, j0 = 0, j1 = height - 1;
        if (win) {
            i0 = i0 > win[0] ? i0 : win[0];
            j0 = j0 > win[1] ? j0 : win[1];
            i1 = i1 < win[2] ? i1 : win[2];
            j1 = j1 < win[3] ? j1 : win[3];
        }
        for (int j = j0; j <= j1; ++j) {
            for (int i = i0; i <= i1; ++i) {
                uint32_t q;
                int m = orc_cover(a, b, i, j, r_min, c->znear, inv_range, &q);
                if (!m) continue;
                uint64_t key = ((uint64_t)q << ORC_ID_BITS) | (uint64_t)v;
                size_t p = (size_t)j * width + i;
                if ((m & 1) && key < v0[p]) v0[p] = key;
                if ((m & 2) && key < v1[p]) v1[p] = key;
            }
        }
    }
    return 0;
}

/* Count of (segment, pixel) pairs passing each predicate, no min: the
 * algorithmic work of the raster step (one atomic-min per pair and layer). */
int orc_cover_counts(const float *pos_w, const uint8_t *flags, const uint32_t *scene_off,
                     const float *cams, uint32_t n_scenes, int width, int height,
                     float r_min, uint64_t out[3])
{
    uint64_t nc = 0, na = 0, nseg = 0;
    uint64_t n_cp = scene_off[n_scenes];
    uint32_t s = 0;
    for (uint64_t v = 0; v + 1 < n_cp; ++v) {
        if (flags[v] & ORC_TIP) continue;
        while (s + 1 < n_scenes && v >= scene_off[s + 1]) s++;
        const orc_cam *c = (const orc_cam *)(cams + 18 * (size_t)s);
        float inv_range = 1.0f / (c->zfar - c->znear);
        float a[4], b[4];
        nseg++;
        if (!orc_proj(c, pos_w + 4 * v, a) || !orc_proj(c, pos_w + 4 * (v + 1), b)) continue;
        float ra = 0.5f * (a[2] > b[2] ? a[2] : b[2]);
        ra = ra > r_min ? ra : r_min;
        float xmn = (a[0] < b[0] ? a[0] : b[0]) - ra - 2.0f;
        float xmx = (a[0] > b[0] ? a[0] : b[0]) + ra + 2.0f;
        float ymn = (a[1] < b[1] ? a[1] : b[1]) - ra - 2.0f;
        float ymx = (a[1] > b[1] ? a[1] : b[1]) + ra + 2.0f;
        if (xmx < 0.0f || ymx < 0.0f || xmn > (float)width || ymn > (float)height) continue;
        int i0 = xmn > 0.0f ? (int)xmn : 0, j0 = ymn > 0.0f ? (int)ymn : 0;
        int i1 = xmx < (float)(width - 1) ? (int)xmx : width - 1;
        int j1 = ymx < (float)(height - 1) ? (int)ymx : height - 1;
        for (int j = j0; j <= j1; ++j)
            for (int i = i0; i <= i1; ++i) {
                uint32_t q;
                int m = orc_cover(a, b, i, j, r_min, c->znear, inv_range, &q);
                nc += (m & 1) ? 1 : 0;
                na += (m & 2) ? 1 : 0;
            }
    }
    out[0] = nseg;
    out[1] = nc;
    out[2] = na;
    return 0;
}

/* ------------------------------------------------------------ resolve (fp64) */
typedef struct {
    double light_dir[3];  /* towards the light, need not be normalised */
    double light_rgb[3];
    double ka, kd, ks;
    int spec_squarings;   /* specular exponent 2^spec_squarings on (1 - (T.H)^2) */
    int filter_radius;    /* r of the (2r+1)^2 window */
    double s_par, s_perp; /* sigma_par = r * s_par, sigma_perp = r * s_perp */
    double sigma_c;       /* colour similarity */
    double iso_scale;     /* sigma_iso = iso_scale * r */
    uint32_t dq_reject;   /* neighbour depth rejection, in depth-code units */
    uint32_t dq_mismatch; /* centre / conservative depth mismatch, in depth-code units */
    float strip_half2;    /* squared half width of the alpha strip (binary32 decision) */
    float iso_len;        /* screen tangent shorter than this -> isotropic fallback */
    double bg[3];
    int mode;             /* 0 filter, 1 soft (not handled here), 2 centre only */
} orc_shade_params;

typedef struct { double x, y, z; } v3d;
static v3d d3(double x, double y, double z) { v3d r = {x, y, z}; return r; }
static v3d d3_sub(v3d a, v3d b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3d d3_add(v3d a, v3d b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3d d3_scale(v3d a, double s) { return d3(a.x * s, a.y * s, a.z * s); }
static double d3_dot(v3d a, v3d b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3d d3_norm(v3d a)
{
    double n = sqrt(d3_dot(a, a));
    return n > 0.0 ? d3_scale(a, 1.0 / n) : d3(0, 0, 0);
}
static v3d d3_loadf(const float *p) { return d3(p[0], p[1], p[2]); }

/* binary64 projection (continuous quantities) */
static void orc_proj64(const orc_cam *c, const float *p, double o[3])
{
    double dx = (double)p[0] - c->eye[0], dy = (double)p[1] - c->eye[1], dz = (double)p[2] - c->eye[2];
    double X = c->R[0] * dx + c->R[1] * dy + c->R[2] * dz;
    double Y = c->R[3] * dx + c->R[4] * dy + c->R[5] * dz;
    double Z = c->R[6] * dx + c->R[7] * dy + c->R[8] * dz;
    o[0] = c->cx + c->fx * X / Z;
    o[1] = c->cy - c->fy * Y / Z;
    o[2] = 1.0 / Z;
}

/* Tangent of the styled polyline at control point v (Code 1's calcTangent
 * applied to the styled strand). */
static v3d orc_cp_tangent(const float *pos_w, const uint8_t *flags, uint64_t v)
{
    v3d d;
    if (flags[v] & ORC_ROOT) d = d3_sub(d3_loadf(pos_w + 4 * (v + 1)), d3_loadf(pos_w + 4 * v));
    else if (flags[v] & ORC_TIP) d = d3_sub(d3_loadf(pos_w + 4 * v), d3_loadf(pos_w + 4 * (v - 1)));
    else d = d3_sub(d3_loadf(pos_w + 4 * (v + 1)), d3_loadf(pos_w + 4 * (v - 1)));
    return d3_norm(d);
}

/* Deferred 1-spp shading of segment v seen through pixel centre (px, py):
 * Kajiya-Kay style diffuse sin(T, L) term plus a sin^(2^(n+1)) specular lobe
 * about the half vector, one directional light (Sec. 3.4, simplified). */
static void orc_shade_point(const orc_cam *c, const orc_shade_params *sp, v3d X, v3d T,
                            const double albv[3], double shadow, double ao, double out[3]);

static void orc_shade_px(const float *pos_w, const float *rgb, const uint8_t *flags,
                         const orc_cam *c, const orc_shade_params *sp, uint64_t v,
                         double px, double py, double shadow, double out[3])
{
    double a[3], b[3];
    orc_proj64(c, pos_w + 4 * v, a);
    orc_proj64(c, pos_w + 4 * (v + 1), b);
    double dx = b[0] - a[0], dy = b[1] - a[1];
    double len2 = dx * dx + dy * dy;
    double ts = 0.0;
    if (len2 > 0.0) {
        ts = ((px - a[0]) * dx + (py - a[1]) * dy) / len2;
        ts = ts < 0.0 ? 0.0 : (ts > 1.0 ? 1.0 : ts);
    }
    double iz = a[2] + ts * (b[2] - a[2]);
    double t3 = ts * b[2] / iz;        /* screen parameter -> segment parameter */
    v3d P0 = d3_loadf(pos_w + 4 * v), P1 = d3_loadf(pos_w + 4 * (v + 1));
    v3d X = d3_add(P0, d3_scale(d3_sub(P1, P0), t3));
    v3d T0 = orc_cp_tangent(pos_w, flags, v), T1 = orc_cp_tangent(pos_w, flags, v + 1);
    v3d T = d3_norm(d3_add(T0, d3_scale(d3_sub(T1, T0), t3)));
    v3d c0 = d3_loadf(rgb + 4 * v), c1 = d3_loadf(rgb + 4 * (v + 1));
    v3d alb = d3_add(c0, d3_scale(d3_sub(c1, c0), t3));
    double albv[3] = {alb.x, alb.y, alb.z};
    orc_shade_point(c, sp, X, T, albv, shadow, 1.0, out);
}

/* Kajiya-Kay style shading of point X with unit tangent T and albedo alb
 * (Sec. 3.4, simplified): ambient (scaled by the occlusion ao) plus diffuse
 * and specular terms (scaled by the light's transmittance). */
static void orc_shade_point(const orc_cam *c, const orc_shade_params *sp, v3d X, v3d T,
                            const double albv[3], double shadow, double ao, double out[3])
{
    v3d eye = d3(c->eye[0], c->eye[1], c->eye[2]);
    v3d V = d3_norm(d3_sub(eye, X));
    v3d L = d3_norm(d3(sp->light_dir[0], sp->light_dir[1], sp->light_dir[2]));
    v3d H = d3_norm(d3_add(L, V));
    double tl = d3_dot(T, L), th = d3_dot(T, H);
    double sd = 1.0 - tl * tl;
    double diff = sd > 0.0 ? sqrt(sd) : 0.0;
    double sh = 1.0 - th * th;
    sh = sh > 0.0 ? sh : 0.0;
    double spec = sh;
    for (int k = 0; k < sp->spec_squarings; ++k) spec = spec * spec;
    /* the light's transmittance scales the direct terms, not the ambient one */
    for (int ch = 0; ch < 3; ++ch)
        out[ch] = albv[ch] * sp->light_rgb[ch] * (sp->ka * ao + shadow * sp->kd * diff) +
                  shadow * sp->ks * sp->light_rgb[ch] * spec;
}

static int orc_is_hit(uint64_t k)
{
    return k != ORC_EMPTY && (k & ORC_ID_MASK) != ORC_ID_OPAQUE;
}

/* Resolve: centre shading, then strand connection + elliptical bilateral
 * filter + alpha estimation + composite over bg (Sec. 3.3, Code 2 with the
 * readings stated in the design notes).  out_rgba [S][H][W][4] in binary64.
 * center_rgb (optional, [S][H][W][3]) receives the raw centre shading. */
int orc_resolve_shadowed(const float *pos_w, const float *rgb, const uint8_t *flags,
                         const uint64_t *vis, const float *cams, uint32_t n_scenes, int width,
                         int height, const orc_shade_params *sp, const int *win,
                         const double *shadow, double *out_rgba, double *center_rgb);

int orc_resolve(const float *pos_w, const float *rgb, const uint8_t *flags,
                const uint64_t *vis, const float *cams, uint32_t n_scenes, int width,
                int height, const orc_shade_params *sp, const int *win, double *out_rgba,
                double *center_rgb)
{
    return orc_resolve_shadowed(pos_w, rgb, flags, vis, cams, n_scenes, width, height, sp, win,
                                NULL, out_rgba, center_rgb);
}

/* As orc_resolve; shadow (optional, [S][H][W]) is the light's transmittance
 * at each pixel's shaded point. */
int orc_resolve_shadowed(const float *pos_w, const float *rgb, const uint8_t *flags,
                         const uint64_t *vis, const float *cams, uint32_t n_scenes, int width,
                         int height, const orc_shade_params *sp, const int *win,
                         const double *shadow, double *out_rgba, double *center_rgb)
{
    size_t npix = (size_t)width * height;
    if (sp->mode == 1) return -2;   /* soft coverage lives in the binary64 torch oracle */
    double *cc = (double *)calloc(3 * npix, sizeof(double));
    if (!cc) return -1;
    int r = sp->filter_radius;
    double spar = r * sp->s_par, sperp = r * sp->s_perp, siso = sp->iso_scale * r;
    /* output window (inclusive) and the centre-shading window it depends on */
    int oi0 = 0, oj0 = 0, oi1 = width - 1, oj1 = height - 1;
    if (win) { oi0 = win[0]; oj0 = win[1]; oi1 = win[2]; oj1 = win[3]; }
    int ci0 = oi0 - r < 0 ? 0 : oi0 - r, cj0 = oj0 - r < 0 ? 0 : oj0 - r;
    int ci1 = oi1 + r > width - 1 ? width - 1 : oi1 + r;
    int cj1 = oj1 + r > height - 1 ? height - 1 : oj1 + r;
    for (uint32_t s = 0; s < n_scenes; ++s) {
        const orc_cam *c = (const orc_cam *)(cams + 18 * (size_t)s);
        const uint64_t *g = vis + (size_t)s * 2 * npix, *a = g + npix;
        double *out = out_rgba + (size_t)s * 4 * npix;
        /* pass 1: centre shading of every centre-sample hit */
#pragma omp parallel for schedule(dynamic, 4) num_threads(orc_nthreads) if (orc_nthreads > 1)
        for (int j = cj0; j <= cj1; ++j)
            for (int i = ci0; i <= ci1; ++i) {
                size_t p = (size_t)j * width + i;
                double *o = cc + 3 * p;
                o[0] = o[1] = o[2] = 0.0;
                if (orc_is_hit(g[p]))
                    orc_shade_px(pos_w, rgb, flags, c, sp, g[p] & ORC_ID_MASK, i + 0.5, j + 0.5,
                                 shadow ? shadow[(size_t)s * npix + p] : 1.0, o);
                if (center_rgb) {
                    double *q = center_rgb + ((size_t)s * npix + p) * 3;
                    q[0] = o[0]; q[1] = o[1]; q[2] = o[2];
                }
            }
        /* pass 2: reconstruction */
#pragma omp parallel for schedule(dynamic, 4) num_threads(orc_nthreads) if (orc_nthreads > 1)
        for (int j = oj0; j <= oj1; ++j)
            for (int i = oi0; i <= oi1; ++i) {
                size_t p = (size_t)j * width + i;
                double *o = out + 4 * p;
                int hc = orc_is_hit(g[p]), ha = orc_is_hit(a[p]);
                double rgbv[3] = {0, 0, 0}, alpha = 0.0;
                if (sp->mode == 2) {
                    if (hc) { rgbv[0] = cc[3 * p]; rgbv[1] = cc[3 * p + 1]; rgbv[2] = cc[3 * p + 2]; alpha = 1.0; }
                } else if (hc || ha) {
                    uint32_t qc = (uint32_t)(g[p] >> ORC_ID_BITS), qa = (uint32_t)(a[p] >> ORC_ID_BITS);
                    int mism = hc && ha && qc > qa && (qc - qa) >= sp->dq_mismatch;
                    uint64_t src = (hc && !mism) ? g[p] : a[p];
                    uint64_t vs = src & ORC_ID_MASK;
                    uint32_t qP = (uint32_t)(src >> ORC_ID_BITS);
                    /* screen tangent: binary32 for the strip decision ... */
                    float pa[4], pb[4];
                    orc_proj(c, pos_w + 4 * vs, pa);
                    orc_proj(c, pos_w + 4 * (vs + 1), pb);
                    float tdx = pb[0] - pa[0], tdy = pb[1] - pa[1];
                    float tlen = sqrtf(tdx * tdx + tdy * tdy);
                    int iso = !(tlen >= sp->iso_len);
                    float Tx = 0.0f, Ty = 0.0f;
                    if (!iso) { float il = 1.0f / tlen; Tx = tdx * il; Ty = tdy * il; }
                    /* ... binary64 for the weights */
                    double da[3], db[3];
                    orc_proj64(c, pos_w + 4 * vs, da);
                    orc_proj64(c, pos_w + 4 * (vs + 1), db);
                    double ddx = db[0] - da[0], ddy = db[1] - da[1];
                    double dlen = sqrt(ddx * ddx + ddy * ddy);
                    double Txd = iso ? 0.0 : ddx / dlen, Tyd = iso ? 0.0 : ddy / dlen;
                    const double *CP = cc + 3 * p;
                    int colour_sim = hc && !mism;
                    double S[3] = {0, 0, 0}, W = 0.0;
                    int Hc = 0, Ha = 0, nacc = 0;
                    for (int oy = -r; oy <= r; ++oy) {
                        int jq = j + oy;
                        if (jq < 0 || jq >= height) continue;
                        for (int ox = -r; ox <= r; ++ox) {
                            int iq = i + ox;
                            if (iq < 0 || iq >= width) continue;
                            size_t qx = (size_t)jq * width + iq;
                            int qc_hit = orc_is_hit(g[qx]), qa_hit = orc_is_hit(a[qx]);
                            float fx = (float)ox, fy = (float)oy, perp2;
                            if (iso) {
                                perp2 = fx * fx + fy * fy;
                            } else {
                                float par = fx * Tx + fy * Ty;
                                float ex = fx - par * Tx, ey = fy - par * Ty;
                                perp2 = ex * ex + ey * ey;
                            }
                            if (perp2 <= sp->strip_half2) {
                                Ha += (qc_hit || qa_hit) ? 1 : 0;
                                Hc += qc_hit ? 1 : 0;
                            }
                            if (!qc_hit) continue;
                            uint32_t qq = (uint32_t)(g[qx] >> ORC_ID_BITS);
                            uint32_t dq = qq > qP ? qq - qP : qP - qq;
                            if (dq > sp->dq_reject) continue;
                            double ws;
                            if (iso) {
                                ws = exp(-((double)ox * ox + (double)oy * oy) / (siso * siso));
                            } else {
                                double par = ox * Txd + oy * Tyd;
                                double ex = ox - par * Txd, ey = oy - par * Tyd;
                                ws = exp(-(par * par) / (spar * spar) - (ex * ex + ey * ey) / (sperp * sperp));
                            }
                            const double *CQ = cc + 3 * qx;
                            double wc = 1.0;
                            if (colour_sim) {
                                double e0 = CP[0] - CQ[0], e1 = CP[1] - CQ[1], e2 = CP[2] - CQ[2];
                                wc = exp(-(e0 * e0 + e1 * e1 + e2 * e2) / (sp->sigma_c * sp->sigma_c));
                            }
                            double w = ws * wc;
                            S[0] += w * CQ[0]; S[1] += w * CQ[1]; S[2] += w * CQ[2];
                            W += w;
                            nacc++;
                        }
                    }
                    double aP = Ha > 0 ? (double)Hc / (double)Ha : 1.0;
                    if (hc && !mism) {
                        for (int ch = 0; ch < 3; ++ch) rgbv[ch] = S[ch] / W;
                        alpha = aP;
                    } else if (mism) {
                        for (int ch = 0; ch < 3; ++ch) {
                            double rec = nacc > 0 ? S[ch] / W : CP[ch];
                            rgbv[ch] = aP * rec + (1.0 - aP) * CP[ch];
                        }
                        alpha = 1.0;
                    } else if (nacc > 0) {
                        /* promoted: a reconstruction exists iff a centre neighbour was accepted */
                        for (int ch = 0; ch < 3; ++ch) rgbv[ch] = S[ch] / W;
                        alpha = aP;
                    }
                }
                for (int ch = 0; ch < 3; ++ch) o[ch] = alpha * rgbv[ch] + (1.0 - alpha) * sp->bg[ch];
                o[3] = alpha;
            }
    }
    free(cc);
    return 0;
}

/* ------------------------------------------------------------ deep opacity map
 * Shadows of Sec. 3.4 (deep opacity maps, Yuksel & Keyser 2008) queried with
 * the LOD depth correction of Sec. 3.2.3.  The map is built from the light's
 * view: q0(p) is the depth code of the nearest fragment of light pixel p (the
 * conservative layer of the light view's visibility buffer, rasterized
 * without a scene depth), and every (segment, light pixel) pair accepted by
 * the conservative test, at depth code q, is counted in layer
 * min((q - q0) / L, K - 1) of that pixel.  Counting (instead of blending
 * opacities) keeps the map exact and independent of order. */
int orc_dom_accumulate(const float *pos_w, const uint8_t *flags, uint64_t n_cp,
                       const float *lcam, int width, int height, float r_min,
                       const uint64_t *light_vis, uint32_t layer_codes, uint32_t n_layers,
                       uint32_t *counts)
{
    size_t npix = (size_t)width * (size_t)height;
    memset(counts, 0, sizeof(uint32_t) * npix * n_layers);
    const orc_cam *c = (const orc_cam *)lcam;
    float inv_range = 1.0f / (c->zfar - c->znear);
    const uint64_t *va = light_vis + npix;
    for (uint64_t v = 0; v + 1 < n_cp; ++v) {
        if (flags[v] & ORC_TIP) continue;
        float a[4], b[4];
        if (!orc_proj(c, pos_w + 4 * v, a) || !orc_proj(c, pos_w + 4 * (v + 1), b)) continue;
        float ra = 0.5f * (a[2] > b[2] ? a[2] : b[2]);
        ra = ra > r_min ? ra : r_min;
        float xmn = (a[0] < b[0] ? a[0] : b[0]) - ra - 2.0f;
        float xmx = (a[0] > b[0] ? a[0] : b[0]) + ra + 2.0f;
        float ymn = (a[1] < b[1] ? a[1] : b[1]) - ra - 2.0f;
        float ymx = (a[1] > b[1] ? a[1] : b[1]) + ra + 2.0f;
        if (xmx < 0.0f || ymx < 0.0f || xmn > (float)width || ymn > (float)height) continue;
        int i0 = xmn > 0.0f ? (int)xmn : 0, j0 = ymn > 0.0f ? (int)ymn : 0;
        int i1 = xmx < (float)(width - 1) ? (int)xmx : width - 1;
        int j1 = ymx < (float)(height - 1) ? (int)ymx : height - 1;
        for (int j = j0; j <= j1; ++j)
            for (int i = i0; i <= i1; ++i) {
                uint32_t q;
                int m = orc_cover(a, b, i, j, r_min, c->znear, inv_range, &q);
                if (!(m & 2)) continue;
                size_t p = (size_t)j * width + i;
                uint32_t q0 = (uint32_t)(va[p] >> ORC_ID_BITS);
                uint32_t k = q > q0 ? (q - q0) / layer_codes : 0u;
                if (k > n_layers - 1) k = n_layers - 1;
                counts[(size_t)k * npix + p] += 1u;
            }
    }
    return 0;
}

/* Transmittance towards the light at the shaded point of every camera pixel
 * with a centre hit (T = 1 elsewhere).  The point X is the one the resolve
 * shades (binary64), projected by the light camera in binary64: light pixel
 * floor(x), floor(y) and depth code q of its linear depth.  The LOD
 * correction moves it towards the light inside the groom: with
 * beta = N_LOD / N_b of its bundle (binary32), the log of its depth below the
 * first fragment is shifted by -Delta = log beta, i.e. q' = q0 +
 * (uint32)((float)(q - q0) * beta).  The opacity in front of q' is the
 * counts of the layers before q' plus the linearly interpolated part of its
 * own layer (the last layer reaches to infinity and is taken whole once
 * passed), times the per-fragment opacity alpha; T = exp(-opacity). */
int orc_dom_shadow(const float *pos_w, const uint8_t *flags, const uint64_t *vis,
                   const float *cam, int width, int height, const float *lcam, int lwidth,
                   int lheight, const uint64_t *light_vis, const uint32_t *counts,
                   uint32_t layer_codes, uint32_t n_layers, const uint32_t *table,
                   const uint32_t *bundle_nstrands, uint32_t n_bundles, double alpha,
                   double *shadow)
{
    size_t lnpix = (size_t)lwidth * lheight;
    const orc_cam *c = (const orc_cam *)cam, *lc = (const orc_cam *)lcam;
    for (int j = 0; j < height; ++j)
        for (int i = 0; i < width; ++i) {
            size_t p = (size_t)j * width + i;
            shadow[p] = 1.0;
            if (!orc_is_hit(vis[p])) continue;
            uint64_t v = vis[p] & ORC_ID_MASK;
            /* the shaded point, as orc_shade_px computes it */
            double a[3], b[3];
            orc_proj64(c, pos_w + 4 * v, a);
            orc_proj64(c, pos_w + 4 * (v + 1), b);
            double dx = b[0] - a[0], dy = b[1] - a[1];
            double len2 = dx * dx + dy * dy, ts = 0.0;
            if (len2 > 0.0) {
                ts = ((i + 0.5 - a[0]) * dx + (j + 0.5 - a[1]) * dy) / len2;
                ts = ts < 0.0 ? 0.0 : (ts > 1.0 ? 1.0 : ts);
            }
            double iz = a[2] + ts * (b[2] - a[2]);
            double t3 = ts * b[2] / iz;
            v3d P0 = d3_loadf(pos_w + 4 * v), P1 = d3_loadf(pos_w + 4 * (v + 1));
            v3d X = d3_add(P0, d3_scale(d3_sub(P1, P0), t3));
            /* into the light view */
            double ex = X.x - lc->eye[0], ey = X.y - lc->eye[1], ez = X.z - lc->eye[2];
            double LX = lc->R[0] * ex + lc->R[1] * ey + lc->R[2] * ez;
            double LY = lc->R[3] * ex + lc->R[4] * ey + lc->R[5] * ez;
            double LZ = lc->R[6] * ex + lc->R[7] * ey + lc->R[8] * ez;
            if (!(LZ > lc->znear && LZ < lc->zfar)) continue;
            double lx = lc->cx + lc->fx * LX / LZ, ly = lc->cy - lc->fy * LY / LZ;
            if (!(lx >= 0.0 && ly >= 0.0 && lx < (double)lwidth && ly < (double)lheight)) continue;
            size_t lp = (size_t)floor(ly) * lwidth + (size_t)floor(lx);
            uint64_t k0 = light_vis[lnpix + lp];
            if (k0 == ORC_EMPTY) continue;
            uint32_t q0 = (uint32_t)(k0 >> ORC_ID_BITS);
            double dq = (LZ - lc->znear) / ((double)lc->zfar - lc->znear) * 16777216.0;
            uint32_t q = dq > 0.0 ? (dq >= 16777215.0 ? 16777215u : (uint32_t)dq) : 0u;
            if (q <= q0) continue;
            /* bundle of segment v: last b whose first CP is <= v */
            uint32_t lo = 0, hi = n_bundles;
            while (hi - lo > 1) {
                uint32_t mid = (lo + hi) / 2;
                if (table[4 * (size_t)mid + 3] <= v) lo = mid; else hi = mid;
            }
            float beta = (float)table[4 * (size_t)lo] / (float)bundle_nstrands[lo];
            uint32_t d = (uint32_t)((float)(q - q0) * beta);
            uint32_t kq = d / layer_codes;
            double f;
            if (kq >= n_layers - 1) {
                kq = n_layers - 1;
                f = (double)(d - kq * layer_codes) / layer_codes;
                f = f < 1.0 ? f : 1.0;
            } else {
                f = (double)(d - kq * layer_codes) / layer_codes;
            }
            double o = 0.0;
            for (uint32_t k = 0; k < kq; ++k) o += counts[(size_t)k * lnpix + lp];
            o += f * counts[(size_t)kq * lnpix + lp];
            shadow[p] = exp(-alpha * o);
        }
    (void)flags;
    return 0;
}

/* ------------------------------------------------------------ compressed G-buffer
 * The paper's 64-bit deferred-shading word (Sec. 3.1.2, deferred atomic
 * shading): the 24-bit depth code in the high bits (so that the atomic
 * minimum still keeps the nearest fragment), then 40 bits of shading inputs
 * quantised to 8 or 6 bits.  Reading (the bit layout is not printed):
 *   bits 39..32, 31..24  octahedral tangent (u, v), 8 bits each
 *   bits 23..18, 17..12, 11..6  albedo r, g, b, 6 bits each (the appearance
 *                                parameters; the paper stores uvw to look
 *                                them up, here they are the colours)
 *   bits 5..0   ambient occlusion, 6 bits (no baked AO: always 63)
 * Position is not stored: the resolve reconstructs it from the depth at the
 * pixel centre.  Every step that decides bits is binary32, in the order
 * written. */

/* unit tangent of CP v as the resolve computes it (binary32); zero for a CP
 * that is both root and tip (it starts no segment) */
static v3f orc_cp_tangent32(const float *pos_w, const uint8_t *flags, uint64_t v)
{
    const uint8_t f = flags[v];
    v3f d = {0.0f, 0.0f, 0.0f};
    if ((f & ORC_ROOT) && (f & ORC_TIP)) return d;
    if (f & ORC_ROOT) d = v3_sub(v3_load(pos_w + 4 * (v + 1)), v3_load(pos_w + 4 * v));
    else if (f & ORC_TIP) d = v3_sub(v3_load(pos_w + 4 * v), v3_load(pos_w + 4 * (v - 1)));
    else d = v3_sub(v3_load(pos_w + 4 * (v + 1)), v3_load(pos_w + 4 * (v - 1)));
    return v3_norm(d);
}

/* x in [-1, 1] -> 0 .. 255 (round to nearest) */
static uint32_t orc_q8(float x)
{
    float f = (x * 0.5f + 0.5f) * 255.0f + 0.5f;
    f = f > 0.0f ? f : 0.0f;
    f = f < 255.0f ? f : 255.0f;
    return (uint32_t)f;
}

/* c in [0, 1] -> 0 .. 63 (round to nearest) */
static uint32_t orc_q6(float c)
{
    float f = c * 63.0f + 0.5f;
    f = f > 0.0f ? f : 0.0f;
    f = f < 63.0f ? f : 63.0f;
    return (uint32_t)f;
}

/* Octahedral map of a direction (Meyer et al. 2010; survey by Cigolle et
 * al. 2014): project onto the octahedron |x| + |y| + |z| = 1, fold the lower
 * half (z < 0) over the diagonals, keep (x, y).  A zero vector maps to the
 * centre. */
static uint32_t orc_oct16(v3f t)
{
    float l1 = (fabsf(t.x) + fabsf(t.y)) + fabsf(t.z);
    float px = 0.0f, py = 0.0f;
    if (l1 > 0.0f) {
        px = t.x / l1;
        py = t.y / l1;
        if (t.z < 0.0f) {
            float ax = fabsf(px), ay = fabsf(py);
            float sx = px >= 0.0f ? 1.0f : -1.0f, sy = py >= 0.0f ? 1.0f : -1.0f;
            px = (1.0f - ay) * sx;
            py = (1.0f - ax) * sy;
        }
    }
    return (orc_q8(px) << 8) | orc_q8(py);
}

uint32_t orc_oct16_export(const float t[3])
{
    v3f v = {t[0], t[1], t[2]};
    return orc_oct16(v);
}

/* 40-bit payload of segment v at closest-point parameter ts with linear depth
 * z: perspective-correct segment parameter t3 = ts * (1/z_1) * z, tangent and
 * albedo interpolated at t3 */
static uint64_t orc_payload(const v3f *T, const float *rgb, uint64_t v, float ts, float z,
                            float iz1)
{
    float t3 = (ts * iz1) * z;
    v3f t = v3_lerp(T[v], T[v + 1], t3);
    v3f c = v3_lerp(v3_load(rgb + 4 * v), v3_load(rgb + 4 * (v + 1)), t3);
    uint64_t w = (uint64_t)orc_oct16(t) << 24;
    w |= (uint64_t)orc_q6(c.x) << 18;
    w |= (uint64_t)orc_q6(c.y) << 12;
    w |= (uint64_t)orc_q6(c.z) << 6;
    w |= 63u;
    return w;
}

/* Visibility buffer with G-buffer payloads: as orc_raster (bounding-box
 * enumeration), every covering segment's key being depth << 40 | payload. */
int orc_raster_gbuf(const float *pos_w, const float *rgb, const uint8_t *flags,
                    const uint32_t *scene_off, const float *cams, uint32_t n_scenes, int width,
                    int height, float r_min, const float *scene_z, uint64_t *vis)
{
    size_t npix = (size_t)width * (size_t)height;
    uint64_t n_cp = scene_off[n_scenes];
    v3f *T = (v3f *)malloc(sizeof(v3f) * (n_cp ? n_cp : 1));
    if (!T) return -1;
    for (uint64_t v = 0; v < n_cp; ++v) T[v] = orc_cp_tangent32(pos_w, flags, v);
    for (uint32_t s = 0; s < n_scenes; ++s) {
        const orc_cam *c = (const orc_cam *)(cams + 18 * (size_t)s);
        float inv_range = 1.0f / (c->zfar - c->znear);
        uint64_t *v0 = vis + (size_t)s * 2 * npix, *v1 = v0 + npix;
        for (size_t p = 0; p < npix; ++p) {
            uint64_t k = ORC_EMPTY;
            if (scene_z) {
                float z = scene_z[(size_t)s * npix + p];
                if (z > c->znear && z < c->zfar)
                    k = ((uint64_t)orc_qdepth(z, c->znear, inv_range) << ORC_ID_BITS) | ORC_ID_OPAQUE;
            }
            v0[p] = k;
            v1[p] = k;
        }
    }
    uint32_t s = 0;
    for (uint64_t v = 0; v + 1 < n_cp; ++v) {
        if (flags[v] & ORC_TIP) continue;
        while (s + 1 < n_scenes && v >= scene_off[s + 1]) s++;
        const orc_cam *c = (const orc_cam *)(cams + 18 * (size_t)s);
        float inv_range = 1.0f / (c->zfar - c->znear);
        float a[4], b[4];
        if (!orc_proj(c, pos_w + 4 * v, a) || !orc_proj(c, pos_w + 4 * (v + 1), b)) continue;
        float iz1 = b[3];     /* 1/z of the segment's second endpoint */
        uint64_t *v0 = vis + (size_t)s * 2 * npix, *v1 = v0 + npix;
        float ra = 0.5f * (a[2] > b[2] ? a[2] : b[2]);
        ra = ra > r_min ? ra : r_min;
        float xmn = (a[0] < b[0] ? a[0] : b[0]) - ra - 2.0f;
        float xmx = (a[0] > b[0] ? a[0] : b[0]) + ra + 2.0f;
        float ymn = (a[1] < b[1] ? a[1] : b[1]) - ra - 2.0f;
        float ymx = (a[1] > b[1] ? a[1] : b[1]) + ra + 2.0f;
        if (xmx < 0.0f || ymx < 0.0f || xmn > (float)width || ymn > (float)height) continue;
        int i0 = xmn > 0.0f ? (int)xmn : 0, j0 = ymn > 0.0f ? (int)ymn : 0;
        int i1 = xmx < (float)(width - 1) ? (int)xmx : width - 1;
        int j1 = ymx < (float)(height - 1) ? (int)ymx : height - 1;
        for (int j = j0; j <= j1; ++j)
            for (int i = i0; i <= i1; ++i) {
                uint32_t q;
                float ts, z;
                int m = orc_cover_tz(a, b, i, j, r_min, c->znear, inv_range, &q, &ts, &z);
                if (!m) continue;
                uint64_t key = ((uint64_t)q << ORC_ID_BITS) | orc_payload(T, rgb, v, ts, z, iz1);
                size_t p = (size_t)j * width + i;
                if ((m & 1) && key < v0[p]) v0[p] = key;
                if ((m & 2) && key < v1[p]) v1[p] = key;
            }
    }
    free(T);
    return 0;
}

/* Shading of one G-buffer pixel (binary64): the position is reconstructed
 * at the pixel centre from the depth code (the middle of its code interval),
 * the tangent from its octahedral code, the albedo and AO from their 6-bit
 * codes; then the shading of the resolve (AO scales the ambient term). */
static void orc_gbuf_decode(const orc_cam *c, uint64_t key, double px, double py, v3d *X,
                            v3d *T, double alb[3], double *ao)
{
    uint64_t w = key & ORC_ID_MASK;
    double q = (double)(key >> ORC_ID_BITS);
    double z = c->znear + (q + 0.5) / 16777216.0 * ((double)c->zfar - c->znear);
    double xc = (px - c->cx) * z / c->fx, yc = -(py - c->cy) * z / c->fy;
    /* world = eye + R^T (xc, yc, z) */
    X->x = c->eye[0] + (c->R[0] * xc + c->R[3] * yc + c->R[6] * z);
    X->y = c->eye[1] + (c->R[1] * xc + c->R[4] * yc + c->R[7] * z);
    X->z = c->eye[2] + (c->R[2] * xc + c->R[5] * yc + c->R[8] * z);
    double u = (double)((w >> 32) & 0xFFu) / 255.0 * 2.0 - 1.0;
    double v = (double)((w >> 24) & 0xFFu) / 255.0 * 2.0 - 1.0;
    double tz = 1.0 - fabs(u) - fabs(v);
    if (tz < 0.0) {
        double au = fabs(u), av = fabs(v);
        u = (1.0 - av) * (u >= 0.0 ? 1.0 : -1.0);
        v = (1.0 - au) * (v >= 0.0 ? 1.0 : -1.0);
    }
    *T = d3_norm(d3(u, v, tz));
    alb[0] = (double)((w >> 18) & 63u) / 63.0;
    alb[1] = (double)((w >> 12) & 63u) / 63.0;
    alb[2] = (double)((w >> 6) & 63u) / 63.0;
    *ao = (double)(w & 63u) / 63.0;
}

/* Centre-only resolve of a G-buffer visibility buffer (decode, shade, alpha 1
 * over the background; empty and opaque pixels show the background). */
int orc_resolve_gbuf(const uint64_t *vis, const float *cams, uint32_t n_scenes, int width,
                     int height, const orc_shade_params *sp, double *out_rgba)
{
    size_t npix = (size_t)width * height;
    for (uint32_t s = 0; s < n_scenes; ++s) {
        const orc_cam *c = (const orc_cam *)(cams + 18 * (size_t)s);
        const uint64_t *g = vis + (size_t)s * 2 * npix;
        for (int j = 0; j < height; ++j)
            for (int i = 0; i < width; ++i) {
                size_t p = (size_t)j * width + i;
                double *o = out_rgba + ((size_t)s * npix + p) * 4;
                if (!orc_is_hit(g[p])) {
                    o[0] = sp->bg[0]; o[1] = sp->bg[1]; o[2] = sp->bg[2]; o[3] = 0.0;
                    continue;
                }
                v3d X, T;
                double alb[3], ao;
                orc_gbuf_decode(c, g[p], i + 0.5, j + 0.5, &X, &T, alb, &ao);
                orc_shade_point(c, sp, X, T, alb, 1.0, ao, o);
                o[3] = 1.0;
            }
    }
    return 0;
}
