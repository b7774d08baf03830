/*
 * hm.h -- C ABI of libhm, an MI355X (gfx950) implementation of deferred
 * software rasterization of strand hair after Lipp, Jarabo, Wimmer and Bode,
 * "Deferred Software Rasterization for Efficient Real-time Hair Rendering".
 *
 * Pipeline (Sec. 3, pipeline figure): a per-bundle LOD pre-pass produces the
 * dispatch table; strands are generated from the hair mesh; every styled
 * segment is rasterized into two 64-bit visibility layers with an atomic
 * minimum on (depth, segment id); a deferred per-pixel resolve shades the
 * visible segments and reconstructs / filters the strands, or evaluates the
 * differentiable soft-coverage resolve.  Also: deep-opacity-map shadows with
 * the LOD depth correction (hm_dom_accumulate, hm_dom_shadow), the paper's
 * compressed G-buffer keys (hm_raster_params.payload), and generation fused
 * with the raster (hm_generate_raster).
 *
 * General conventions
 *   - Every pointer inside a struct or passed as an array argument is a DEVICE
 *     pointer unless marked "host".  Struct arguments themselves (the hm_*
 *     descriptors) are host pointers read during the call only.
 *   - The caller owns every buffer.  The library never allocates device
 *     memory; scratch space is the caller's workspace (size from
 *     hm_workspace_size).  Nothing is retained between calls, except by
 *     hm_resolve_shade_noalloc, whose scratch is a fixed array inside the
 *     library.
 *   - Every call is asynchronous on `stream` (a hipStream_t, NULL = the null
 *     stream): it validates its arguments on the host, enqueues kernels and
 *     returns; it never synchronises.  Calls are safe to capture in a HIP
 *     graph (no memset nodes, no host reads of device data).
 *   - Return value: HM_OK, or an error code with nothing enqueued for
 *     argument errors.  hm_last_error() gives a message (per host thread).
 *   - Images are row-major, pixel (i, j) = column i, row j, centre at
 *     (i + 0.5, j + 0.5).  A frame holds S scenes ("views") of equal size.
 *   - Counts of strands and control points (CPs) are 32-bit: one call handles
 *     fewer than 2^32 - 1 control points (137 GB of strand stream).
 */
#ifndef HM_H
#define HM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HM_OK = 0,
    HM_ERR_INVALID = 1,   /* null pointer, zero size, bad enum, inconsistent descriptor */
    HM_ERR_RANGE = 2,     /* a size outside the supported range */
    HM_ERR_WORKSPACE = 3, /* workspace smaller than hm_workspace_size() */
    HM_ERR_HIP = 4        /* a HIP launch failed (message in hm_last_error) */
} hm_status;

/* Pinhole camera (Sec. 3.2.1 projects bundles "to screen space").
 * R: world-to-camera rotation, rows = camera right, up, forward.  Camera
 * space has +z forward and +y up; pixel x = cx + fx X/Z, y = cy - fy Y/Z.
 * Depth is normalised linear view depth (Z - znear)/(zfar - znear). */
typedef struct {
    float R[9];
    float eye[3];
    float fx, fy, cx, cy, znear, zfar;
} hm_camera;

/* S scenes of width x height pixels; scene s uses camera s. */
typedef struct {
    uint32_t n_scenes;
    uint32_t width;   /* 1 .. 16384 */
    uint32_t height;  /* 1 .. 16384 */
} hm_frame;

/* Hair mesh (Sec. 2, "Background: Hair mesh rendering"): bundles of n_layers
 * stacked quads, roots on layer 0, tips on layer n_layers - 1.  Bundle b uses
 * the vertices quads[b][0..3] = (A, B, C, D), counter-clockwise, of every
 * layer.  Several scenes may share one mesh: bundle b belongs to scene
 * bundle_scene[b] (non-decreasing in b). */
typedef struct {
    const float *layer_pos;          /* [n_layers][n_verts][3] */
    const uint32_t *quads;           /* [n_bundles][4] vertex indices < n_verts */
    const uint32_t *bundle_key;      /* [n_bundles] hash key: strand k of a bundle is
                                        determined by (seed, key, k) */
    const uint32_t *bundle_nstrands; /* [n_bundles] full strand count N_b */
    const uint32_t *bundle_cmax;     /* [n_bundles] control points per strand: the cap
                                        C_max of eq. cp-lod, or the count when LOD is off;
                                        values below 2 are taken as 2 (a strand has at
                                        least one segment) */
    const uint32_t *bundle_scene;    /* [n_bundles] scene index < n_scenes */
    uint32_t n_bundles;              /* >= 1 */
    uint32_t n_layers;               /* 2 .. 64 */
    uint32_t n_verts;                /* >= 1 */
} hm_hair_mesh;

/* Generated strand stream: control points of all strands, strand after
 * strand, bundle after bundle (table order).  Segment v joins CP v and CP
 * v + 1 when CP v is not a tip.  When scene_off[n_scenes] exceeds cap, the
 * stream is truncated to its first cap CPs and CP cap - 1 is flagged as a
 * tip, so that no call reads past cap. */
typedef struct {
    float *pos_w;               /* [cap][4]: x, y, z (world), width (world units) */
    float *rgb;                 /* [cap][4]: albedo r, g, b, ambient occlusion (1) */
    uint8_t *flags;             /* [cap]: bit0 root CP, bit1 tip CP */
    const uint32_t *scene_off;  /* [n_scenes + 1]: first CP of each scene; scene_off[S] = n_cp */
    uint32_t n_scenes;
    uint32_t cap;               /* host upper bound on n_cp; sizes the launches */
} hm_strands;

/* ------------------------------------------------------------------ LOD */
enum { HM_LOD_OFF = 0, HM_LOD_ON = 1 };

typedef struct {
    int32_t mode;     /* HM_LOD_OFF: N_b strands with bundle_cmax[b] CPs, no culling.
                         HM_LOD_ON: Sec. 3.2.1 / 3.2.2 */
    float lambda;     /* LOD sensitivity (eq. lod-factor) */
    uint32_t seed;    /* per-bundle offset delta ~ U[0,1) of eq. strand-lod */
} hm_lod_params;

/* LOD pre-pass (Sec. 3.2; one thread per bundle as in the paper).  For every
 * bundle: project the quad vertices of all layers, take the screen AABB,
 * L = clamp(|AABB diagonal| / height * lambda, 0, 1) (eq. lod-factor);
 * bundles whose AABB lies outside the viewport, or with every vertex at or
 * behind the near plane, are culled (0 strands); a bundle crossing the near
 * plane gets L = 1.  N_LOD = clamp(ceil(L (N_b + delta)), 1, N_b)
 * (eq. strand-lod); C = min(2^floor(log2(C_raw - 1)) + 1, C_max) with
 * C_raw = max(floor(sqrt(L) C_max), n_layers) (eqs. cp-lod, cp-snap).
 * Outputs (device):
 *   table[n_bundles][4] = {N_LOD, C, first strand, first CP} -- the paper's
 *     one uint4 per bundle, plus the exclusive prefix sums that replace its
 *     indirect dispatch;
 *   scene_off[n_scenes + 1] = first CP of each scene, scene_off[S] = n_cp;
 *   totals[2] = {n_strands, n_cp} (uint64).
 * If n_cp would reach 2^32 - 1 the counts are clamped and totals[1] reports
 * the true count (callers compare it against their cap).
 * ws: hm_workspace_size(HM_CALL_LOD, ...) bytes. */
hm_status hm_lod_select(const hm_hair_mesh *mesh, const hm_camera *cams, const hm_frame *frame,
                        const hm_lod_params *p, uint32_t *table, uint32_t *scene_off,
                        uint64_t *totals, void *ws, size_t ws_bytes, void *stream);

/* Depth correction of Sec. 3.2.3: after stochastic strand removal the
 * remaining fraction beta = N_LOD / N_b of a bundle attenuates like a medium
 * of density sigma * beta (Beer-Lambert), which equals traversing the depth
 * beta * d; expressed as an additive shift in log-depth space,
 * delta = -log(beta).  Writes delta_out[b] (float, device) for every bundle:
 * 0 when nothing was removed, +inf for culled bundles (beta = 0), and 0 for
 * bundles with N_b = 0.  table: hm_lod_select's output. */
hm_status hm_lod_depth_offset(const uint32_t *table, const uint32_t *bundle_nstrands,
                              uint32_t n_bundles, float *delta_out, void *stream);

/* ------------------------------------------------------------------ generation */
typedef struct {
    uint32_t seed;        /* strand (u, v) and curl phase hash seed */
    float width;          /* strand width (world units), written to every CP */
    float curl_amp;       /* styling: curl radius at the tip */
    float curl_turns;     /* styling: turns from root to tip */
    float base_rgb[3];    /* albedo when strand_rgb is NULL */
} hm_gen_params;

/* Strand generation (Sec. 3.1.1, Code 1).  Strand k of bundle b: (u, v) and
 * a curl phase from the PCG hash of (seed, bundle_key[b], k); base points =
 * bilinear interpolation of each layer quad at (u, v); finite-difference unit
 * tangents (Code 1's calcTangent); cubic Hermite between layers with tangents
 * scaled by the interval chord; C CPs uniformly spaced in w in [0, 1]; then
 * the styling f(x): a curl of radius curl_amp * w about the bundle axis.
 * table: the LOD table of hm_lod_select.  strand_base[b]: index of bundle b's
 * first record in strand_rgb ([.][3], per full strand); strand_rgb may be
 * NULL (base_rgb for all).  out->pos_w/rgb/flags receive n_cp CPs;
 * out->scene_off must already hold the LOD output.  Launch shape (the
 * output does not depend on it): one wave per bundle when n_bundles >= 4096
 * or out->cap <= 512 * n_bundles, else one workgroup per bundle. */
hm_status hm_generate_strands(const hm_hair_mesh *mesh, const uint32_t *table,
                              const uint32_t *strand_base, const float *strand_rgb,
                              const hm_gen_params *p, const hm_strands *out, void *stream);

/* ------------------------------------------------------------------ rasterization */
/* Strand generation fused with the raster (Sec. 3.1.1 with 3.1.2: the paper
 * assembles strands and rasterizes their segments in the same workgroup,
 * without a separate pass over a stored stream).  One workgroup or one
 * wave per bundle (the rule of hm_generate_strands) generates its control
 * points exactly as hm_generate_strands, projects each one where it is
 * made, and rasterizes every segment of a finished chunk of strands from LDS
 * with global atomic minima on both layers.  vis receives exactly what
 * hm_raster_vis writes for the same stream and payload (frame->n_scenes
 * scenes, scene of bundle b = mesh->bundle_scene[b]; r_min as
 * hm_raster_params.r_min; scene_z optional as there); no binning, so no
 * workspace.  One view per scene (no shared views).
 * payload = HM_PAYLOAD_SEGMENT: the stream is also written to out (the
 *   resolve reads it back by segment id).
 * payload = HM_PAYLOAD_GBUFFER: the keys carry the compressed G-buffer data
 *   (tangents from the points' neighbours and the strand colour, computed in
 *   LDS) and NOTHING of the stream is written -- out->pos_w, rgb and flags
 *   may be NULL; out->scene_off (the LOD output) and out->cap bound the
 *   points as for any stream.  A CENTER resolve of these keys
 *   (hm_shade_params.payload = HM_PAYLOAD_GBUFFER) reads no stream either:
 *   the paper's stream-free frame. */
hm_status hm_generate_raster(const hm_hair_mesh *mesh, const uint32_t *table,
                             const uint32_t *strand_base, const float *strand_rgb,
                             const hm_gen_params *p, const hm_strands *out,
                             const hm_camera *cams, const hm_frame *frame, float r_min,
                             int32_t payload, const float *scene_z, uint64_t *vis, void *stream);

/* HM_RASTER_TILED: screen tiles resolved in LDS, candidate pixels spread one
 *   per lane (workgroups of at most 256 threads);
 * HM_RASTER_DIRECT: one thread per segment, 64-bit atomics on the buffer;
 * HM_RASTER_TILED_ROWS: screen tiles, each lane walks whole pixel rows. */
enum { HM_RASTER_TILED = 0, HM_RASTER_DIRECT = 1, HM_RASTER_TILED_ROWS = 2 };

/* Low 40 bits of a visibility key.
 * HM_PAYLOAD_SEGMENT: the segment id (the stream index of its first point).
 * HM_PAYLOAD_GBUFFER: the paper's compressed deferred-shading data (Sec.
 *   3.1.2, deferred atomic shading) at the covered point: bits 39..24 the
 *   octahedral code of the tangent (u, v: 8 bits each, each component
 *   rounded from (c + 1) / 2 * 255), bits 23..6 the albedo r, g, b (6 bits
 *   each, rounded from c * 63), bits 5..0 the ambient occlusion (63: none
 *   baked).  Tangent and albedo are the control points' values interpolated
 *   at the perspective-correct segment parameter t3 = ts * (1/z_1) * z of the
 *   closest point (ts) at depth z; the control-point tangent is the resolve's
 *   (central difference, one-sided at root and tip).  The position is not
 *   stored: the resolve rebuilds it from the depth code at the pixel centre.
 *   Depth bits, coverage and the opaque prefill are those of SEGMENT keys;
 *   equal depths break ties by payload.  Needs shared_views = 0 and
 *   strands.rgb. */
enum { HM_PAYLOAD_SEGMENT = 0, HM_PAYLOAD_GBUFFER = 1 };

typedef struct {
    float r_min;              /* minimum coverage half width (px): the centre sample's
                                 "configurable diameter" / 2 (Sec. 3.1.2); 0 = exact width */
    int32_t algo;             /* HM_RASTER_TILED, HM_RASTER_DIRECT or HM_RASTER_TILED_ROWS */
    uint32_t tile;            /* tile edge in pixels: 8, 16 or 32 */
    uint32_t chunk;           /* segments per work item of a tile (>= 1) */
    uint32_t max_tiles_per_seg; /* K: segments touching more than min(K, 24) tiles take
                                   the direct path (1..64) */
    uint32_t block;           /* threads per workgroup: a multiple of 64 in [64, 1024]
                                 (at most 256 for HM_RASTER_TILED); the tile kernel's LDS
                                 (layers + per-lane records) must stay within 64 KiB */
    uint32_t grid;            /* persistent workgroups (0 = auto) */
    uint32_t shared_views;    /* 0: scene s draws its own stream range scene_off[s..s+1];
                                 1: multiview -- one stream (strands.n_scenes = 1) drawn
                                 into every scene of the frame, each with its camera */
    uint32_t payload;         /* HM_PAYLOAD_SEGMENT (default) or HM_PAYLOAD_GBUFFER */
} hm_raster_params;

/* Visibility buffer (Sec. 3.1.2).  vis[s][0] = centre-sample layer,
 * vis[s][1] = conservative layer, each [height][width] uint64.  Key of a
 * segment v at pixel p: depth24 << 40 | v, where depth24 is the 24-bit
 * truncated normalised linear depth at the segment point closest to the
 * pixel centre (perspective-correct through 1/z); empty = 2^64 - 1.
 * Centre layer: the pixel centre lies within max(w(t)/2, r_min) of the
 * projected segment with the perpendicular foot at t in [0, 1).
 * Conservative layer: the segment meets the pixel square dilated by
 * max(max(w0, w1)/2, r_min).  vis[s][l][p] = min(prefill, keys of covering
 * segments); results are bit-identical for every tuning parameter.
 * scene_z (optional, [S][height][width] float): linear view depth of the
 * opaque scene (Sec. 3's existing depth buffer); pixels with znear < z < zfar
 * are prefilled with depth24(z) << 40 | (2^40 - 2) for early rejection.
 * ws: hm_workspace_size(HM_CALL_RASTER, ...) bytes. */
hm_status hm_raster_vis(const hm_strands *s, const hm_camera *cams, const hm_frame *frame,
                        const hm_raster_params *p, const float *scene_z, uint64_t *vis,
                        void *ws, size_t ws_bytes, void *stream);

/* Strand generation (Sec. 3.1.1) and the tiled raster (Sec. 3.1.2) in one
 * call, the generator binning as it assembles: each workgroup of
 * hm_generate_strands also projects every control point it makes and files
 * every segment of its finished strands into its screen tiles (tile box,
 * separating-axis test, per-workgroup LDS table of (segment, tile) counts),
 * which replaces the raster's first pass over the stored stream; the tile
 * lists are then filled and the tiles rasterized as by hm_raster_vis.  The
 * stream written to out and vis are exactly those of hm_generate_strands
 * followed by hm_raster_vis with the same arguments.  Requires p->algo =
 * HM_RASTER_TILED, p->payload = HM_PAYLOAD_SEGMENT, p->shared_views = 0 and
 * out->n_scenes = frame->n_scenes (else HM_ERR_INVALID).  Arguments as for
 * those two calls; ws: hm_workspace_size(HM_CALL_GEN_RASTER, frame,
 * mesh->n_bundles, out->cap, p) bytes. */
hm_status hm_generate_raster_tiled(const hm_hair_mesh *mesh, const uint32_t *table,
                                   const uint32_t *strand_base, const float *strand_rgb,
                                   const hm_gen_params *gp, const hm_strands *out,
                                   const hm_camera *cams, const hm_frame *frame,
                                   const hm_raster_params *p, const float *scene_z,
                                   uint64_t *vis, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ resolve */
enum { HM_RESOLVE_FILTER = 0, HM_RESOLVE_SOFT = 1, HM_RESOLVE_CENTER = 2 };

typedef struct {
    float light_dir[3];    /* towards the directional light (normalised internally) */
    float light_rgb[3];
    float ka, kd, ks;      /* ambient, Kajiya-Kay diffuse, specular weights */
    int32_t spec_squarings;/* specular (1 - (T.H)^2)^(2^n), 0 .. 8 */
    int32_t filter_radius; /* r of the (2r+1)^2 window (Sec. 3.3.1), 0 .. 8 */
    float s_par, s_perp;   /* sigma_par = r s_par, sigma_perp = r s_perp */
    float sigma_c;         /* colour similarity sigma */
    float iso_scale;       /* isotropic fallback sigma_iso = iso_scale r */
    float depth_reject;    /* neighbour depth rejection threshold (normalised depth) */
    float depth_mismatch;  /* centre vs conservative depth mismatch (normalised depth) */
    float strip_half;      /* alpha strip half width in px, [0, 16] (Sec. 3.3.3) */
    float iso_len;         /* screen tangent shorter than this (px) -> isotropic */
    float soft_sigma;      /* soft coverage: std of the Gaussian pixel filter (px) */
    float bg[3];           /* background the result is composited over */
    int32_t mode;          /* HM_RESOLVE_FILTER / HM_RESOLVE_SOFT / HM_RESOLVE_CENTER */
    const float *shadow;   /* optional (device, [S][height][width]): the light's
                              transmittance at each pixel's shaded point (from
                              hm_dom_shadow); scales the diffuse and specular
                              terms of the centre shading.  NULL: unshadowed */
    int32_t payload;       /* what vis holds: HM_PAYLOAD_SEGMENT, or HM_PAYLOAD_GBUFFER
                              (CENTER mode only, no shadow): each centre-hit pixel is
                              shaded from its decoded key -- position rebuilt at the
                              pixel centre from the middle of its depth code's
                              interval, unit tangent from the octahedral code,
                              albedo and AO (which scales the ambient term) from
                              their 6-bit codes -- with no read of the stream (its
                              arrays may then be NULL; scene_off and cap are
                              still checked) */
} hm_shade_params;

/* Deferred resolve, out_rgba[S][height][width][4] float (straight colour
 * composited over bg, alpha in .w).
 * FILTER (Sec. 3.3, 3.4, Code 2): centre pixels are shaded once (Kajiya-Kay
 * diffuse + specular, one directional light); each hair pixel is then
 * reconstructed with the elliptical bilateral filter over centre hits within
 * the depth threshold, conservative-only pixels are promoted (colour term off),
 * a nearer conservative strand (depth mismatch) is blended over the centre
 * hit with alpha 1, and alpha = centre hits / all hits in the tangent strip.
 * CENTER: plain 1-spp deferred shading of the centre layer.
 * SOFT: coverage of the visible segment (centre layer first) under a Gaussian
 * pixel filter, alpha = Phi((d + w/2)/s) - Phi((d - w/2)/s), composited over bg.
 * ws: hm_workspace_size(HM_CALL_RESOLVE, ...) bytes. */
hm_status hm_resolve_shade(const hm_strands *s, const uint64_t *vis, const hm_camera *cams,
                           const hm_frame *frame, const hm_shade_params *p, float *out_rgba,
                           void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * resolve of hm_resolve_shade without a workspace argument.  Same arguments
 * (minus ws), kernels and results.  The FILTER mode's per-pixel records (16
 * B per pixel, written by the centre shading before the filter reads them,
 * so nothing has to start at zero) live in a scratch array inside the
 * library of HM_NOALLOC_MAX_PIXELS records (64 MiB), which every GPU the
 * library runs on holds until the process ends; CENTER and SOFT use none.
 * A FILTER frame with more than HM_NOALLOC_MAX_PIXELS pixels
 * (n_scenes * width * height) is rejected with HM_ERR_WORKSPACE before
 * anything is enqueued.  Nothing is allocated.  `stream` must belong to the
 * current device; the first call on each device looks up that device's copy
 * of the array (HM_ERR_HIP if the lookup fails), so make it outside graph
 * capture.  All calls on one GPU share its array and it keeps the last
 * call's contents: calls that overlap on one GPU (different streams, or
 * graphs replayed concurrently) race, and callers must serialise them. */
#define HM_NOALLOC_MAX_PIXELS 4194304u
hm_status hm_resolve_shade_noalloc(const hm_strands *s, const uint64_t *vis,
                                   const hm_camera *cams, const hm_frame *frame,
                                   const hm_shade_params *p, float *out_rgba, void *stream);

/* Backward of the SOFT resolve with the visibility held fixed: given
 * d_out = dLoss/d out_rgba ([S][H][W][4]), ACCUMULATES dLoss/d pos_w into
 * grad_pos_w[cap][4] (x, y, z, width) and dLoss/d rgb into grad_rgb[cap][4]
 * (.w untouched).  Callers zero the gradients first. */
hm_status hm_resolve_shade_bwd(const hm_strands *s, const uint64_t *vis, const hm_camera *cams,
                               const hm_frame *frame, const hm_shade_params *p,
                               const float *d_out, float *grad_pos_w, float *grad_rgb,
                               void *stream);

/* ------------------------------------------------------------------ shadows */
/* Deep-opacity-map shadows (Sec. 3.4, which cites Yuksel & Keyser 2008 for
 * the map) queried with the LOD depth correction of Sec. 3.2.3.  Single
 * scene.  The light is a pinhole camera; hm_dom_accumulate rasterizes the
 * stream from it (as hm_raster_vis does for frame {1, width, height}, no
 * scene depth, r_min below) into light_vis, whose conservative layer gives
 * the nearest fragment q0 of every light pixel, and then counts the
 * fragments behind q0 per layer. */
typedef struct {
    uint32_t width, height;  /* light map resolution */
    uint32_t n_layers;       /* layers behind the nearest fragment, 1 .. 8 */
    uint32_t layer_codes;    /* layer thickness in 24-bit depth-code units, >= 1 */
    float r_min;             /* fragment coverage half width in the light view (px) */
    float alpha;             /* opacity of one fragment (> 0) */
} hm_dom_params;

/* light_vis[2][height][width] (uint64, device, overwritten): the light
 * view's visibility buffer.  counts[n_layers][height][width] (uint32,
 * device, overwritten): every (segment, light pixel) pair accepted by the
 * conservative test, at depth code q, adds 1 to layer
 * min((q - q0) / layer_codes, n_layers - 1) of its pixel (exact and
 * order-independent).  ws: hm_workspace_size(HM_CALL_DOM, {1, width,
 * height}, 0, cap, NULL) bytes; the light view's bins are built there and
 * walked twice (visibility, then counts). */
hm_status hm_dom_accumulate(const hm_strands *s, const hm_camera *light, const hm_dom_params *p,
                            uint64_t *light_vis, uint32_t *counts, void *ws, size_t ws_bytes,
                            void *stream);

/* shadow[height][width] (float, device) of the camera frame `frame` (one
 * scene) with visibility vis: for a pixel with a centre hit, the shaded point
 * (as the resolve computes it, binary64) is projected by the light camera to
 * a light pixel and a depth code q; the LOD correction moves it towards the
 * light inside the groom, q' = q0 + (uint32)((float)(q - q0) * beta) with
 * beta = N_LOD / N_b of its bundle (table and bundle_nstrands as given to
 * and returned by hm_lod_select), which shifts the log of its depth below q0
 * by Delta = -log beta; the opacity in front of q' is the counts of the
 * layers before it plus the linearly interpolated part of its own layer (the
 * last layer is taken whole once passed), and shadow = exp(-alpha *
 * opacity).  Other pixels, and points outside the light frustum or map, get
 * 1.  Pass the result as hm_shade_params.shadow. */
hm_status hm_dom_shadow(const hm_strands *s, const uint64_t *vis, const hm_camera *cam,
                        const hm_frame *frame, const hm_camera *light, const hm_dom_params *p,
                        const uint64_t *light_vis, const uint32_t *counts,
                        const uint32_t *table, const uint32_t *bundle_nstrands,
                        uint32_t n_bundles, float *shadow, void *stream);

/* ------------------------------------------------------------------ workspace */
enum { HM_CALL_LOD = 0, HM_CALL_RASTER = 1, HM_CALL_RESOLVE = 2, HM_CALL_DOM = 3,
       HM_CALL_GEN_RASTER = 4 };

/* Workspace bytes for `call`.  n_bundles (LOD, GEN_RASTER) and cap (raster,
 * GEN_RASTER) size it; raster params may be NULL (defaults).  Returns
 * HM_ERR_RANGE on overflow. */
hm_status hm_workspace_size(int32_t call, const hm_frame *frame, uint32_t n_bundles,
                            uint32_t cap, const hm_raster_params *p, size_t *bytes);

/* Default raster parameters for a frame. */
hm_status hm_raster_defaults(const hm_frame *frame, hm_raster_params *p);

/* ------------------------------------------------------------------ whole frames */
/* Everything one frame needs: the arguments of the four calls above.  Several
 * scenes (views / characters of uneven strand counts and LOD levels) are one
 * frame with frame.n_scenes > 1: every kernel then covers all scenes in one
 * launch, and the raster's persistent workgroups pull (scene tile, chunk)
 * work items from one device queue (the paper renders grooms one after the
 * other, Sec. 4; batching is an extension). */
typedef struct {
    hm_hair_mesh mesh;
    const hm_camera *cams;             /* [n_scenes] */
    hm_frame frame;
    hm_lod_params lod;
    uint32_t *table;                   /* [n_bundles][4] */
    void *ws_lod;
    size_t ws_lod_bytes;
    const uint32_t *strand_base;
    const float *strand_rgb;
    hm_gen_params gen;
    hm_strands strands;                /* strands.scene_off must be the LOD call's scene_off */
    uint64_t *totals;                  /* [2] */
    hm_raster_params raster;
    const float *scene_z;
    uint64_t *vis;
    void *ws_raster;
    size_t ws_raster_bytes;
    hm_shade_params shade;
    float *out_rgba;
    void *ws_resolve;
    size_t ws_resolve_bytes;
} hm_frame_desc;

/* Enqueue hm_lod_select, hm_generate_strands, hm_raster_vis and
 * hm_resolve_shade for one frame on `stream`. */
hm_status hm_render_frame(const hm_frame_desc *d, void *stream);

/* A frame captured once into a HIP graph and replayed with one launch.  The
 * graph records the descriptor's device pointers: the buffers must outlive it
 * and keep their addresses; their contents may change between launches.
 * `stream` must not be the null stream.  hm_graph_create captures (it
 * enqueues nothing); hm_graph_launch replays on any stream. */
typedef struct hm_graph_s *hm_graph;
hm_status hm_graph_create(const hm_frame_desc *d, void *stream, hm_graph *out);
hm_status hm_graph_launch(hm_graph g, void *stream);
hm_status hm_graph_destroy(hm_graph g);

/* ------------------------------------------------------------------ profiling */
/* Opt-in kernel timing for benchmarks: while enabled, every kernel the
 * library launches is bracketed by two HIP events on its stream (do not
 * enable while capturing a graph).  hm_timing_collect waits for the recorded
 * events, writes one line "kernel total_ms launches" per kernel into buf
 * (host, len bytes, NUL-terminated, truncated if short) and forgets them. */
hm_status hm_timing_enable(int32_t on);
hm_status hm_timing_collect(char *buf, size_t len);

/* Message of the last error on this host thread ("" if none). */
const char *hm_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t hm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HM_H */
