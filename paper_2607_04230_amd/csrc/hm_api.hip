// C ABI of libhm: argument validation, workspace sizing, error reporting.
// Kernels are enqueued on the caller's stream; nothing here synchronises or
// allocates device memory.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "hm_device.hpp"
#include "hm_internal.hpp"

namespace hm {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

uint32_t stride_grid(size_t n, uint32_t block)
{
    size_t g = (n + block - 1) / block;
    const size_t cap = 256u * 16u;        // 256 CUs x 16 resident workgroups
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (uint32_t)g;
}

uint32_t full_grid(size_t n, uint32_t block)
{
    size_t g = (n + block - 1) / block;
    const size_t cap = size_t(1) << 20;  // grid-stride kernels cover what lies beyond
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (uint32_t)g;
}

// ------------------------------------------------------------------ kernel timing
struct TimedRec {
    std::string name;
    hipEvent_t a, b;
};
static std::mutex g_tmu;
static bool g_timing = false;
static std::vector<TimedRec> g_recs;

KTimer::KTimer(const char *name, hipStream_t st) : name_(name), st_(st)
{
    if (!g_timing) return;
    if (hipEventCreate(&a_) != hipSuccess) {
        a_ = nullptr;
        return;
    }
    if (hipEventCreate(&b_) != hipSuccess || hipEventRecord(a_, st_) != hipSuccess) {
        // timing is best effort: a launch that cannot be timed is not recorded
        (void)hipEventDestroy(a_);
        if (b_) (void)hipEventDestroy(b_);
        a_ = b_ = nullptr;
    }
}

KTimer::~KTimer()
{
    if (!a_) return;
    if (hipEventRecord(b_, st_) != hipSuccess) {
        (void)hipEventDestroy(a_);
        (void)hipEventDestroy(b_);
        return;
    }
    std::lock_guard<std::mutex> g(g_tmu);
    g_recs.push_back({name_, a_, b_});
}

}  // namespace hm

using namespace hm;

static thread_local char g_err[512] = "";

static hm_status fail(hm_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

static hm_status ok() { g_err[0] = 0; return HM_OK; }

static hm_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

#define REQUIRE(cond, code, ...) \
    do { if (!(cond)) return fail(code, __VA_ARGS__); } while (0)

static hm_status check_frame(const hm_frame *f)
{
    REQUIRE(f, HM_ERR_INVALID, "frame is NULL");
    REQUIRE(f->n_scenes >= 1, HM_ERR_INVALID, "frame.n_scenes must be >= 1");
    REQUIRE(f->width >= 1 && f->width <= 16384 && f->height >= 1 && f->height <= 16384,
            HM_ERR_RANGE, "frame size %ux%u outside [1, 16384]", f->width, f->height);
    const double pix = (double)f->width * f->height * f->n_scenes;
    REQUIRE(pix < 4.0e9, HM_ERR_RANGE, "frame has too many pixels (%.0f)", pix);
    return HM_OK;
}

static hm_status check_mesh(const hm_hair_mesh *m)
{
    REQUIRE(m, HM_ERR_INVALID, "mesh is NULL");
    REQUIRE(m->layer_pos && m->quads && m->bundle_key && m->bundle_nstrands && m->bundle_cmax &&
                m->bundle_scene,
            HM_ERR_INVALID, "mesh has a NULL array");
    REQUIRE(m->n_bundles >= 1 && m->n_verts >= 1, HM_ERR_INVALID, "mesh has no bundles / vertices");
    REQUIRE(m->n_layers >= 2 && m->n_layers <= 64, HM_ERR_RANGE, "n_layers %u outside [2, 64]",
            m->n_layers);
    return HM_OK;
}

// The stream's extent (scene offsets, scene count, capacity), for calls that
// read no control point.
static hm_status check_stream_bounds(const hm_strands *s)
{
    REQUIRE(s, HM_ERR_INVALID, "strands is NULL");
    REQUIRE(s->scene_off, HM_ERR_INVALID, "strands.scene_off is NULL");
    REQUIRE(s->n_scenes >= 1, HM_ERR_INVALID, "strands.n_scenes must be >= 1");
    REQUIRE(s->cap >= 1 && s->cap < 0xFFFFFFFFu, HM_ERR_RANGE,
            "strands.cap must be in [1, 2^32 - 2]");
    return HM_OK;
}

static hm_status check_strands(const hm_strands *s)
{
    REQUIRE(s, HM_ERR_INVALID, "strands is NULL");
    REQUIRE(s->pos_w && s->rgb && s->flags, HM_ERR_INVALID, "strands has a NULL array");
    return check_stream_bounds(s);
}

static hm_status check_ws(void *ws, size_t have, size_t need)
{
    REQUIRE(have >= need, HM_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", have, need);
    REQUIRE(need == 0 || ws, HM_ERR_INVALID, "workspace is NULL");
    return HM_OK;
}

static hm_status check_raster_params(const hm_raster_params *p)
{
    REQUIRE(p, HM_ERR_INVALID, "raster params NULL");
    REQUIRE(p->algo == HM_RASTER_TILED || p->algo == HM_RASTER_DIRECT ||
                p->algo == HM_RASTER_TILED_ROWS,
            HM_ERR_INVALID, "unknown raster algo %d", p->algo);
    REQUIRE(p->tile == 8 || p->tile == 16 || p->tile == 32, HM_ERR_RANGE,
            "tile must be 8, 16 or 32 (got %u)", p->tile);
    REQUIRE(p->chunk >= 1 && p->chunk <= (1u << 20), HM_ERR_RANGE, "chunk outside [1, 2^20]");
    REQUIRE(p->max_tiles_per_seg >= 1 && p->max_tiles_per_seg <= 64, HM_ERR_RANGE,
            "max_tiles_per_seg outside [1, 64]");
    REQUIRE(p->block >= 64 && p->block <= 1024 && p->block % 64 == 0, HM_ERR_RANGE,
            "block must be a multiple of 64 in [64, 1024]");
    REQUIRE(p->grid <= 65536, HM_ERR_RANGE, "grid outside [0, 65536]");
    REQUIRE(p->shared_views <= 1, HM_ERR_INVALID, "shared_views must be 0 or 1");
    REQUIRE(p->payload == HM_PAYLOAD_SEGMENT || p->payload == HM_PAYLOAD_GBUFFER,
            HM_ERR_INVALID, "unknown payload %u", p->payload);
    REQUIRE(p->payload == HM_PAYLOAD_SEGMENT || !p->shared_views, HM_ERR_INVALID,
            "G-buffer keys need shared_views = 0");
    REQUIRE(p->algo != HM_RASTER_TILED || p->block <= 256, HM_ERR_RANGE,
            "HM_RASTER_TILED takes at most 256 threads per workgroup (got %u)", p->block);
    REQUIRE(p->algo == HM_RASTER_DIRECT || raster_lds_bytes(*p) <= 65536u, HM_ERR_RANGE,
            "tile %u with %u threads needs %u B of LDS (limit 65536)", p->tile, p->block,
            raster_lds_bytes(*p));
    REQUIRE(isfinite(p->r_min) && p->r_min >= 0.0f && p->r_min <= 64.0f, HM_ERR_RANGE,
            "r_min outside [0, 64]");
    return HM_OK;
}

static hm_status make_shade(const hm_shade_params *p, ShadeK &k)
{
    REQUIRE(p, HM_ERR_INVALID, "shade params NULL");
    REQUIRE(p->mode == HM_RESOLVE_FILTER || p->mode == HM_RESOLVE_SOFT ||
                p->mode == HM_RESOLVE_CENTER,
            HM_ERR_INVALID, "unknown resolve mode %d", p->mode);
    REQUIRE(p->filter_radius >= 0 && p->filter_radius <= 8, HM_ERR_RANGE,
            "filter_radius outside [0, 8]");
    REQUIRE(p->spec_squarings >= 0 && p->spec_squarings <= 8, HM_ERR_RANGE,
            "spec_squarings outside [0, 8]");
    REQUIRE(p->s_par > 0 && p->s_perp > 0 && p->sigma_c > 0 && p->iso_scale > 0 &&
                p->soft_sigma > 0,
            HM_ERR_RANGE, "filter / soft sigmas must be > 0");
    REQUIRE(p->depth_reject >= 0 && p->depth_reject < 1 && p->depth_mismatch >= 0 &&
                p->depth_mismatch < 1,
            HM_ERR_RANGE, "depth thresholds outside [0, 1)");
    const double lx = p->light_dir[0], ly = p->light_dir[1], lz = p->light_dir[2];
    const double ln = sqrt(lx * lx + ly * ly + lz * lz);
    REQUIRE(ln > 0, HM_ERR_INVALID, "light_dir is zero");
    k.Lx = (float)(lx / ln); k.Ly = (float)(ly / ln); k.Lz = (float)(lz / ln);
    k.Er = p->light_rgb[0]; k.Eg = p->light_rgb[1]; k.Eb = p->light_rgb[2];
    k.ka = p->ka; k.kd = p->kd; k.ks = p->ks;
    k.nsq = p->spec_squarings;
    k.r = p->filter_radius;
    const double r = p->filter_radius > 0 ? p->filter_radius : 1;
    const double spar = r * p->s_par, sperp = r * p->s_perp, siso = r * p->iso_scale;
    k.inv_spar2 = (float)(1.0 / (spar * spar));
    k.inv_sperp2 = (float)(1.0 / (sperp * sperp));
    k.inv_siso2 = (float)(1.0 / (siso * siso));
    k.inv_sc2 = (float)(1.0 / ((double)p->sigma_c * p->sigma_c));
    // depth thresholds in 24-bit code units: reject |dq| > floor(t 2^24),
    // mismatch when nearer by >= ceil(t 2^24)
    k.dq_rej = (uint32_t)floor((double)p->depth_reject * 16777216.0);
    k.dq_mis = (uint32_t)ceil((double)p->depth_mismatch * 16777216.0);
    REQUIRE(isfinite(p->strip_half) && p->strip_half >= 0.0f && p->strip_half <= 16.0f,
            HM_ERR_RANGE, "strip_half outside [0, 16]");
    const float h = p->strip_half;
    k.strip_half = h;
    k.strip2 = h * h;
    k.iso_len = p->iso_len;
    k.soft_k = (float)(1.0 / ((double)p->soft_sigma * sqrt(2.0)));
    k.bgr = p->bg[0]; k.bgg = p->bg[1]; k.bgb = p->bg[2];
    k.mode = p->mode;
    REQUIRE(!p->shadow || p->mode != HM_RESOLVE_SOFT, HM_ERR_INVALID,
            "shadow applies to the FILTER and CENTER resolves only");
    k.shadow = p->shadow;
    REQUIRE(p->payload == HM_PAYLOAD_SEGMENT || p->payload == HM_PAYLOAD_GBUFFER,
            HM_ERR_INVALID, "unknown payload %d", p->payload);
    REQUIRE(p->payload == HM_PAYLOAD_SEGMENT || (p->mode == HM_RESOLVE_CENTER && !p->shadow),
            HM_ERR_INVALID, "G-buffer keys resolve in CENTER mode only, without shadow");
    k.payload = p->payload;
    return HM_OK;
}

static hm_status check_dom(const hm_dom_params *p)
{
    REQUIRE(p, HM_ERR_INVALID, "dom params NULL");
    hm_frame lf{1, p->width, p->height};
    hm_status st = check_frame(&lf);
    if (st) return st;
    REQUIRE(p->n_layers >= 1 && p->n_layers <= 8, HM_ERR_RANGE, "n_layers %u outside [1, 8]",
            p->n_layers);
    REQUIRE(p->layer_codes >= 1 && p->layer_codes <= 16777216u, HM_ERR_RANGE,
            "layer_codes outside [1, 2^24]");
    REQUIRE(isfinite(p->r_min) && p->r_min >= 0.0f, HM_ERR_RANGE, "r_min must be finite, >= 0");
    REQUIRE(isfinite(p->alpha) && p->alpha > 0.0f, HM_ERR_RANGE, "alpha must be finite, > 0");
    REQUIRE((double)p->width * p->height * p->n_layers < 4.0e9, HM_ERR_RANGE,
            "light map too large");
    return HM_OK;
}

extern "C" {

const char *hm_last_error(void) { return g_err; }

hm_status hm_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> g(g_tmu);
    g_timing = on != 0;
    return ok();
}

hm_status hm_timing_collect(char *buf, size_t len)
{
    REQUIRE(buf && len > 0, HM_ERR_INVALID, "buffer is NULL");
    std::vector<TimedRec> recs;
    {
        std::lock_guard<std::mutex> g(g_tmu);
        recs.swap(g_recs);
    }
    std::map<std::string, std::pair<double, unsigned long>> acc;
    for (auto &r : recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto &e = acc[r.name];
            e.first += ms;
            e.second += 1;
        }
        (void)hipEventDestroy(r.a);   // nothing to do if a destroy fails
        (void)hipEventDestroy(r.b);
    }
    size_t o = 0;
    buf[0] = 0;
    for (auto &kv : acc) {
        int n = snprintf(buf + o, len - o, "%s %.6f %lu\n", kv.first.c_str(), kv.second.first,
                         kv.second.second);
        if (n < 0 || (size_t)n >= len - o) break;
        o += (size_t)n;
    }
    return ok();
}

int32_t hm_version(void) { return 100; }

hm_status hm_raster_defaults(const hm_frame *frame, hm_raster_params *p)
{
    hm_status st = check_frame(frame);
    if (st) return st;
    REQUIRE(p, HM_ERR_INVALID, "params NULL");
    raster_defaults(*frame, *p);
    return ok();
}

hm_status hm_workspace_size(int32_t call, const hm_frame *frame, uint32_t n_bundles, uint32_t cap,
                            const hm_raster_params *p, size_t *bytes)
{
    REQUIRE(bytes, HM_ERR_INVALID, "bytes is NULL");
    hm_status st = check_frame(frame);
    if (st) return st;
    if (call == HM_CALL_LOD) {
        REQUIRE(n_bundles >= 1, HM_ERR_INVALID, "n_bundles must be >= 1");
        *bytes = lod_workspace(n_bundles);
    } else if (call == HM_CALL_RASTER) {
        REQUIRE(cap >= 1 && cap < 0xFFFFFFFFu, HM_ERR_RANGE, "cap outside [1, 2^32 - 2]");
        hm_raster_params d;
        if (!p) { raster_defaults(*frame, d); p = &d; }
        st = check_raster_params(p);
        if (st) return st;
        *bytes = raster_workspace(*frame, cap, *p);
    } else if (call == HM_CALL_GEN_RASTER) {
        REQUIRE(n_bundles >= 1, HM_ERR_INVALID, "n_bundles must be >= 1");
        REQUIRE(cap >= 1 && cap < 0xFFFFFFFFu, HM_ERR_RANGE, "cap outside [1, 2^32 - 2]");
        hm_raster_params d;
        if (!p) { raster_defaults(*frame, d); p = &d; }
        st = check_raster_params(p);
        if (st) return st;
        *bytes = gen_raster_workspace(n_bundles, *frame, cap, *p);
    } else if (call == HM_CALL_RESOLVE) {
        *bytes = resolve_workspace(*frame);
    } else if (call == HM_CALL_DOM) {
        REQUIRE(cap >= 1 && cap < 0xFFFFFFFFu, HM_ERR_RANGE, "cap outside [1, 2^32 - 2]");
        REQUIRE(frame->n_scenes == 1, HM_ERR_INVALID, "the light map frame has one scene");
        *bytes = dom_workspace(*frame, cap);
    } else {
        return fail(HM_ERR_INVALID, "unknown call %d", call);
    }
    return ok();
}

hm_status hm_lod_select(const hm_hair_mesh *mesh, const hm_camera *cams, const hm_frame *frame,
                        const hm_lod_params *p, uint32_t *table, uint32_t *scene_off,
                        uint64_t *totals, void *ws, size_t ws_bytes, void *stream)
{
    hm_status st;
    if ((st = check_mesh(mesh)) || (st = check_frame(frame))) return st;
    REQUIRE(cams && p && table && scene_off && totals, HM_ERR_INVALID, "NULL argument");
    REQUIRE(p->mode == HM_LOD_OFF || p->mode == HM_LOD_ON, HM_ERR_INVALID, "unknown LOD mode %d",
            p->mode);
    REQUIRE(isfinite(p->lambda) && p->lambda >= 0, HM_ERR_RANGE, "lambda must be finite, >= 0");
    if ((st = check_ws(ws, ws_bytes, lod_workspace(mesh->n_bundles)))) return st;
    launch_lod(*mesh, cams, *frame, *p, table, scene_off, totals, ws, (hipStream_t)stream);
    return check_launch("hm_lod_select");
}

hm_status hm_generate_strands(const hm_hair_mesh *mesh, const uint32_t *table,
                              const uint32_t *strand_base, const float *strand_rgb,
                              const hm_gen_params *p, const hm_strands *out, void *stream)
{
    hm_status st;
    if ((st = check_mesh(mesh)) || (st = check_strands(out))) return st;
    REQUIRE(table && p, HM_ERR_INVALID, "NULL argument");
    REQUIRE(!strand_rgb || strand_base, HM_ERR_INVALID, "strand_rgb needs strand_base");
    REQUIRE(isfinite(p->width) && isfinite(p->curl_amp) && isfinite(p->curl_turns) &&
                p->curl_turns >= 0,
            HM_ERR_RANGE, "generation parameters must be finite (curl_turns >= 0)");
    launch_generate(*mesh, table, strand_base, strand_rgb, *p, *out, (hipStream_t)stream);
    return check_launch("hm_generate_strands");
}

hm_status hm_generate_raster(const hm_hair_mesh *mesh, const uint32_t *table,
                             const uint32_t *strand_base, const float *strand_rgb,
                             const hm_gen_params *p, const hm_strands *out,
                             const hm_camera *cams, const hm_frame *frame, float r_min,
                             int32_t payload, const float *scene_z, uint64_t *vis, void *stream)
{
    hm_status st;
    if ((st = check_mesh(mesh)) || (st = check_frame(frame))) return st;
    REQUIRE(payload == HM_PAYLOAD_SEGMENT || payload == HM_PAYLOAD_GBUFFER, HM_ERR_INVALID,
            "unknown payload %d", payload);
    // G-buffer keys write no stream: its arrays may be NULL
    if ((st = payload == HM_PAYLOAD_GBUFFER ? check_stream_bounds(out) : check_strands(out)))
        return st;
    REQUIRE(table && p && cams && vis, HM_ERR_INVALID, "NULL argument");
    REQUIRE(!strand_rgb || strand_base, HM_ERR_INVALID, "strand_rgb needs strand_base");
    REQUIRE(isfinite(p->width) && isfinite(p->curl_amp) && isfinite(p->curl_turns) &&
                p->curl_turns >= 0,
            HM_ERR_RANGE, "generation parameters must be finite (curl_turns >= 0)");
    REQUIRE(out->n_scenes == frame->n_scenes, HM_ERR_INVALID,
            "strands.n_scenes (%u) != frame.n_scenes (%u)", out->n_scenes, frame->n_scenes);
    REQUIRE(isfinite(r_min) && r_min >= 0.0f, HM_ERR_RANGE, "r_min must be finite, >= 0");
    launch_generate_raster(*mesh, table, strand_base, strand_rgb, *p, *out, cams, *frame, r_min,
                           payload, scene_z, vis, (hipStream_t)stream);
    return check_launch("hm_generate_raster");
}

hm_status hm_raster_vis(const hm_strands *s, const hm_camera *cams, const hm_frame *frame,
                        const hm_raster_params *p, const float *scene_z, uint64_t *vis,
                        void *ws, size_t ws_bytes, void *stream)
{
    hm_status st;
    if ((st = check_strands(s)) || (st = check_frame(frame)) || (st = check_raster_params(p)))
        return st;
    REQUIRE(cams && vis, HM_ERR_INVALID, "NULL argument");
    if (p->shared_views) {
        REQUIRE(s->n_scenes == 1, HM_ERR_INVALID, "shared views need a single-scene stream");
    } else {
        REQUIRE(s->n_scenes == frame->n_scenes, HM_ERR_INVALID,
                "strands.n_scenes != frame.n_scenes");
    }
    const double tiles = (double)((frame->width + p->tile - 1) / p->tile) *
                         ((frame->height + p->tile - 1) / p->tile) * frame->n_scenes;
    REQUIRE(tiles < 1.0e9, HM_ERR_RANGE, "too many tiles");
    const double units = (double)s->cap * (p->shared_views ? frame->n_scenes : 1u);
    REQUIRE(units < 4.0e9, HM_ERR_RANGE, "cap * views exceeds 32-bit segment units");
    REQUIRE(units * p->max_tiles_per_seg < 4.0e9, HM_ERR_RANGE,
            "cap * max_tiles_per_seg exceeds 32-bit bin offsets");
    if ((st = check_ws(ws, ws_bytes, raster_workspace(*frame, s->cap, *p)))) return st;
    launch_raster(*s, cams, *frame, *p, scene_z, vis, ws, (hipStream_t)stream);
    return check_launch("hm_raster_vis");
}

hm_status hm_generate_raster_tiled(const hm_hair_mesh *mesh, const uint32_t *table,
                                   const uint32_t *strand_base, const float *strand_rgb,
                                   const hm_gen_params *gp, const hm_strands *out,
                                   const hm_camera *cams, const hm_frame *frame,
                                   const hm_raster_params *p, const float *scene_z,
                                   uint64_t *vis, void *ws, size_t ws_bytes, void *stream)
{
    hm_status st;
    if ((st = check_mesh(mesh)) || (st = check_strands(out)) || (st = check_frame(frame)) ||
        (st = check_raster_params(p)))
        return st;
    REQUIRE(table && gp && cams && vis, HM_ERR_INVALID, "NULL argument");
    REQUIRE(!strand_rgb || strand_base, HM_ERR_INVALID, "strand_rgb needs strand_base");
    REQUIRE(isfinite(gp->width) && isfinite(gp->curl_amp) && isfinite(gp->curl_turns) &&
                gp->curl_turns >= 0,
            HM_ERR_RANGE, "generation parameters must be finite (curl_turns >= 0)");
    REQUIRE(p->algo == HM_RASTER_TILED && p->payload == HM_PAYLOAD_SEGMENT && !p->shared_views,
            HM_ERR_INVALID,
            "generation with binning needs the tiled algorithm, segment ids and one view per "
            "scene");
    REQUIRE(out->n_scenes == frame->n_scenes, HM_ERR_INVALID,
            "strands.n_scenes (%u) != frame.n_scenes (%u)", out->n_scenes, frame->n_scenes);
    const double tiles = (double)((frame->width + p->tile - 1) / p->tile) *
                         ((frame->height + p->tile - 1) / p->tile) * frame->n_scenes;
    REQUIRE(tiles < 1.0e9, HM_ERR_RANGE, "too many tiles");
    REQUIRE((double)out->cap * p->max_tiles_per_seg < 4.0e9, HM_ERR_RANGE,
            "cap * max_tiles_per_seg exceeds 32-bit bin offsets");
    if ((st = check_ws(ws, ws_bytes, gen_raster_workspace(mesh->n_bundles, *frame, out->cap, *p))))
        return st;
    launch_gen_raster_tiled(*mesh, table, strand_base, strand_rgb, *gp, *out, cams, *frame, *p,
                            scene_z, vis, ws, (hipStream_t)stream);
    return check_launch("hm_generate_raster_tiled");
}

hm_status hm_resolve_shade(const hm_strands *s, const uint64_t *vis, const hm_camera *cams,
                           const hm_frame *frame, const hm_shade_params *p, float *out_rgba,
                           void *ws, size_t ws_bytes, void *stream)
{
    hm_status st;
    ShadeK k;
    if ((st = check_frame(frame)) || (st = make_shade(p, k))) return st;
    // a buffer of G-buffer keys is resolved without reading the stream
    if ((st = k.payload == HM_PAYLOAD_GBUFFER ? check_stream_bounds(s) : check_strands(s)))
        return st;
    REQUIRE(vis && cams && out_rgba, HM_ERR_INVALID, "NULL argument");
    if (k.mode == HM_RESOLVE_FILTER) {
        if ((st = check_ws(ws, ws_bytes, resolve_workspace(*frame)))) return st;
    }
    launch_resolve(*s, vis, cams, *frame, k, out_rgba, ws, (hipStream_t)stream);
    return check_launch("hm_resolve_shade");
}

}  // extern "C"

// ------------------------------------------------------------------ no-allocation resolve
// Scratch of hm_resolve_shade_noalloc: the filter's per-pixel records (one
// float4 per pixel), for frames of at most HM_NOALLOC_MAX_PIXELS pixels.  Each
// GPU holds its own copy at its own address; host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address) but the address hipGetSymbolAddress gives for the current device,
// looked up once per device and kept in g_scratch_ptr.
static __device__ __align__(256) float4 scratch[HM_NOALLOC_MAX_PIXELS];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SCRATCH_MAX_DEVICES];

static hm_status scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HM_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    REQUIRE(dev >= 0 && dev < SCRATCH_MAX_DEVICES, HM_ERR_RANGE,
            "device ordinal %d beyond the %d devices the scratch table covers", dev,
            SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(HM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HM_OK;
}

extern "C" {

hm_status hm_resolve_shade_noalloc(const hm_strands *s, const uint64_t *vis,
                                   const hm_camera *cams, const hm_frame *frame,
                                   const hm_shade_params *p, float *out_rgba, void *stream)
{
    hm_status st;
    ShadeK k;
    if ((st = check_frame(frame)) || (st = make_shade(p, k))) return st;
    if ((st = k.payload == HM_PAYLOAD_GBUFFER ? check_stream_bounds(s) : check_strands(s)))
        return st;
    REQUIRE(vis && cams && out_rgba, HM_ERR_INVALID, "NULL argument");
    void *ws = nullptr;
    if (k.mode == HM_RESOLVE_FILTER) {
        const size_t pix = (size_t)frame->width * frame->height * frame->n_scenes;
        REQUIRE(pix <= HM_NOALLOC_MAX_PIXELS, HM_ERR_WORKSPACE,
                "frame of %zu pixels exceeds the %u pixels of the no-allocation scratch", pix,
                HM_NOALLOC_MAX_PIXELS);
        if (resolve_workspace(*frame) > sizeof(float4) * (size_t)HM_NOALLOC_MAX_PIXELS)
            return fail(HM_ERR_WORKSPACE, "resolve records exceed the no-allocation scratch");
        if ((st = scratch_address(&ws))) return st;
    }
    launch_resolve(*s, vis, cams, *frame, k, out_rgba, ws, (hipStream_t)stream);
    return check_launch("hm_resolve_shade_noalloc");
}

hm_status hm_resolve_shade_bwd(const hm_strands *s, const uint64_t *vis, const hm_camera *cams,
                               const hm_frame *frame, const hm_shade_params *p,
                               const float *d_out, float *grad_pos_w, float *grad_rgb,
                               void *stream)
{
    hm_status st;
    ShadeK k;
    if ((st = check_strands(s)) || (st = check_frame(frame)) || (st = make_shade(p, k))) return st;
    REQUIRE(vis && cams && d_out && grad_pos_w && grad_rgb, HM_ERR_INVALID, "NULL argument");
    REQUIRE(k.mode == HM_RESOLVE_SOFT, HM_ERR_INVALID, "backward exists for the SOFT resolve only");
    launch_resolve_bwd(*s, vis, cams, *frame, k, d_out, grad_pos_w, grad_rgb,
                       (hipStream_t)stream);
    return check_launch("hm_resolve_shade_bwd");
}

}  // extern "C"

// ------------------------------------------------------------------ whole frames
struct hm_graph_s {
    hipGraphExec_t exec;
};

extern "C" {

hm_status hm_render_frame(const hm_frame_desc *d, void *stream)
{
    REQUIRE(d, HM_ERR_INVALID, "frame descriptor is NULL");
    hm_status st;
    if ((st = hm_lod_select(&d->mesh, d->cams, &d->frame, &d->lod, d->table,
                            (uint32_t *)d->strands.scene_off, d->totals, d->ws_lod,
                            d->ws_lod_bytes, stream)))
        return st;
    if ((st = hm_generate_strands(&d->mesh, d->table, d->strand_base, d->strand_rgb, &d->gen,
                                  &d->strands, stream)))
        return st;
    if ((st = hm_raster_vis(&d->strands, d->cams, &d->frame, &d->raster, d->scene_z, d->vis,
                            d->ws_raster, d->ws_raster_bytes, stream)))
        return st;
    return hm_resolve_shade(&d->strands, d->vis, d->cams, &d->frame, &d->shade, d->out_rgba,
                            d->ws_resolve, d->ws_resolve_bytes, stream);
}

hm_status hm_graph_create(const hm_frame_desc *d, void *stream, hm_graph *out)
{
    REQUIRE(d && out, HM_ERR_INVALID, "NULL argument");
    REQUIRE(stream, HM_ERR_INVALID, "graph capture needs a non-null stream");
    *out = nullptr;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return fail(HM_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    hm_status rs = hm_render_frame(d, stream);
    char msg[512];
    snprintf(msg, sizeof msg, "%s", g_err);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (rs != HM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(rs, "%s", msg);
    }
    if (e != hipSuccess || !graph)
        return fail(HM_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);       // the executable graph no longer needs it
    if (e != hipSuccess) return fail(HM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    hm_graph g = new (std::nothrow) hm_graph_s{exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        return fail(HM_ERR_INVALID, "out of host memory");
    }
    *out = g;
    return ok();
}

hm_status hm_graph_launch(hm_graph g, void *stream)
{
    REQUIRE(g, HM_ERR_INVALID, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(HM_ERR_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
    return ok();
}

hm_status hm_graph_destroy(hm_graph g)
{
    if (!g) return ok();
    const hipError_t e = hipGraphExecDestroy(g->exec);
    delete g;
    if (e != hipSuccess) return fail(HM_ERR_HIP, "hipGraphExecDestroy: %s", hipGetErrorString(e));
    return ok();
}

}  // extern "C"

extern "C" hm_status hm_lod_depth_offset(const uint32_t *table, const uint32_t *bundle_nstrands,
                                         uint32_t n_bundles, float *delta_out, void *stream)
{
    REQUIRE(table && bundle_nstrands && delta_out, HM_ERR_INVALID, "NULL argument");
    REQUIRE(n_bundles >= 1, HM_ERR_INVALID, "n_bundles must be >= 1");
    hm::launch_lod_delta(table, bundle_nstrands, n_bundles, delta_out, (hipStream_t)stream);
    return check_launch("hm_lod_depth_offset");
}

extern "C" hm_status hm_dom_accumulate(const hm_strands *s, const hm_camera *light,
                                       const hm_dom_params *p, uint64_t *light_vis,
                                       uint32_t *counts, void *ws, size_t ws_bytes, void *stream)
{
    hm_status st;
    if ((st = check_strands(s)) || (st = check_dom(p))) return st;
    REQUIRE(s->n_scenes == 1, HM_ERR_INVALID, "deep opacity maps take a single scene");
    REQUIRE(light && light_vis && counts, HM_ERR_INVALID, "NULL argument");
    const hm_frame lf{1, p->width, p->height};
    if ((st = check_ws(ws, ws_bytes, hm::dom_workspace(lf, s->cap)))) return st;
    hm::launch_dom_accum(*s, light, *p, light_vis, counts, ws, (hipStream_t)stream);
    return check_launch("hm_dom_accumulate");
}

extern "C" hm_status hm_dom_shadow(const hm_strands *s, const uint64_t *vis, const hm_camera *cam,
                                   const hm_frame *frame, const hm_camera *light,
                                   const hm_dom_params *p, const uint64_t *light_vis,
                                   const uint32_t *counts, const uint32_t *table,
                                   const uint32_t *bundle_nstrands, uint32_t n_bundles,
                                   float *shadow, void *stream)
{
    hm_status st;
    if ((st = check_strands(s)) || (st = check_frame(frame)) || (st = check_dom(p))) return st;
    REQUIRE(frame->n_scenes == 1 && s->n_scenes == 1, HM_ERR_INVALID,
            "deep opacity maps take a single scene");
    REQUIRE(vis && cam && light && light_vis && counts && table && bundle_nstrands && shadow,
            HM_ERR_INVALID, "NULL argument");
    REQUIRE(n_bundles >= 1, HM_ERR_INVALID, "n_bundles must be >= 1");
    hm::launch_dom_shadow(*s, vis, cam, *frame, light, *p, light_vis, counts, table,
                          bundle_nstrands, n_bundles, shadow, (hipStream_t)stream);
    return check_launch("hm_dom_shadow");
}
