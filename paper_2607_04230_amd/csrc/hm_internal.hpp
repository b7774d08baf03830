// Host-side launchers shared by the C-ABI layer (hm_api.hip) and the kernel
// translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hm.h"
#include "hm_bin.hpp"

namespace hm {

// Resolve constants prepared on the host.
struct ShadeK {
    float Lx, Ly, Lz;          // normalised direction towards the light
    float Er, Eg, Eb;          // light colour
    float ka, kd, ks;
    int nsq;                   // specular squarings
    int r;                     // filter radius
    float inv_spar2, inv_sperp2, inv_siso2, inv_sc2;
    uint32_t dq_rej, dq_mis;   // depth thresholds in 24-bit code units
    float strip_half;          // strip half width (px)
    float strip2;              // its square (binary32)
    float iso_len;
    float soft_k;              // 1 / (sigma * sqrt(2))
    float bgr, bgg, bgb;
    int mode;
    const float *shadow;       // light transmittance per pixel, or nullptr
    int payload;               // HM_PAYLOAD_SEGMENT or HM_PAYLOAD_GBUFFER keys
};

size_t align_up(size_t x, size_t a = 256);

// LOD + generation
void launch_lod(const hm_hair_mesh &m, const hm_camera *cams, const hm_frame &f,
                const hm_lod_params &p, uint32_t *table, uint32_t *scene_off, uint64_t *totals,
                void *ws, hipStream_t st);
size_t lod_workspace(uint32_t n_bundles);
void launch_lod_delta(const uint32_t *table, const uint32_t *nstr, uint32_t B, float *delta,
                      hipStream_t st);
void launch_generate(const hm_hair_mesh &m, const uint32_t *table, const uint32_t *strand_base,
                     const float *strand_rgb, const hm_gen_params &p, const hm_strands &s,
                     hipStream_t st);

// rasterization
size_t raster_workspace(const hm_frame &f, uint32_t cap, const hm_raster_params &p);
uint32_t raster_lds_bytes(const hm_raster_params &p);   // dynamic LDS of the tile kernel
void raster_defaults(const hm_frame &f, hm_raster_params &p);
void launch_raster(const hm_strands &s, const hm_camera *cams, const hm_frame &f,
                   const hm_raster_params &p, const float *scene_z, uint64_t *vis, void *ws,
                   hipStream_t st);

// resolve
size_t resolve_workspace(const hm_frame &f);
void launch_resolve(const hm_strands &s, const uint64_t *vis, const hm_camera *cams,
                    const hm_frame &f, const ShadeK &k, float *out, void *ws, hipStream_t st);
void launch_resolve_bwd(const hm_strands &s, const uint64_t *vis, const hm_camera *cams,
                        const hm_frame &f, const ShadeK &k, const float *d_out, float *gpos,
                        float *grgb, hipStream_t st);

// strand generation fused with the raster (direct, global atomics)
void launch_prefill(uint64_t *vis, const float *scene_z, const hm_camera *cams,
                    const hm_frame &f, hipStream_t st);
void launch_generate_raster(const hm_hair_mesh &m, const uint32_t *table,
                            const uint32_t *strand_base, const float *strand_rgb,
                            const hm_gen_params &p, const hm_strands &s, const hm_camera *cams,
                            const hm_frame &f, float r_min, int payload, const float *scene_z,
                            uint64_t *vis, hipStream_t st);

// strand generation that also does the tile raster's first binning pass, and
// the tile raster that follows it (single-view frames, tiled algorithm)
uint32_t gen_bundles_per_group(uint32_t n_bundles, uint32_t cap);
uint32_t gen_grid(uint32_t n_bundles, uint32_t cap);
void launch_generate_bin(const hm_hair_mesh &m, const uint32_t *table, const uint32_t *strand_base,
                         const float *strand_rgb, const hm_gen_params &p, const hm_strands &s,
                         const BinK &bk, hipStream_t st);
size_t gen_raster_workspace(uint32_t n_bundles, const hm_frame &f, uint32_t cap,
                            const hm_raster_params &p);
void launch_gen_raster_tiled(const hm_hair_mesh &m, const uint32_t *table,
                             const uint32_t *strand_base, const float *strand_rgb,
                             const hm_gen_params &gp, const hm_strands &s, const hm_camera *cams,
                             const hm_frame &f, const hm_raster_params &p, const float *scene_z,
                             uint64_t *vis, void *ws, hipStream_t st);

// deep-opacity-map shadows
size_t dom_workspace(const hm_frame &light_frame, uint32_t cap);
void launch_dom_accum(const hm_strands &s, const hm_camera *light, const hm_dom_params &p,
                      uint64_t *light_vis, uint32_t *counts, void *ws, hipStream_t st);
void launch_dom_shadow(const hm_strands &s, const uint64_t *vis, const hm_camera *cam,
                       const hm_frame &f, const hm_camera *light, const hm_dom_params &p,
                       const uint64_t *light_vis, const uint32_t *counts, const uint32_t *table,
                       const uint32_t *nstr, uint32_t n_bundles, float *shadow, hipStream_t st);

// number of workgroups for grid-stride kernels
uint32_t stride_grid(size_t n, uint32_t block);
// one thread per item (up to 2^20 workgroups), for latency-bound grid-stride
// kernels that gain from every resident wave having a single item
uint32_t full_grid(size_t n, uint32_t block);

}  // namespace hm

namespace hm {

// Opt-in per-kernel timing (hm_timing_enable): when on, a KTimer records a
// pair of HIP events around one launch on its stream.
struct KTimer {
    KTimer(const char *name, hipStream_t st);
    ~KTimer();
    const char *name_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace hm

// Every kernel launch of the library goes through this macro, so that the
// opt-in timer can bracket it with events on the launch stream.
#undef hipLaunchKernelGGL
#define hipLaunchKernelGGL(kernelName, numBlocks, numThreads, memPerBlock, streamId, ...)      \
    do {                                                                                      \
        ::hm::KTimer hm_kt_(#kernelName, (streamId));                                         \
        kernelName<<<(numBlocks), (numThreads), (memPerBlock), (streamId)>>>(__VA_ARGS__);    \
    } while (0)
