// Visibility-buffer rasterization (Sec. 3.1.2) for gfx950.
//
// The paper draws every styled segment with a DDA line and a 64-bit
// image atomicMin per pixel and layer.  Here:
//   1. k_prefill writes both layers (empty or the opaque scene depth);
//   2. each control point's screen record is computed once, by the first
//      binning pass (or by k_project on the direct path, or by the strand
//      generator when it bins as it assembles);
//   3. TILED path: k_bin pass 0 finds each segment's screen tiles (T x T
//      pixels), stores them as an 8-byte record and counts (segment, tile)
//      pairs in LDS tables flushed once per (span, tile); an exclusive scan
//      turns counts into offsets and each tile is cut into work items of
//      `chunk` segments; pass 1 (or k_bin_spans after the generator's
//      counting) walks the records and scatters the segment ids into the
//      per-tile lists;
//   4. k_raster_flat is a persistent kernel: each workgroup pulls work items
//      from a device counter, keeps the tile's two layers in LDS, resolves all
//      coverage with LDS ds_min_u64, then merges the touched pixels into the
//      global buffer with one 64-bit atomic min each (plain stores when the
//      tile is a single work item);
//   5. segments touching more than min(max_tiles_per_seg, 24) tiles go to a
//      list rasterized by k_raster_long (one wave per segment, global atomics).
// The DIRECT path (one thread per segment, global atomics everywhere) is kept
// as the reference launch shape.  Every path evaluates the same binary32
// predicates per pixel, and min is order-independent, so the buffer is
// bit-identical across paths and tuning parameters.  The same kernels also
// build compressed G-buffer keys (depth | tangent, albedo, AO; k_cp_tangent
// supplies the per-point tangents) and, for deep-opacity-map shadows, walk
// a light view's work items a second time to count fragments per layer.
#include <algorithm>
#include <type_traits>

#include "hm_bin.hpp"
#include "hm_device.hpp"
#include "hm_internal.hpp"
#include "hm_scan.hpp"

namespace hm {


// ------------------------------------------------------------------ prefill
// Prefill of both layers by block (bx, by) of an nbx x nby grid: the grid's
// rows take scenes (all scenes of a frame at once, no division per pixel),
// two pixels per 16-byte store when the scene has an even pixel count and the
// buffers are aligned.
__device__ __forceinline__ void prefill_pixels(uint64_t *vis, const float *scene_z,
                                               const hm_camera *cams, uint32_t S, uint32_t W,
                                               uint32_t H, uint32_t bx, uint32_t nbx,
                                               uint32_t by, uint32_t nby)
{
    const size_t hw = (size_t)W * H;
    const size_t tid = bx * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)nbx * blockDim.x;
    for (uint32_t s = by; s < S; s += nby) {
        const float *zs = scene_z ? scene_z + (size_t)s * hw : nullptr;
        const float zn = cams[s].znear, zf = cams[s].zfar;
        const float inv_range = 1.0f / (zf - zn);
        auto key_of = [&](float z) -> uint64_t {
            return (z > zn && z < zf)
                       ? ((uint64_t)depth_code(z, zn, inv_range) << HM_ID_BITS) | HM_ID_OPAQUE
                       : HM_EMPTY;
        };
        uint64_t *base = vis + (size_t)s * 2 * hw;
        const bool pairs = (hw & 1) == 0 && ((uintptr_t)vis & 15u) == 0 &&
                           ((uintptr_t)scene_z & 7u) == 0;
        if (pairs) {
            for (size_t q = tid; q < hw / 2; q += stride) {
                uint64_t k0 = HM_EMPTY, k1 = HM_EMPTY;
                if (zs) {
                    const float2 z2 = reinterpret_cast<const float2 *>(zs)[q];
                    k0 = key_of(z2.x);
                    k1 = key_of(z2.y);
                }
                const ulonglong2 kk = make_ulonglong2(k0, k1);
                reinterpret_cast<ulonglong2 *>(base)[q] = kk;
                reinterpret_cast<ulonglong2 *>(base + hw)[q] = kk;
            }
        } else {
            for (size_t loc = tid; loc < hw; loc += stride) {
                const uint64_t key = zs ? key_of(zs[loc]) : HM_EMPTY;
                base[loc] = key;
                base[hw + loc] = key;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_prefill(uint64_t *vis, const float *scene_z,
                                                 const hm_camera *cams, uint32_t S, uint32_t W,
                                                 uint32_t H, uint32_t *clr0, uint32_t n0,
                                                 uint32_t *clr1, uint32_t n1)
{
    // also zero the binning counters of this call (saves separate fill launches)
    if (blockIdx.y == 0) {
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n0 || i < n1;
             i += gridDim.x * blockDim.x) {
            if (i < n0) clr0[i] = 0u;
            if (i < n1) clr1[i] = 0u;
        }
    }
    prefill_pixels(vis, scene_z, cams, S, W, H, blockIdx.x, gridDim.x, blockIdx.y, gridDim.y);
}

// The prefill as extra workgroups of the first binning pass (which neither
// reads nor writes the buffer), so that it overlaps the binning.
struct PrefillK {
    uint64_t *vis;
    const float *scene_z;
    uint32_t per, rows;     // the prefill grid (per x rows workgroups)
};

// ------------------------------------------------------------------ projection
__global__ __launch_bounds__(256) void k_project(const float4 *pos_w, const uint32_t *scene_off,
                                                 RasterK rk, const hm_camera *cams, uint32_t cap,
                                                 float4 *proj)
{
    const uint32_t n = stream_len(scene_off, rk, cap);
    const uint32_t nu = unit_count(n, rk);
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nu;
         u += gridDim.x * blockDim.x) {
        uint32_t s, v;
        unit_map(scene_off, rk, n, u, s, v);
        const Cam cam = load_cam(cams + s);
        proj[u] = project(cam, pos_w[v]);
    }
}

// ------------------------------------------------------------------ helpers
// Segment of unit u (stream point v): v must not be a tip; both screen
// records must be inside the depth range.
__device__ __forceinline__ bool load_seg(const float4 *proj, const uint8_t *flags, uint32_t u,
                                         uint32_t v, uint32_t n_cp, float r_min, Seg &sg)
{
    if (v + 1 >= n_cp || (flags[v] & HM_TIP)) return false;
    const float4 a = proj[u], b = proj[u + 1];
    if (a.w == 0.0f || b.w == 0.0f) return false;
    sg = make_seg(a, b, r_min);
    return true;
}

// Stream inputs of one bin entry's segment (unit u, stream point v): loaded
// one batch ahead by the tile raster.  proj[u + 1] is read only when v + 1 is
// a stream point; seg_from gives what load_seg gives for the same unit.
struct EntryIn {
    float4 a, b;
    uint32_t v;
    uint8_t f;
};

__device__ __forceinline__ EntryIn entry_load(const float4 *proj, const uint8_t *flags,
                                              const uint32_t *scene_off, const RasterK &rk,
                                              uint32_t n, uint32_t u)
{
    EntryIn in;
    uint32_t s;
    unit_map(scene_off, rk, n, u, s, in.v);
    in.f = flags[in.v];
    in.a = in.b = make_float4(0.f, 0.f, 0.f, 0.f);
    if (in.v + 1 < n) {
        in.a = proj[u];
        in.b = proj[u + 1];
    }
    return in;
}

__device__ __forceinline__ bool seg_from(const EntryIn &in, uint32_t n_cp, float r_min, Seg &sg)
{
    if (in.v + 1 >= n_cp || (in.f & HM_TIP)) return false;
    if (in.a.w == 0.0f || in.b.w == 0.0f) return false;
    sg = make_seg(in.a, in.b, r_min);
    return true;
}

__device__ __forceinline__ void scene_depth_consts(const hm_camera *cams, uint32_t s, float &zn,
                                                   float &inv_range)
{
    zn = cams[s].znear;
    inv_range = 1.0f / (cams[s].zfar - zn);
}

// ------------------------------------------------------------------ direct path
template <bool GB>
__global__ __launch_bounds__(256) void k_raster_direct(const float4 *proj, const uint8_t *flags,
                                                       const uint32_t *scene_off,
                                                       const hm_camera *cams, RasterK rk,
                                                       uint32_t cap, uint64_t *vis, GbK gk)
{
    const uint32_t n = stream_len(scene_off, rk, cap);
    const uint32_t nu = unit_count(n, rk);
    const size_t hw = (size_t)rk.W * rk.H;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nu;
         u += gridDim.x * blockDim.x) {
        uint32_t s, v;
        unit_map(scene_off, rk, n, u, s, v);
        Seg sg;
        if (!load_seg(proj, flags, u, v, n, rk.r_min, sg)) continue;
        int i0, i1, j0, j1;
        if (!seg_box(sg, rk.W, rk.H, i0, i1, j0, j1)) continue;
        float zn, inv_range;
        scene_depth_consts(cams, s, zn, inv_range);
        uint64_t *vc = vis + (size_t)s * 2 * hw, *va = vc + hw;
        for (int j = j0; j <= j1; ++j) {
            int a0, a1;
            row_span(sg, j, a0, a1);
            a0 = a0 > i0 ? a0 : i0;
            a1 = a1 < i1 ? a1 : i1;
            for (int i = a0; i <= a1; ++i) {
                uint32_t q;
                bool cc, ca;
                float ts, z;
                const bool msk = cover_tz(sg, i, j, rk.r_min, zn, inv_range, cc, ca, q, ts, z);
                if (!msk) continue;
                const uint64_t low =
                    GB ? gb_payload(gk.tan, gk.rgb, v, ts, z, sg.iz1) : (uint64_t)v;
                const uint64_t key = ((uint64_t)q << HM_ID_BITS) | low;
                const size_t p = (size_t)j * rk.W + i;
                if (cc) atomicMin((unsigned long long *)(vc + p), (unsigned long long)key);
                if (ca) atomicMin((unsigned long long *)(va + p), (unsigned long long)key);
            }
        }
    }
}

// ------------------------------------------------------------------ G-buffer tangents
// Unit tangent of every stream point for the compressed G-buffer keys, as the
// resolve computes it: root -> next, tip <- previous, else the central
// difference; zero for a point that is both root and tip (no segment).
__global__ __launch_bounds__(256) void k_cp_tangent(const float4 *pos, const uint8_t *flags,
                                                    const uint32_t *scene_off, RasterK rk,
                                                    uint32_t cap, float4 *tan)
{
    const uint32_t n = stream_len(scene_off, rk, cap);
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += gridDim.x * blockDim.x) {
        const uint8_t f = flags[v];
        const float4 a = (f & HM_ROOT) ? pos[v] : pos[v - 1];
        const float4 b = (f & HM_TIP) ? pos[v] : pos[v + 1];
        const float4 t = cp_unit_tangent(a, b, (f & HM_ROOT) && (f & HM_TIP));
        tan[v] = t;
    }
}

// ------------------------------------------------------------------ binning

// Stream inputs of one unit's segment.  The binning loads them one step
// ahead, so that their latency overlaps the previous segment's tile work.
struct SegIn {
    float4 p0, p1;      // control points v and v + 1 (world)
    uint32_t s, v;      // scene, stream index
    uint8_t f;          // flags of v
    bool live;          // u < unit count
};

__device__ __forceinline__ SegIn seg_load(const float4 *pos_w, const uint8_t *flags,
                                          const uint32_t *scene_off, const RasterK &rk,
                                          uint32_t u, uint32_t n)
{
    SegIn in;
    in.live = u < unit_count(n, rk);
    in.s = 0;
    in.v = 0;
    in.f = 0;
    in.p0 = in.p1 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (in.live) {
        unit_map(scene_off, rk, n, u, in.s, in.v);
        in.p0 = pos_w[in.v];
        in.f = flags[in.v];
        if (in.v + 1 < n) in.p1 = pos_w[in.v + 1];
    }
    return in;
}

// The unit's screen record (stored in proj[u]), and, when it starts a
// segment, the segment's tile box.
__device__ __forceinline__ bool seg_tiles(const SegIn &in, const hm_camera *cams, float4 *proj,
                                          const RasterK &rk, uint32_t u, uint32_t n,
                                          SegTiles &st)
{
    st.nt = 0;
    if (!in.live) return false;
    const Cam cam = load_cam(cams + in.s);
    const float4 a = project(cam, in.p0);
    proj[u] = a;
    if (in.v + 1 >= n || (in.f & HM_TIP)) return false;
    return seg_tiles_of(a, project(cam, in.p1), in.s, rk, st);
}


#ifndef HM_BIN_SUB
#define HM_BIN_SUB 8
#endif
#ifndef HM_BIN_BLOCK
#define HM_BIN_BLOCK 512
#endif
#ifndef HM_BIN_WGS
#define HM_BIN_WGS 1024
#endif
constexpr uint32_t BIN_SUB = HM_BIN_SUB;      // most segments per thread between table flushes
// threads per binning workgroup: 512 measured 33.1 against 34.5 us per pass on
// the full head and 419 against 435 us on the 64-scene batch (1024: 46 and
// 520 us)
constexpr uint32_t BIN_BLOCK = HM_BIN_BLOCK;
static_assert(BIN_BLOCK % 64 == 0 && BIN_BLOCK <= 1024, "binning workgroups are whole waves");
constexpr uint32_t BIN_WGS = HM_BIN_WGS;      // workgroups the segments are spread over (at least)

// Per-tile segment lists.  Each workgroup takes nsub * blockDim consecutive
// segments (a "span"; consecutive segments belong to the same few strands, so
// they fall in a few tiles) and aggregates its (segment, tile) pairs per tile
// in an LDS table:
//   pass 0: projects the control points (screen records), finds each
//           segment's tiles (tile box + separating-axis test) and stores them
//           as one 8-byte record per segment: the first tile of its box, the
//           box width and a bit mask of the accepted tiles (segments with
//           more than BIN_KMAX or K tiles go to the long list); counts pairs
//           per tile in the table, flushes them with one non-returning
//           global add per (span, tile) and saves the table's occupied
//           slots (slot, tile, count);
//   pass 1: restores the span's table, reserves a range of each tile's list
//           with one returning global add per (span, tile), then walks the
//           segment records and gives each pair an LDS-atomic rank inside
//           its range -- no screen record is read again.
// Pairs that found the table full go straight to global counters in both
// passes.

__global__ __launch_bounds__(BIN_BLOCK) void k_bin(int pass, float4 *proj, const float4 *pos_w,
                                                   const hm_camera *cams, const uint8_t *flags,
                                                   const uint32_t *scene_off, RasterK rk,
                                                   uint32_t cap, uint32_t *tile_cnt,
                                                   const uint32_t *tile_off, uint32_t *tile_cur,
                                                   uint32_t *entries, uint32_t *long_list,
                                                   uint32_t *counters, uint32_t nsub,
                                                   uint2 *segrec, uint32_t *saved,
                                                   const uint32_t *item_off, uint32_t *item_tile,
                                                   uint32_t max_items, uint32_t nbin, PrefillK pf)
{
    __shared__ uint32_t keys[BIN_SLOTS], cnt[BIN_SLOTS], basev[BIN_SLOTS];
    __shared__ uint32_t sh_nsave;
    if (blockIdx.x >= nbin) {
        // a prefill workgroup
        const uint32_t b = blockIdx.x - nbin;
        const uint32_t by = b / pf.per;
        prefill_pixels(pf.vis, pf.scene_z, cams, rk.S, rk.W, rk.H, b - by * pf.per, pf.per, by,
                       pf.rows);
        return;
    }
    const uint32_t n = stream_len(scene_off, rk, cap);
    const uint32_t nu = unit_count(n, rk);
    const uint32_t span = BIN_BLOCK * nsub;        // segments per table flush
    const uint32_t kmax = rk.K < BIN_KMAX ? rk.K : BIN_KMAX;
    if (pass == 1) {
        // the tile of every work item of the raster (item_tile[i] = t for
        // item_off[t] <= i < item_off[t + 1]), one wave per tile, so that a
        // raster workgroup finds its tile with one load
        const uint32_t nw = blockDim.x >> 6, lane = threadIdx.x & 63u;
        for (uint32_t t = blockIdx.x * nw + (threadIdx.x >> 6); t < rk.n_tiles;
             t += nbin * nw) {
            const uint32_t i1 = min(item_off[t + 1], max_items);
            for (uint32_t i = item_off[t] + lane; i < i1; i += 64u) item_tile[i] = t;
        }
    }
    // v below is a segment unit (see unit_map); lists store units
    for (uint32_t base = blockIdx.x * span; base < nu; base += nbin * span) {
        uint32_t *sv = saved + (size_t)(base / span) * BIN_SAVE_WORDS;
        if (pass == 0) {
            for (uint32_t x = threadIdx.x; x < BIN_SLOTS; x += blockDim.x) {
                keys[x] = BIN_FREE;
                cnt[x] = 0;
            }
            __syncthreads();
            SegIn nxt = seg_load(pos_w, flags, scene_off, rk, base + threadIdx.x, n);
            for (uint32_t sub = 0; sub < nsub; ++sub) {
                const uint32_t v = base + sub * blockDim.x + threadIdx.x;
                const SegIn cur = nxt;
                if (sub + 1 < nsub) nxt = seg_load(pos_w, flags, scene_off, rk, v + blockDim.x, n);
                SegTiles st;
                const bool ok = seg_tiles(cur, cams, proj, rk, v, n, st);
                const uint2 rec = bin_count(st, ok, v, rk, kmax, keys, cnt, tile_cnt, long_list,
                                            counters);
                if (v < nu) segrec[v] = rec;
            }
            __syncthreads();
            if (threadIdx.x == 0) sh_nsave = 0u;
            __syncthreads();
            // flush, and save the occupied slots as (slot, tile, count)
            for (uint32_t x = threadIdx.x; x < BIN_SLOTS; x += blockDim.x) {
                const uint32_t t = keys[x], c = cnt[x];
                if (t == BIN_FREE) continue;
                atomicAdd(&tile_cnt[t], c);
                const uint32_t i = atomicAdd(&sh_nsave, 1u);
                sv[1 + 3 * i] = x;
                sv[2 + 3 * i] = t;
                sv[3 + 3 * i] = c;
            }
            __syncthreads();
            if (threadIdx.x == 0) sv[0] = sh_nsave;
        } else {
            for (uint32_t x = threadIdx.x; x < BIN_SLOTS; x += blockDim.x) {
                keys[x] = BIN_FREE;
                cnt[x] = 0;
            }
            __syncthreads();
            const uint32_t m = sv[0];
            for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
                const uint32_t x = sv[1 + 3 * i], t = sv[2 + 3 * i];
                keys[x] = t;
                basev[x] = tile_off[t] + atomicAdd(&tile_cur[t], sv[3 + 3 * i]);
            }
            __syncthreads();
            // records loaded one step ahead (see SegIn)
            const uint2 none = make_uint2(BIN_NONE, 0u);
            uint2 nrec = base + threadIdx.x < nu ? segrec[base + threadIdx.x] : none;
            for (uint32_t sub = 0; sub < nsub; ++sub) {
                const uint32_t v = base + sub * blockDim.x + threadIdx.x;
                const uint2 rec = nrec;
                if (sub + 1 < nsub) nrec = v + blockDim.x < nu ? segrec[v + blockDim.x] : none;
                if (v >= nu) continue;
                bin_scatter(rec, v, rk, keys, cnt, basev, tile_off, tile_cur, entries);
            }
            __syncthreads();
        }
    }
}

// Scatter pass after binning by the strand generator: workgroup w takes the
// units of generator workgroup w (bundles [w nb, (w + 1) nb), a contiguous
// range of the stream), restores that workgroup's saved table, reserves each
// of its tiles' ranges with one returning global add, and ranks every
// (unit, tile) pair in LDS.  Like pass 1, it first writes the tile of every
// raster work item.
__global__ __launch_bounds__(BIN_BLOCK) void k_bin_spans(RasterK rk, const uint32_t *table,
                                                         uint32_t n_bundles, uint32_t nb,
                                                         const uint32_t *scene_off, uint32_t cap,
                                                         const uint32_t *tile_off,
                                                         uint32_t *tile_cur, uint32_t *entries,
                                                         const uint2 *segrec,
                                                         const uint32_t *saved,
                                                         const uint32_t *item_off,
                                                         uint32_t *item_tile, uint32_t max_items)
{
    __shared__ uint32_t keys[BIN_SLOTS], cnt[BIN_SLOTS], basev[BIN_SLOTS];
    {
        const uint32_t nw = blockDim.x >> 6, lane = threadIdx.x & 63u;
        for (uint32_t t = blockIdx.x * nw + (threadIdx.x >> 6); t < rk.n_tiles;
             t += gridDim.x * nw) {
            const uint32_t i1 = min(item_off[t + 1], max_items);
            for (uint32_t i = item_off[t] + lane; i < i1; i += 64u) item_tile[i] = t;
        }
    }
    const uint32_t n = stream_len(scene_off, rk, cap);
    const uint32_t b0 = blockIdx.x * nb;
    const uint32_t b1 = min(b0 + nb, n_bundles) - 1u;        // last bundle of the span
    const uint4 t0 = reinterpret_cast<const uint4 *>(table)[b0];
    const uint4 t1 = reinterpret_cast<const uint4 *>(table)[b1];
    const uint32_t u0 = min(t0.w, n);
    const uint32_t u1 = (uint32_t)min<uint64_t>((uint64_t)t1.w + (uint64_t)t1.x * t1.y, n);
    for (uint32_t x = threadIdx.x; x < BIN_SLOTS; x += blockDim.x) {
        keys[x] = BIN_FREE;
        cnt[x] = 0u;
    }
    __syncthreads();
    if (u0 < u1) {
        const uint32_t *sv = saved + (size_t)blockIdx.x * BIN_SAVE_WORDS;
        const uint32_t m = sv[0];
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            const uint32_t x = sv[1 + 3 * i], t = sv[2 + 3 * i];
            keys[x] = t;
            basev[x] = tile_off[t] + atomicAdd(&tile_cur[t], sv[3 + 3 * i]);
        }
    }
    __syncthreads();
    // records loaded one step ahead
    const uint2 none = make_uint2(BIN_NONE, 0u);
    uint32_t v = u0 + threadIdx.x;
    uint2 nrec = v < u1 ? segrec[v] : none;
    for (; v < u1; v += blockDim.x) {
        const uint2 rec = nrec;
        if (v + blockDim.x < u1) nrec = segrec[v + blockDim.x];
        bin_scatter(rec, v, rk, keys, cnt, basev, tile_off, tile_cur, entries);
    }
}

// Orders the LDS accesses of one wave around a hand-off between its lanes.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// items per tile = ceil(count / chunk); also resets the cursors.
__global__ __launch_bounds__(256) void k_tile_items(const uint32_t *tile_off, uint32_t n_tiles,
                                                    uint32_t chunk, uint32_t *items,
                                                    uint32_t *tile_cur)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t c = tile_off[t + 1] - tile_off[t];
    items[t] = (c + chunk - 1) / chunk;
    tile_cur[t] = 0;
}

// Frames with few tiles: one workgroup turns the tile counts into list offsets
// (in place, total at [nt]), computes the work items of each tile and their
// offsets (total at [nt]) and resets the scatter cursors.
constexpr uint32_t PLAN_SMALL = 8192;

__global__ __launch_bounds__(1024) void k_plan_small(uint32_t *tile_cnt, uint32_t nt,
                                                     uint32_t chunk, uint32_t *items,
                                                     uint32_t *tile_cur)
{
    __shared__ uint32_t l1[1024 / 64 + 1], l2[1024 / 64 + 1];
    uint32_t cs = 0, ci = 0;
    for (uint32_t base = 0; base < nt; base += blockDim.x) {
        const uint32_t t = base + threadIdx.x;
        const uint32_t c = t < nt ? tile_cnt[t] : 0u;
        const uint32_t it = (c + chunk - 1) / chunk;
        uint32_t s1, s2;
        const uint32_t o1 = block_exclusive_scan<uint32_t>(c, l1, s1) + cs;
        const uint32_t o2 = block_exclusive_scan<uint32_t>(it, l2, s2) + ci;
        if (t < nt) {
            tile_cnt[t] = o1;
            items[t] = o2;
            tile_cur[t] = 0u;
        }
        cs += s1;
        ci += s2;
    }
    if (threadIdx.x == 0) {
        tile_cnt[nt] = cs;
        items[nt] = ci;
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, uint32_t n, uint32_t val)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = val;
}

// ------------------------------------------------------------------ tiled raster
// Shared by both tile kernels.  A work item is a tile and a chunk of its
// segment list; a tile that is one work item owns its pixels (it starts from
// the prefilled values and writes back with plain stores), a split tile merges
// every touched pixel with one 64-bit global atomic minimum per layer.
//
// The tile's layers live in LDS with a row pitch of T + 1 keys, so that one
// column of consecutive rows falls in different banks (the per-pixel spread
// walks steep segments down columns).
__host__ __device__ constexpr uint32_t tile_pitch(uint32_t T) { return T + 1u; }

// Tile words of a pass: two layers of 64-bit keys, or (deep-opacity counting)
// the first-fragment depth code plus one count per layer, 32 bits each; TP =
// T * pitch words per layer.
__host__ __device__ inline uint32_t tile_words(uint32_t TP, bool dom, uint32_t n_layers)
{
    return dom ? (1u + n_layers) * TP : 4u * TP;
}

// Deep-opacity counting pass of the tile raster: q0 of every pixel comes from
// the light view's conservative layer (vis), accepted conservative pairs are
// counted in layer min((q - q0) / layer_codes, n_layers - 1).
struct DomK {
    uint32_t *counts;       // [n_layers][H][W]
    uint32_t layer_codes, n_layers;
};

__device__ __forceinline__ void dom_count(uint32_t *cnt, const uint32_t *q0t, uint32_t x,
                                          uint32_t TP, uint32_t q, const DomK &dk)
{
    const uint32_t q0 = q0t[x];
    uint32_t k = q > q0 ? (q - q0) / dk.layer_codes : 0u;
    k = k < dk.n_layers - 1u ? k : dk.n_layers - 1u;
    atomicAdd(&cnt[k * TP + x], 1u);
}

// Geometry of one work item.
struct TileItem {
    uint32_t beg, end, s;
    int px0, py0, px1, py1;
    uint32_t tw, th;
    bool whole;
};

__device__ __forceinline__ TileItem tile_item(const RasterK &rk, uint32_t item,
                                              const uint32_t *tile_off, const uint32_t *item_off,
                                              const uint32_t *item_tile)
{
    TileItem it;
    const uint32_t t = item_tile[item];         // item_off[t] <= item < item_off[t + 1]
    it.beg = tile_off[t] + (item - item_off[t]) * rk.chunk;
    const uint32_t end0 = it.beg + rk.chunk, tend = tile_off[t + 1];
    it.end = end0 < tend ? end0 : tend;
    const uint32_t tiles_per_scene = rk.ntx * rk.nty;
    it.s = t / tiles_per_scene;
    const uint32_t r = t - it.s * tiles_per_scene;
    const uint32_t ty = r / rk.ntx, tx = r - ty * rk.ntx;
    it.px0 = (int)(tx * rk.T);
    it.py0 = (int)(ty * rk.T);
    it.px1 = min(it.px0 + (int)rk.T, (int)rk.W) - 1;
    it.py1 = min(it.py0 + (int)rk.T, (int)rk.H) - 1;
    it.tw = (uint32_t)(it.px1 - it.px0 + 1);
    it.th = (uint32_t)(it.py1 - it.py0 + 1);
    it.whole = tend - tile_off[t] <= rk.chunk;
    return it;
}

// Two key layers of a tile: set empty, or (a tile that is one work item) load
// the prefilled values.
__device__ __forceinline__ void tile_keys_init(uint64_t *lc, uint64_t *la, const TileItem &it,
                                               const RasterK &rk, const uint64_t *vc,
                                               const uint64_t *va)
{
    const uint32_t P = tile_pitch(rk.T);
    for (uint32_t x = threadIdx.x; x < rk.T * rk.T; x += blockDim.x) {
        const uint32_t ly = x / rk.T, lx = x - ly * rk.T;
        uint64_t kc = HM_EMPTY, ka = HM_EMPTY;
        if (it.whole && lx < it.tw && ly < it.th) {
            const size_t p = (size_t)(it.py0 + (int)ly) * rk.W + (size_t)(it.px0 + (int)lx);
            kc = vc[p];
            ka = va[p];
        }
        lc[ly * P + lx] = kc;
        la[ly * P + lx] = ka;
    }
}

// Merge the tile's layers into the buffer: plain stores for a tile that is one
// work item, else one atomic minimum per touched pixel and layer.
__device__ __forceinline__ void tile_keys_store(const uint64_t *lc, const uint64_t *la,
                                                const TileItem &it, const RasterK &rk,
                                                uint64_t *vc, uint64_t *va)
{
    const uint32_t P = tile_pitch(rk.T);
    for (uint32_t x = threadIdx.x; x < rk.T * rk.T; x += blockDim.x) {
        const uint32_t ly = x / rk.T, lx = x - ly * rk.T;
        if (lx >= it.tw || ly >= it.th) continue;
        const size_t p = (size_t)(it.py0 + (int)ly) * rk.W + (size_t)(it.px0 + (int)lx);
        const uint64_t kc = lc[ly * P + lx], ka = la[ly * P + lx];
        if (it.whole) {
            vc[p] = kc;
            va[p] = ka;
        } else {
            if (kc != HM_EMPTY) atomicMin((unsigned long long *)(vc + p), (unsigned long long)kc);
            if (ka != HM_EMPTY) atomicMin((unsigned long long *)(va + p), (unsigned long long)ka);
        }
    }
}

// ------------------------------------------------------------------ row walker
// Per-segment records of a batch, struct of arrays with stride nb (fields a
// caller does not use are not read: the loads are plain LDS reads): the 16
// geometric fields of Seg (the slack e is recomputed from them), with
// G-buffer keys also 1/z of the second endpoint, then the stream id, then the
// segment's first row slot (15 bits: at most 1024 * 32 slots) with its row /
// column clip inside the tile (5 bits each, T <= 32):
// slot | (j0 - py0) << 15 | (i0 - px0) << 20 | (i1 - px0) << 25.
constexpr uint32_t REC_FLOATS = 16;
__host__ __device__ constexpr uint32_t rec_floats(bool gb) { return gb ? REC_FLOATS + 1 : REC_FLOATS; }
__host__ __device__ constexpr uint32_t rec_words(bool gb) { return rec_floats(gb) + 2; }
__device__ __forceinline__ uint32_t rc_slot(uint32_t rc) { return rc & 0x7FFFu; }
__device__ __forceinline__ int rc_j0(uint32_t rc) { return (int)((rc >> 15) & 31u); }
__device__ __forceinline__ int rc_i0(uint32_t rc) { return (int)((rc >> 20) & 31u); }
__device__ __forceinline__ int rc_i1(uint32_t rc) { return (int)(rc >> 25); }

template <bool GB>
__device__ __forceinline__ void rec_store(float *rf, uint32_t nb, uint32_t k, const Seg &s)
{
    const float f[REC_FLOATS] = {s.x0,    s.y0, s.w0,   s.iz0,  s.dx,   s.dy,   s.dw,   s.diz,
                                 s.len2, s.ilen2, s.ra, s.sxmn, s.sxmx, s.symn, s.symx, s.idy};
#pragma unroll
    for (uint32_t i = 0; i < REC_FLOATS; ++i) rf[i * nb + k] = f[i];
    if (GB) rf[REC_FLOATS * nb + k] = s.iz1;
}

template <bool GB>
__device__ __forceinline__ Seg rec_load(const float *rf, uint32_t nb, uint32_t k)
{
    Seg s;
    s.x0 = rf[0 * nb + k]; s.y0 = rf[1 * nb + k]; s.w0 = rf[2 * nb + k]; s.iz0 = rf[3 * nb + k];
    s.dx = rf[4 * nb + k]; s.dy = rf[5 * nb + k]; s.dw = rf[6 * nb + k]; s.diz = rf[7 * nb + k];
    s.len2 = rf[8 * nb + k]; s.ilen2 = rf[9 * nb + k]; s.ra = rf[10 * nb + k];
    s.sxmn = rf[11 * nb + k]; s.sxmx = rf[12 * nb + k]; s.symn = rf[13 * nb + k];
    s.symx = rf[14 * nb + k]; s.idy = rf[15 * nb + k];
    s.e = seg_slack(s);
    s.iz1 = GB ? rf[REC_FLOATS * nb + k] : 0.0f;
    return s;
}

// Rows [j0, j1] of a tile that the segment can reach: clip the segment to the
// tile's column slab widened by ra (+ slack) and keep the rows whose band
// [j - ra, j + 1 + ra] meets the clipped part's y extent (same argument and
// slack as row_span, with x and y exchanged).  False if none remain.
__device__ __forceinline__ bool tile_rows(const Seg &sg, int px0, int px1, int &j0, int &j1)
{
    const float e = sg.e;
    const float xl = ((float)px0 - sg.ra) - e, xh = (((float)px1 + 1.0f) + sg.ra) + e;
    float ya = sg.symn, yb = sg.symx;
    if (fabsf(sg.dx) > 1e-3f) {
        const float idx = 1.0f / sg.dx;
        const float ta = (xl - sg.x0) * idx, tb = (xh - sg.x0) * idx;
        const float t0 = fmaxx(fminx(ta, tb), 0.0f), t1 = fminx(fmaxx(ta, tb), 1.0f);
        if (t0 > t1) return false;
        const float y_a = sg.y0 + t0 * sg.dy, y_b = sg.y0 + t1 * sg.dy;
        ya = fminx(y_a, y_b);
        yb = fmaxx(y_a, y_b);
    } else if (sg.sxmx < xl || sg.sxmn > xh) {
        return false;
    }
    const float flo = ((ya - 1.0f) - sg.ra) - e, fhi = (yb + sg.ra) + e;
    if (flo > -1.0e9f) j0 = max(j0, (int)ceilf(flo));
    if (fhi < 1.0e9f) j1 = min(j1, (int)floorf(fhi));
    return j0 <= j1;
}

// dynamic LDS bytes of k_raster_rows: two layers and the segment records
static inline uint32_t rows_lds_bytes(uint32_t T, uint32_t block, bool gb)
{
    return 2u * T * tile_pitch(T) * 8u + block * 4u * rec_words(gb);
}

// Tile raster, row walker (HM_RASTER_TILED_ROWS).  Work items (a tile and a
// chunk of its segment list) are pulled from counters[1].  Segments are taken
// in batches of nb: each lane builds one segment's record (screen geometry,
// the rows and columns of the tile it can reach, stream id) and one block scan
// both compacts the segments that reach the tile and numbers their (segment,
// row) pairs ("row slots"); each lane then takes a contiguous run of row slots
// and loops over the candidate pixels of each row.  NBC: the workgroup size
// when known at compile time (the record fields then sit at fixed LDS
// offsets), 0 for any blockDim.
template <uint32_t NBC, bool GB>
__global__ void k_raster_rows(const float4 *proj, const uint8_t *flags,
                              const uint32_t *scene_off, const hm_camera *cams, RasterK rk,
                              uint32_t cap, const uint32_t *tile_off, const uint32_t *item_off,
                              const uint32_t *item_tile, const uint32_t *entries,
                              uint32_t *counters, uint64_t *vis, GbK gk)
{
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t sh_item;
    __shared__ uint32_t sh_scan[1024 / 64 + 1];
    const uint32_t P = tile_pitch(rk.T);
    const uint32_t TP = rk.T * P;
    const uint32_t nb = NBC ? NBC : blockDim.x;
    uint64_t *lc = lds, *la = lds + TP;
    float *rf = reinterpret_cast<float *>(lds) + tile_words(TP, false, 1u);
    uint32_t *rw = reinterpret_cast<uint32_t *>(rf);
    uint32_t *r_sid = rw + rec_floats(GB) * nb;      // stream id
    uint32_t *r_rc = r_sid + nb;                     // first row slot + clip

    const uint32_t n = stream_len(scene_off, rk, cap);
    const uint32_t n_items = item_off[rk.n_tiles];
    const size_t hw = (size_t)rk.W * rk.H;
    for (;;) {
        if (threadIdx.x == 0) sh_item = atomicAdd(&counters[1], 1u);
        __syncthreads();
        const uint32_t item = sh_item;
        if (item >= n_items) break;
        const TileItem it = tile_item(rk, item, tile_off, item_off, item_tile);
        const int px0 = it.px0, py0 = it.py0;
        float zn, inv_range;
        scene_depth_consts(cams, it.s, zn, inv_range);
        uint64_t *vc = vis + (size_t)it.s * 2 * hw, *va = vc + hw;
        tile_keys_init(lc, la, it, rk, vc, va);
        __syncthreads();

        uint32_t nx_u = 0;
        EntryIn nx{};
        if (it.beg + threadIdx.x < it.end) {
            nx_u = entries[it.beg + threadIdx.x];
            nx = entry_load(proj, flags, scene_off, rk, n, nx_u);
        }
        for (uint32_t e0 = it.beg; e0 < it.end; e0 += nb) {
            const uint32_t e = e0 + threadIdx.x;
            const EntryIn cur = nx;
            const bool more = e0 + nb < it.end;
            if (more && e + nb < it.end) nx_u = entries[e + nb];
            uint32_t nr = 0, vu = 0;
            Seg sg;
            int i0, i1, j0, j1;
            if (e < it.end) {
                vu = cur.v;
                if (seg_from(cur, n, rk.r_min, sg) && seg_box(sg, rk.W, rk.H, i0, i1, j0, j1)) {
                    j0 = max(j0, py0);
                    j1 = min(j1, it.py1);
                    i0 = max(i0, px0);
                    i1 = min(i1, it.px1);
                    if (i0 <= i1 && j0 <= j1 && tile_rows(sg, px0, it.px1, j0, j1))
                        nr = (uint32_t)(j1 - j0 + 1);
                }
            }
            // one scan: low 16 bits number the row slots (at most nb * T),
            // high 16 bits compact the segments that reach the tile
            uint32_t totp;
            const uint32_t pre = block_exclusive_scan((nr ? 0x10000u : 0u) | nr, sh_scan, totp);
            const uint32_t tot = totp & 0xFFFFu, nseg = totp >> 16;
            if (nr) {
                const uint32_t c = pre >> 16, r0 = pre & 0xFFFFu;
                rec_store<GB>(rf, nb, c, sg);
                r_sid[c] = vu;
                r_rc[c] = r0 | ((uint32_t)(j0 - py0) << 15) | ((uint32_t)(i0 - px0) << 20) |
                          ((uint32_t)(i1 - px0) << 25);
            }
            __syncthreads();
            if (more && e + nb < it.end) nx = entry_load(proj, flags, scene_off, rk, n, nx_u);
            const uint32_t per = (tot + nb - 1) / nb;
            const uint32_t r_beg = threadIdx.x * per;
            const uint32_t r_end = min(r_beg + per, tot);
            uint32_t ow = 0;
            if (r_beg < r_end) {            // owner of the first slot: binary search
                uint32_t h2 = nseg;
                while (h2 - ow > 1) {
                    const uint32_t mid = (ow + h2) >> 1;
                    if (rc_slot(r_rc[mid]) <= r_beg) ow = mid; else h2 = mid;
                }
            }
            uint32_t curo = 0xFFFFFFFFu, vo = 0, rc = 0;
            Seg sr;
            int jb = 0;
            uint32_t pb = 0;
            for (uint32_t rr = r_beg; rr < r_end; ++rr) {
                while (ow + 1 < nseg && rc_slot(r_rc[ow + 1]) <= rr) ++ow;
                if (ow != curo) {
                    curo = ow;
                    sr = rec_load<GB>(rf, nb, ow);
                    vo = r_sid[ow];
                    rc = r_rc[ow];
                    jb = py0 + rc_j0(rc);
                    pb = rc_slot(rc);
                }
                const int j = jb + (int)(rr - pb);
                int a0, a1;
                row_span(sr, j, a0, a1);
                a0 = max(a0, px0 + rc_i0(rc));
                a1 = min(a1, px0 + rc_i1(rc));
                for (int i = a0; i <= a1; ++i) {
                    uint32_t q;
                    bool cc, ca;
                    float ts, z;
                    if (!cover_tz(sr, i, j, rk.r_min, zn, inv_range, cc, ca, q, ts, z)) continue;
                    const uint32_t x = (uint32_t)(j - py0) * P + (uint32_t)(i - px0);
                    const uint64_t low =
                        GB ? gb_payload(gk.tan, gk.rgb, vo, ts, z, sr.iz1) : (uint64_t)vo;
                    const unsigned long long key = ((unsigned long long)q << HM_ID_BITS) | low;
                    if (cc) atomicMin((unsigned long long *)&lc[x], key);
                    if (ca) atomicMin((unsigned long long *)&la[x], key);
                }
            }
            __syncthreads();
        }
        tile_keys_store(lc, la, it, rk, vc, va);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ per-pixel spread
// The spread walks each segment along lines of candidate pixels parallel to
// its major axis: a steep segment (|dy| > |dx|) down columns, any other along
// rows, so that a line holds several candidates.  Its records are those of the
// row walker (rec_store) with the last field, the reciprocal used to clip a
// line, holding 1 / dx for a column segment (1 / dy for a row one, 0 when that
// displacement is below 1e-3), then the stream id and the line word: first
// line slot (14 bits) | first fixed coordinate in the tile (5) << 14 |
// varying clip v0, v1 in the tile (5 + 5) << 19, 24 | orientation (1 =
// columns) << 29.  The candidates themselves are tested with cover_tz's
// expressions in (x, y), whatever the orientation.

// Pixel descriptors per wave between evaluations (a window of one wave's
// candidates, gathered over several 64-line groups).
constexpr uint32_t PIX_WINDOW = 240;

// dynamic LDS bytes of k_raster_flat for tile edge T, `block` threads and a
// tile of `tile_w` 32-bit words: the tile, the segment records, the bitmap of
// first line slots, the first segment of every 64-slot group, and per wave a
// window of pixel descriptors.  T = 32 with 256 threads takes 40704 B, so four
// workgroups fit a CU's 160 KiB.
static inline uint32_t flat_lds_bytes(uint32_t T, uint32_t block, bool gb, uint32_t tile_w)
{
    const uint32_t slots = block * T;
    return tile_w * 4u + block * 4u * rec_words(gb) + slots / 8u + ((slots + 63u) / 64u) * 4u +
           (block / 64u) * PIX_WINDOW * 4u;
}

// Fixed coordinates [f0, f1] of the tile that the segment can reach: clip it to
// the tile's slab [v_lo, v_hi] of the varying axis widened by ra (+ slack) and
// keep the lines whose band [c - ra, c + 1 + ra] meets the clipped part's f
// extent (tile_rows in the segment's frame: rows for col = false, columns for
// col = true).  False if none remain.
__device__ __forceinline__ bool tile_lines(const Seg &sg, bool col, int v_lo, int v_hi, int &f0,
                                           int &f1)
{
    const float e = sg.e;
    const float o = col ? sg.y0 : sg.x0, of = col ? sg.x0 : sg.y0;
    const float a = col ? sg.dy : sg.dx, b = col ? sg.dx : sg.dy;
    const float vmn = col ? sg.symn : sg.sxmn, vmx = col ? sg.symx : sg.sxmx;
    float fa = col ? sg.sxmn : sg.symn, fb = col ? sg.sxmx : sg.symx;
    const float xl = ((float)v_lo - sg.ra) - e, xh = (((float)v_hi + 1.0f) + sg.ra) + e;
    if (fabsf(a) > 1e-3f) {
        const float ia = 1.0f / a;
        const float ta = (xl - o) * ia, tb = (xh - o) * ia;
        const float t0 = fmaxx(fminx(ta, tb), 0.0f), t1 = fminx(fmaxx(ta, tb), 1.0f);
        if (t0 > t1) return false;
        const float y_a = of + t0 * b, y_b = of + t1 * b;
        fa = fminx(y_a, y_b);
        fb = fmaxx(y_a, y_b);
    } else if (vmx < xl || vmn > xh) {
        return false;
    }
    const float flo = ((fa - 1.0f) - sg.ra) - e, fhi = (fb + sg.ra) + e;
    if (flo > -1.0e9f) f0 = max(f0, (int)ceilf(flo));
    if (fhi < 1.0e9f) f1 = min(f1, (int)floorf(fhi));
    return f0 <= f1;
}

// Candidate varying coordinates [v0, v1] of the line at fixed coordinate cf of
// record k (row_span in the segment's frame: pixel (v, cf) can pass either test
// only if the segment has a point within ra of both of its bands; same slack).
__device__ __forceinline__ void line_span(const float *rf, uint32_t nb, uint32_t k, bool col,
                                          int cf, int &v0, int &v1)
{
    const Seg sg = rec_load<false>(rf, nb, k);      // e recomputed; ifx in the idy slot
    const float e = sg.e, ra = sg.ra;
    const float of = col ? sg.x0 : sg.y0, ifx = sg.idy;
    const float ylo = ((float)cf - ra) - e, yhi = (((float)cf + 1.0f) + ra) + e;
    float xlo = col ? sg.symn : sg.sxmn, xhi = col ? sg.symx : sg.sxmx;
    if (ifx != 0.0f) {
        const float ta = (ylo - of) * ifx, tb = (yhi - of) * ifx;
        const float t0 = fmaxx(fminx(ta, tb), 0.0f), t1 = fminx(fmaxx(ta, tb), 1.0f);
        if (t0 > t1) { v0 = 1; v1 = 0; return; }
        const float o = col ? sg.y0 : sg.x0, a = col ? sg.dy : sg.dx;
        const float xa = o + t0 * a, xb = o + t1 * a;
        xlo = fminx(xa, xb);
        xhi = fmaxx(xa, xb);
    } else if ((col ? sg.sxmx : sg.symx) < ylo || (col ? sg.sxmn : sg.symn) > yhi) {
        v0 = 1; v1 = 0;
        return;
    }
    const float flo = ((xlo - 1.0f) - ra) - e, fhi = (xhi + ra) + e;
    v0 = flo > -1.0e9f ? (int)ceilf(flo) : -1000000000;
    v1 = fhi < 1.0e9f ? (int)floorf(fhi) : 1000000000;
}

// Tile raster with the per-pixel spread (HM_RASTER_TILED; also the counting
// pass of deep-opacity maps, DOM, and compressed G-buffer keys, GB).  Work
// items are pulled from counters[1]; segments are taken in batches of nb = the
// workgroup size, one per lane:
//   1. each lane builds its segment's oriented record and the lines (rows or
//      columns) of the tile it can reach; one block scan compacts the segments
//      and numbers their lines ("line slots"); a bitmap marks every segment's
//      first slot and each 64-slot group notes the segments before it;
//   2. waves take 64-slot groups from an LDS counter; each lane computes one
//      line's candidate span, and the wave appends the candidates' descriptors
//      (segment | row and column in the tile) to its window, which gathers the
//      candidates of several groups;
//   3. a full window (and the last one of the batch) is evaluated two
//      candidates per lane at a time (one with G-buffer keys), with LDS 64-bit
//      minima into the tile.
// NB: the workgroup size when known at compile time (fixed LDS offsets), 0 for
// any blockDim (at most 256).
template <uint32_t NB, bool DOM, bool GB>
__global__ __launch_bounds__(256) void k_raster_flat(
    const float4 *proj, const uint8_t *flags, const uint32_t *scene_off, const hm_camera *cams,
    RasterK rk, uint32_t cap, const uint32_t *tile_off, const uint32_t *item_off,
    const uint32_t *item_tile, const uint32_t *entries, uint32_t *counters, uint64_t *vis,
    DomK dk, GbK gk)
{
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t sh_item, sh_group;
    __shared__ uint32_t sh_scan[1024 / 64 + 1];
    const uint32_t P = tile_pitch(rk.T);
    const uint32_t TP = rk.T * P;
    const uint32_t nb = NB ? NB : blockDim.x;
    uint64_t *lc = lds, *la = lds + TP;
    uint32_t *q0t = reinterpret_cast<uint32_t *>(lds), *cnt = q0t + TP;    // DOM only
    float *rf = reinterpret_cast<float *>(lds) + tile_words(TP, DOM, dk.n_layers);
    uint32_t *rw = reinterpret_cast<uint32_t *>(rf);
    uint32_t *r_sid = rw + rec_floats(GB) * nb;      // stream id
    uint32_t *r_rc = r_sid + nb;                     // line word
    const uint32_t slots_max = nb * rk.T;
    uint32_t *bmp = r_rc + nb;                       // first slot of each segment
    uint32_t *gfirst = bmp + slots_max / 32u;        // segment count before each group
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    uint32_t *pdesc = gfirst + (slots_max + 63u) / 64u + wv * PIX_WINDOW;
    const uint64_t le = (2ull << lane) - 1ull;          // lanes <= this one
    const float rmin = __builtin_canonicalizef(rk.r_min);

    const uint32_t n = stream_len(scene_off, rk, cap);
    const uint32_t n_items = item_off[rk.n_tiles];
    const size_t hw = (size_t)rk.W * rk.H;
    for (;;) {
        if (threadIdx.x == 0) sh_item = atomicAdd(&counters[1], 1u);
        __syncthreads();
        const uint32_t item = sh_item;
        if (item >= n_items) break;
        const TileItem it = tile_item(rk, item, tile_off, item_off, item_tile);
        const int px0 = it.px0, py0 = it.py0;
        const float zn = cams[it.s].znear, zf = cams[it.s].zfar;
        const float inv_range = 1.0f / (zf - zn);
        // every 1/z of the item lies in (1/zf, 1/zn) up to a few ulps
        const bool fast = zn >= 0x1p-124f && zf <= 0x1p124f;
        uint64_t *vc = vis + (size_t)it.s * 2 * hw, *va = vc + hw;
        if (DOM) {
            for (uint32_t x = threadIdx.x; x < rk.T * rk.T; x += blockDim.x) {
                const uint32_t ly = x / rk.T, lx = x - ly * rk.T;
                uint32_t q0 = 0xFFFFFFFFu;
                if (lx < it.tw && ly < it.th) {
                    const size_t p = (size_t)(py0 + (int)ly) * rk.W + (size_t)(px0 + (int)lx);
                    q0 = (uint32_t)(va[p] >> HM_ID_BITS);
                }
                q0t[ly * P + lx] = q0;
            }
            for (uint32_t x = threadIdx.x; x < dk.n_layers * TP; x += blockDim.x) cnt[x] = 0u;
        } else {
            tile_keys_init(lc, la, it, rk, vc, va);
        }
        __syncthreads();

        // each batch's stream inputs are loaded during the previous batch
        uint32_t nx_u = 0;
        EntryIn nx{};
        if (it.beg + threadIdx.x < it.end) {
            nx_u = entries[it.beg + threadIdx.x];
            nx = entry_load(proj, flags, scene_off, rk, n, nx_u);
        }
        for (uint32_t e0 = it.beg; e0 < it.end; e0 += nb) {
            const uint32_t e = e0 + threadIdx.x;
            const EntryIn cur = nx;
            const bool more = e0 + nb < it.end;
            if (more && e + nb < it.end) nx_u = entries[e + nb];
            // 1. oriented record and reachable lines of this lane's segment
            uint32_t nr = 0, vu = 0;
            bool col = false;
            Seg sg;
            int f0 = 0, f1 = -1, v0c = 0, v1c = -1;
            if (e < it.end) {
                vu = cur.v;
                int i0, i1, j0, j1;
                if (seg_from(cur, n, rk.r_min, sg) && seg_box(sg, rk.W, rk.H, i0, i1, j0, j1)) {
                    i0 = max(i0, px0);
                    i1 = min(i1, it.px1);
                    j0 = max(j0, py0);
                    j1 = min(j1, it.py1);
                    col = fabsf(sg.dy) > fabsf(sg.dx);
                    f0 = col ? i0 : j0;
                    f1 = col ? i1 : j1;
                    v0c = col ? j0 : i0;
                    v1c = col ? j1 : i1;
                    if (i0 <= i1 && j0 <= j1 && tile_lines(sg, col, v0c, v1c, f0, f1))
                        nr = (uint32_t)(f1 - f0 + 1);
                }
            }
            for (uint32_t x = threadIdx.x; x < slots_max / 32u; x += blockDim.x) bmp[x] = 0u;
            // one scan: bits 0..13 number the line slots (at most nb * T <=
            // 8192), bits 14..22 compact the segments that reach the tile,
            // bits 23..31 count those of zero length (at most nb <= 256 each)
            const bool degen = nr && !(sg.len2 > 0.0f);
            uint32_t totp;
            const uint32_t pre = block_exclusive_scan(
                nr | (nr ? 1u << 14 : 0u) | (degen ? 1u << 23 : 0u), sh_scan, totp);
            const uint32_t tot = totp & 0x3FFFu;
            const bool any_degen = (totp >> 23) != 0u;
            if (nr) {
                const uint32_t c = (pre >> 14) & 0x1FFu, r0 = pre & 0x3FFFu;
                const int fb0 = col ? px0 : py0, vb0 = col ? py0 : px0;
                // the line-clipping reciprocal of the segment's orientation
                Seg sr = sg;
                const float b = col ? sg.dx : sg.dy;
                sr.idy = fabsf(b) > 1e-3f ? 1.0f / b : 0.0f;
                rec_store<GB>(rf, nb, c, sr);
                r_sid[c] = vu;
                r_rc[c] = r0 | ((uint32_t)(f0 - fb0) << 14) | ((uint32_t)(v0c - vb0) << 19) |
                          ((uint32_t)(v1c - vb0) << 24) | ((uint32_t)col << 29);
                atomicOr(&bmp[r0 >> 5], 1u << (r0 & 31u));
                // groups whose first slot lies in this segment's slots: the
                // segments before the group are this one's predecessors, plus
                // this one unless the group starts at its first slot
                for (uint32_t g = (r0 + 63u) >> 6; (g << 6) < r0 + nr; ++g)
                    gfirst[g] = c + ((g << 6) > r0 ? 1u : 0u);
            }
            if (threadIdx.x == 0) sh_group = 0u;
            __syncthreads();
            if (more && e + nb < it.end) nx = entry_load(proj, flags, scene_off, rk, n, nx_u);

            // 2. + 3. lines and candidates, per wave
            const uint32_t ng = (tot + 63u) >> 6;
            uint32_t fill = 0;                    // wave-uniform window fill
            uint32_t Ptot = 0, done = 0;
            bool pend = false, exhausted = ng == 0;
            uint32_t cntl = 0, pcl = 0, d0 = 0, dstep = 0;   // this lane's line of the pending group
            for (;;) {
                if (!pend && !exhausted) {
                    uint32_t gg = 0;
                    if (lane == 0) gg = atomicAdd(&sh_group, 1u);
                    const uint32_t g = (uint32_t)__builtin_amdgcn_readfirstlane((int)gg);
                    if (g >= ng) {
                        exhausted = true;
                        continue;
                    }
                    const uint32_t rr = g * 64u + lane;
                    const bool start = rr < tot && ((bmp[rr >> 5] >> (rr & 31u)) & 1u);
                    const uint64_t M = __ballot(start);
                    cntl = 0;
                    if (rr < tot) {
                        const uint32_t o = gfirst[g] + (uint32_t)__popcll(M & le) - 1u;
                        const uint32_t rc = r_rc[o];
                        const bool cl = (rc >> 29) & 1u;
                        const int vb0 = cl ? py0 : px0;
                        const uint32_t frel = ((rc >> 14) & 31u) + (rr - (rc & 0x3FFFu));
                        int a0, a1;
                        line_span(rf, nb, o, cl, (cl ? px0 : py0) + (int)frel, a0, a1);
                        a0 = max(a0, vb0 + (int)((rc >> 19) & 31u));
                        a1 = min(a1, vb0 + (int)((rc >> 24) & 31u));
                        if (a1 >= a0) cntl = (uint32_t)(a1 - a0 + 1);
                        // descriptor of the line's first candidate: segment |
                        // row in the tile << 8 | column << 13; the next
                        // candidates step down the column or along the row
                        const uint32_t vr = (uint32_t)(a0 - vb0);
                        d0 = o | ((cl ? vr : frel) << 8) | ((cl ? frel : vr) << 13);
                        dstep = cl ? 1u << 8 : 1u << 13;
                    }
                    const uint32_t inc = wave_inclusive_scan(cntl);
                    pcl = inc - cntl;
                    Ptot = wave_last(inc);
                    if (Ptot == 0) continue;
                    pend = true;
                    done = 0;
                }
                bool eval;
                if (pend) {
                    // append the part of the group's candidates that fits
                    const uint32_t room = PIX_WINDOW - fill;
                    const uint32_t nn = min(Ptot - done, room);
                    const uint32_t m0 = max(pcl, done), m1 = min(pcl + cntl, done + nn);
                    if (m0 < m1) {
                        uint32_t *dst = pdesc + fill + (m0 - done);
                        const uint32_t db = d0 + (m0 - pcl) * dstep;
                        for (uint32_t s = 0; s < m1 - m0; ++s) dst[s] = db + s * dstep;
                    }
                    fill += nn;
                    done += nn;
                    if (done == Ptot) pend = false;
                    eval = fill == PIX_WINDOW;
                } else {
                    if (fill == 0) break;     // no group left
                    eval = true;
                }
                if (!eval) continue;
                wave_sync();
                // evaluate the window; compiled apart for the (uniform)
                // reciprocal path and for batches holding a segment of zero
                // length
                auto evaluate = [&](auto fast_tag, auto degen_tag) {
                    constexpr bool FAST = decltype(fast_tag)::value;
                    constexpr bool DEGEN = decltype(degen_tag)::value;
                    // coverage of both layers and the key of candidate d
                    auto cand = [&](uint32_t d, bool &cc, bool &ca, uint32_t &x, uint32_t &q,
                                    unsigned long long &key) {
                        const uint32_t o = d & 0xFFu;
                        const uint32_t jl = (d >> 8) & 31u, il = d >> 13;
                        x = __umul24(jl, P) + il;
                        const float fi = (float)(px0 + (int)il), fj = (float)(py0 + (int)jl);
                        const float x0 = rf[0 * nb + o], y0 = rf[1 * nb + o];
                        const float w0 = rf[2 * nb + o], dx = rf[4 * nb + o];
                        const float dy = rf[5 * nb + o], dw = rf[6 * nb + o];
                        const float len2 = rf[8 * nb + o], ilen2 = rf[9 * nb + o];
                        const float ra = rf[10 * nb + o];
                        // cover_tz's expressions: centre sample
                        const float ux = (fi + 0.5f) - x0;
                        const float uy = (fj + 0.5f) - y0;
                        const float tn = ux * dx + uy * dy;
                        const float t = tn * ilen2;
                        const float wt = w0 + t * dw;
                        const float r = fmaxf(0.5f * wt, rmin);
                        const float r2 = r * r;
                        const float cr = ux * dy - uy * dx;
                        cc = (tn >= 0.0f) & (tn < len2) & (cr * cr <= r2 * len2);
                        // a segment of zero length: distance to its point
                        if (DEGEN && !(len2 > 0.0f)) cc = (ux * ux + uy * uy) <= r2;
                        // conservative: separating axes x, y and the normal
                        const float bx0 = fi - ra, bx1 = (fi + 1.0f) + ra;
                        const float by0 = fj - ra, by1 = (fj + 1.0f) + ra;
                        const float fa = (bx0 - x0) * dy, fb = (bx1 - x0) * dy;
                        const float ga = (by0 - y0) * dx, gb = (by1 - y0) * dx;
                        const float lo = fminf(fa, fb) - fmaxf(ga, gb);
                        const float hi = fmaxf(fa, fb) - fminf(ga, gb);
                        ca = (rf[11 * nb + o] <= bx1) & (rf[12 * nb + o] >= bx0) &
                             (rf[13 * nb + o] <= by1) & (rf[14 * nb + o] >= by0) &
                             (lo <= 0.0f) & (hi >= 0.0f);
                        // depth at the clamped closest point
                        float ts = t;
                        ts = fmaxx(ts, 0.0f);
                        ts = fminx(ts, 1.0f);
                        const float iz = rf[3 * nb + o] + ts * rf[7 * nb + o];
                        const float z = FAST ? rcp_refined(iz) : 1.0f / iz;
                        q = depth_code(z, zn, inv_range);
                        const uint64_t low =
                            GB ? gb_payload(gk.tan, gk.rgb, r_sid[o], ts, z,
                                            rf[REC_FLOATS * nb + o])
                               : (uint64_t)r_sid[o];
                        key = ((unsigned long long)q << HM_ID_BITS) | low;
                    };
                    auto merge = [&](bool cc, bool ca, uint32_t x, uint32_t q,
                                     unsigned long long key) {
                        if (DOM) {
                            if (ca) dom_count(cnt, q0t, x, TP, q, dk);
                        } else {
                            if (cc) atomicMin((unsigned long long *)&lc[x], key);
                            if (ca) atomicMin((unsigned long long *)&la[x], key);
                        }
                    };
                    if constexpr (GB) {
                        // one candidate per lane and step: the payload's
                        // registers would cost occupancy with two
                        for (uint32_t p0 = 0; p0 < fill; p0 += 64) {
                            const uint32_t pa = p0 + lane;
                            if (pa >= fill) continue;
                            bool cca, caa;
                            uint32_t xa, qa;
                            unsigned long long ka;
                            cand(pdesc[pa], cca, caa, xa, qa, ka);
                            merge(cca, caa, xa, qa, ka);
                        }
                    } else {
                        // two candidates per lane and step (pl and pl + 64),
                        // both evaluated without branches so that their LDS
                        // reads and arithmetic interleave; a lane past the
                        // window's end evaluates the window's first
                        // descriptor and discards the result
                        for (uint32_t p0 = 0; p0 < fill; p0 += 128) {
                            const uint32_t pa = p0 + lane, pb = pa + 64u;
                            const bool va = pa < fill, vb = pb < fill;
                            const uint32_t da = pdesc[va ? pa : 0u], db = pdesc[vb ? pb : 0u];
                            bool cca, caa, ccb, cab;
                            uint32_t xa, xb, qa, qb;
                            unsigned long long ka, kb;
                            cand(da, cca, caa, xa, qa, ka);
                            cand(db, ccb, cab, xb, qb, kb);
                            merge(va & cca, va & caa, xa, qa, ka);
                            merge(vb & ccb, vb & cab, xb, qb, kb);
                        }
                    }
                };
                using yes = std::true_type;
                using no = std::false_type;
                if (fast) {
                    if (any_degen) evaluate(yes{}, yes{}); else evaluate(yes{}, no{});
                } else {
                    if (any_degen) evaluate(no{}, yes{}); else evaluate(no{}, no{});
                }
                wave_sync();
                fill = 0;
            }
            __syncthreads();
        }
        if (DOM) {
            for (uint32_t x = threadIdx.x; x < rk.T * rk.T; x += blockDim.x) {
                const uint32_t ly = x / rk.T, lx = x - ly * rk.T;
                if (lx >= it.tw || ly >= it.th) continue;
                const size_t p = (size_t)(py0 + (int)ly) * rk.W + (size_t)(px0 + (int)lx);
                for (uint32_t k = 0; k < dk.n_layers; ++k) {
                    const uint32_t c = cnt[k * TP + ly * P + lx];
                    if (it.whole) dk.counts[(size_t)k * hw + p] = c;
                    else if (c) atomicAdd(dk.counts + (size_t)k * hw + p, c);
                }
            }
        } else {
            tile_keys_store(lc, la, it, rk, vc, va);
        }
        __syncthreads();
    }
}

// One wave per long segment: lanes stride over its candidate rows (DOM: the
// counting pass, one global add per accepted conservative pair).
template <bool DOM, bool GB>
__global__ __launch_bounds__(256) void k_raster_long(const float4 *proj, const uint8_t *flags,
                                                     const uint32_t *scene_off,
                                                     const hm_camera *cams, RasterK rk,
                                                     uint32_t cap, const uint32_t *long_list,
                                                     const uint32_t *counters, uint64_t *vis,
                                                     DomK dk, GbK gk)
{
    const uint32_t n = stream_len(scene_off, rk, cap);
    const uint32_t n_long = counters[0];
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    const uint32_t wid = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = lane_id();
    const size_t hw = (size_t)rk.W * rk.H;
    for (uint32_t e = wid; e < n_long; e += waves) {
        const uint32_t u = long_list[e];
        uint32_t s, v;
        unit_map(scene_off, rk, n, u, s, v);
        Seg sg;
        if (!load_seg(proj, flags, u, v, n, rk.r_min, sg)) continue;
        int i0, i1, j0, j1;
        if (!seg_box(sg, rk.W, rk.H, i0, i1, j0, j1)) continue;
        float zn, inv_range;
        scene_depth_consts(cams, s, zn, inv_range);
        uint64_t *vc = vis + (size_t)s * 2 * hw, *va = vc + hw;
        for (int j = j0 + lane; j <= j1; j += 64) {
            int a0, a1;
            row_span(sg, j, a0, a1);
            a0 = max(a0, i0);
            a1 = min(a1, i1);
            for (int i = a0; i <= a1; ++i) {
                uint32_t q;
                bool cc, ca;
                float ts, z;
                const bool msk = cover_tz(sg, i, j, rk.r_min, zn, inv_range, cc, ca, q, ts, z);
                const size_t p = (size_t)j * rk.W + i;
                if (DOM) {
                    if (!ca) continue;
                    const uint32_t q0 = (uint32_t)(va[p] >> HM_ID_BITS);
                    uint32_t k = q > q0 ? (q - q0) / dk.layer_codes : 0u;
                    k = k < dk.n_layers - 1u ? k : dk.n_layers - 1u;
                    atomicAdd(dk.counts + (size_t)k * hw + p, 1u);
                    continue;
                }
                if (!msk) continue;
                const uint64_t low =
                    GB ? gb_payload(gk.tan, gk.rgb, v, ts, z, sg.iz1) : (uint64_t)v;
                const uint64_t key = ((uint64_t)q << HM_ID_BITS) | low;
                if (cc) atomicMin((unsigned long long *)(vc + p), (unsigned long long)key);
                if (ca) atomicMin((unsigned long long *)(va + p), (unsigned long long)key);
            }
        }
    }
}

// ------------------------------------------------------------------ deep opacity map
// Zero the counts and rewind the work-item counter for the counting pass (the
// long-segment count of the binning, counters[0], is kept).
__global__ __launch_bounds__(256) void k_dom_clear(uint32_t *counts, uint32_t n, uint32_t *counters)
{
    const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) counters[1] = 0u;
    for (uint32_t i = i0; i < n; i += gridDim.x * blockDim.x) counts[i] = 0u;
}

// ------------------------------------------------------------------ host side
static RasterK make_rk(const hm_frame &f, const hm_raster_params &p)
{
    RasterK rk;
    rk.S = f.n_scenes;
    rk.W = f.width;
    rk.H = f.height;
    rk.r_min = p.r_min;
    rk.T = p.tile;
    rk.ntx = (f.width + p.tile - 1) / p.tile;
    rk.nty = (f.height + p.tile - 1) / p.tile;
    rk.n_tiles = rk.ntx * rk.nty * f.n_scenes;
    rk.chunk = p.chunk;
    rk.K = p.max_tiles_per_seg;
    rk.views = p.shared_views ? 1u : 0u;
    return rk;
}

// segment units per stream control point: one, or one per view
static size_t units_per_cp(const hm_frame &f, const hm_raster_params &p)
{
    return p.shared_views ? (size_t)f.n_scenes : 1u;
}

struct RasterWs {
    float4 *proj;
    uint32_t *tile_cnt;   // n_tiles + 1 (scanned in place into offsets)
    uint32_t *tile_cur;   // n_tiles
    uint32_t *items;      // n_tiles + 1 (scanned in place)
    uint32_t *partials;   // scan scratch
    uint32_t *counters;   // [0] long count, [1] work counter
    uint32_t *long_list;  // cap
    uint32_t *entries;    // cap * K
    float4 *tan;          // G-buffer keys: unit tangent per stream point (else null)
    uint2 *segrec;        // per unit: first tile of its box, box width | tile mask << 8
    uint32_t *item_tile;  // per work item: its tile
    uint32_t max_items;   // bound on the work items: n_tiles + units * K / chunk
    uint32_t *saved;      // per binning span: count, then (slot, tile, count) per occupied slot
    uint32_t nsub;        // segments per thread and span
    size_t bytes;
};

// Segments per thread between table flushes: up to BIN_SUB, fewer when that
// would leave fewer than BIN_WGS workgroups.  Measured: a 9 k-segment frame
// bins in 9 us with one segment per thread against 34 us with 8 (5
// workgroups); more workgroups than ~1024 cost more in contended per-tile
// global adds than they gain (2 M segments: 58 us at 1024 or fewer, 62 us at
// 2048, 78 us at 4096).
static uint32_t bin_nsub(size_t units)
{
    const size_t per_sub = (size_t)BIN_BLOCK * BIN_WGS;
    return (uint32_t)std::min<size_t>(std::max<size_t>(units / per_sub, 1), BIN_SUB);
}

static RasterWs carve(void *ws, const hm_frame &f, uint32_t cap, const hm_raster_params &p)
{
    const RasterK rk = make_rk(f, p);
    const size_t nt = rk.n_tiles;
    char *b = (char *)ws;
    size_t o = 0;
    RasterWs w;
    auto take = [&](size_t bytes) { char *r = b ? b + o : nullptr; o += align_up(bytes); return r; };
    const size_t units = (size_t)cap * units_per_cp(f, p);
    w.proj = (float4 *)take(sizeof(float4) * units);
    w.tile_cnt = (uint32_t *)take(sizeof(uint32_t) * (nt + 1));
    w.tile_cur = (uint32_t *)take(sizeof(uint32_t) * nt);
    w.items = (uint32_t *)take(sizeof(uint32_t) * (nt + 1));
    w.partials = (uint32_t *)take(sizeof(uint32_t) * (scan_blocks((uint32_t)nt) + 1));
    w.counters = (uint32_t *)take(sizeof(uint32_t) * 64);
    w.tan = p.payload == HM_PAYLOAD_GBUFFER ? (float4 *)take(sizeof(float4) * (size_t)cap) : nullptr;
    if (p.algo != HM_RASTER_DIRECT) {
        w.long_list = (uint32_t *)take(sizeof(uint32_t) * units);
        w.entries = (uint32_t *)take(sizeof(uint32_t) * units * p.max_tiles_per_seg);
        w.nsub = bin_nsub(units);
        const size_t spans = (units + (size_t)BIN_BLOCK * w.nsub - 1) / ((size_t)BIN_BLOCK * w.nsub);
        w.segrec = (uint2 *)take(sizeof(uint2) * units);
        w.saved = (uint32_t *)take(sizeof(uint32_t) * BIN_SAVE_WORDS * spans);
        // every list entry belongs to one item of its tile: sum over tiles of
        // ceil(count / chunk) <= n_tiles + entries / chunk
        const size_t mi = nt + (units * p.max_tiles_per_seg + p.chunk - 1) / p.chunk;
        w.max_items = (uint32_t)std::min<size_t>(mi, 0xFFFFFFFFu);
        w.item_tile = (uint32_t *)take(sizeof(uint32_t) * w.max_items);
    } else {
        w.long_list = nullptr;
        w.entries = nullptr;
        w.segrec = nullptr;
        w.saved = nullptr;
        w.item_tile = nullptr;
        w.max_items = 0;
        w.nsub = 1;
    }
    w.bytes = o;
    return w;
}

uint32_t raster_lds_bytes(const hm_raster_params &p)
{
    const bool gb = p.payload == HM_PAYLOAD_GBUFFER;
    if (p.algo == HM_RASTER_TILED)
        return flat_lds_bytes(p.tile, p.block, gb, tile_words(p.tile * tile_pitch(p.tile), false, 1u));
    return rows_lds_bytes(p.tile, p.block, gb);
}

size_t raster_workspace(const hm_frame &f, uint32_t cap, const hm_raster_params &p)
{
    return carve(nullptr, f, cap, p).bytes;
}

void raster_defaults(const hm_frame &f, hm_raster_params &p)
{
    (void)f;
    p.r_min = 0.0f;
    p.algo = HM_RASTER_TILED;
    p.tile = 32;
    p.chunk = 512;
    p.max_tiles_per_seg = 16;
    p.block = 256;
    p.grid = 0;
    p.shared_views = 0;
    p.payload = HM_PAYLOAD_SEGMENT;
}

// Prefill grid: one row of workgroups per scene (rows loop when a frame has
// more than 65535 scenes), about 4096 workgroups in all.
static dim3 prefill_grid(const hm_frame &f)
{
    const size_t hw = (size_t)f.width * f.height;
    const uint32_t rows = std::min<uint32_t>(f.n_scenes, 65535u);
    const uint32_t per = std::max<uint32_t>(1u, std::min<uint32_t>(stride_grid(hw, 256),
                                                                     4096u / rows));
    return dim3(per, rows);
}

void launch_prefill(uint64_t *vis, const float *scene_z, const hm_camera *cams,
                    const hm_frame &f, hipStream_t st)
{
    hipLaunchKernelGGL(k_prefill, prefill_grid(f), dim3(256), 0, st, vis, scene_z, cams,
                       f.n_scenes, f.width, f.height, (uint32_t *)nullptr, 0u,
                       (uint32_t *)nullptr, 0u);
}

// Offsets of the tile lists (in place over the counts) and the work items of
// every tile, after the counting pass.
static void plan_items(const RasterK &rk, const RasterWs &w, hipStream_t st)
{
    const uint32_t nt = rk.n_tiles;
    if (nt <= PLAN_SMALL) {
        hipLaunchKernelGGL(k_plan_small, dim3(1), dim3(1024), 0, st, w.tile_cnt, nt, rk.chunk,
                           w.items, w.tile_cur);
    } else {
        scan_exclusive<uint32_t>(w.tile_cnt, w.tile_cnt, nt, w.partials, st);
        hipLaunchKernelGGL(k_tile_items, dim3((nt + 255) / 256), dim3(256), 0, st,
                           (const uint32_t *)w.tile_cnt, nt, rk.chunk, w.items, w.tile_cur);
        scan_exclusive<uint32_t>(w.items, w.items, nt, w.partials, st);
    }
}

// The tile raster over the binned work items, then the long segments.
static void draw_tiles(const hm_strands &s, const hm_camera *cams, const hm_raster_params &p,
                       const RasterK &rk, const RasterWs &w, const GbK &gk, uint64_t *vis,
                       hipStream_t st)
{
    const bool gbuf = p.payload == HM_PAYLOAD_GBUFFER;
    const uint32_t lds = raster_lds_bytes(p);
    uint32_t grid = p.grid ? p.grid : 256u * 8u;
#define HM_FLAT_LAUNCH(NB, GB)                                                                 \
    hipLaunchKernelGGL((k_raster_flat<NB, false, GB>), dim3(grid), dim3(p.block), lds, st,       \
                       (const float4 *)w.proj, (const uint8_t *)s.flags, s.scene_off, cams, rk,  \
                       s.cap, (const uint32_t *)w.tile_cnt, (const uint32_t *)w.items,          \
                       (const uint32_t *)w.item_tile, (const uint32_t *)w.entries, w.counters,  \
                       vis, DomK{nullptr, 1u, 1u}, gk)
#define HM_ROWS_LAUNCH(NB, GB)                                                                 \
    hipLaunchKernelGGL((k_raster_rows<NB, GB>), dim3(grid), dim3(p.block), lds, st,              \
                       (const float4 *)w.proj, (const uint8_t *)s.flags, s.scene_off, cams, rk,  \
                       s.cap, (const uint32_t *)w.tile_cnt, (const uint32_t *)w.items,          \
                       (const uint32_t *)w.item_tile, (const uint32_t *)w.entries, w.counters,  \
                       vis, gk)
    // the default shapes compiled for their block size (fixed LDS offsets),
    // others generic
    if (p.algo == HM_RASTER_TILED) {
        if (gbuf) {
            if (p.block == 256) HM_FLAT_LAUNCH(256, true);
            else HM_FLAT_LAUNCH(0, true);
        } else {
            if (p.block == 256) HM_FLAT_LAUNCH(256, false);
            else HM_FLAT_LAUNCH(0, false);
        }
    } else if (gbuf) {
        HM_ROWS_LAUNCH(0, true);
    } else {
        if (p.block == 512) HM_ROWS_LAUNCH(512, false);
        else if (p.block == 256) HM_ROWS_LAUNCH(256, false);
        else HM_ROWS_LAUNCH(0, false);
    }
#undef HM_FLAT_LAUNCH
#undef HM_ROWS_LAUNCH
    if (gbuf)
        hipLaunchKernelGGL((k_raster_long<false, true>), dim3(256), dim3(256), 0, st,
                           (const float4 *)w.proj, (const uint8_t *)s.flags, s.scene_off, cams,
                           rk, s.cap, (const uint32_t *)w.long_list, (const uint32_t *)w.counters,
                           vis, DomK{nullptr, 1u, 1u}, gk);
    else
        hipLaunchKernelGGL((k_raster_long<false, false>), dim3(256), dim3(256), 0, st,
                           (const float4 *)w.proj, (const uint8_t *)s.flags, s.scene_off, cams,
                           rk, s.cap, (const uint32_t *)w.long_list, (const uint32_t *)w.counters,
                           vis, DomK{nullptr, 1u, 1u}, gk);
}

void launch_raster(const hm_strands &s, const hm_camera *cams, const hm_frame &f,
                   const hm_raster_params &p, const float *scene_z, uint64_t *vis, void *ws,
                   hipStream_t st)
{
    const RasterK rk = make_rk(f, p);
    RasterWs w = carve(ws, f, s.cap, p);
    const bool tiled = p.algo != HM_RASTER_DIRECT;
    // tiled: the binning counters are cleared first and the buffer is
    // prefilled by extra workgroups of the first binning pass
    if (tiled)
        hipLaunchKernelGGL(k_prefill, dim3(1), dim3(256), 0, st, vis, scene_z, cams, 0u,
                           f.width, f.height, w.tile_cnt, rk.n_tiles + 1, w.counters, 64u);
    else
        hipLaunchKernelGGL(k_prefill, prefill_grid(f), dim3(256), 0, st, vis, scene_z, cams,
                           f.n_scenes, f.width, f.height, (uint32_t *)nullptr, 0u,
                           (uint32_t *)nullptr, 0u);
    const float4 *pos = reinterpret_cast<const float4 *>(s.pos_w);
    const size_t units = (size_t)s.cap * units_per_cp(f, p);
    const bool gbuf = p.payload == HM_PAYLOAD_GBUFFER;
    const GbK gk{w.tan, reinterpret_cast<const float4 *>(s.rgb)};
    if (gbuf)
        hipLaunchKernelGGL(k_cp_tangent, dim3(stride_grid(s.cap, 256)), dim3(256), 0, st, pos,
                           (const uint8_t *)s.flags, s.scene_off, rk, s.cap, w.tan);
    if (p.algo == HM_RASTER_DIRECT) {
        hipLaunchKernelGGL(k_project, dim3(stride_grid(units, 256)), dim3(256), 0, st, pos,
                           s.scene_off, rk, cams, s.cap, w.proj);
        if (gbuf)
            hipLaunchKernelGGL(k_raster_direct<true>, dim3(stride_grid(units, 256)), dim3(256), 0,
                               st, (const float4 *)w.proj, (const uint8_t *)s.flags, s.scene_off,
                               cams, rk, s.cap, vis, gk);
        else
            hipLaunchKernelGGL(k_raster_direct<false>, dim3(stride_grid(units, 256)), dim3(256),
                               0, st, (const float4 *)w.proj, (const uint8_t *)s.flags,
                               s.scene_off, cams, rk, s.cap, vis, gk);
        return;
    }
    // pass 0 of the binning also writes every unit's screen record
    const uint32_t nt = rk.n_tiles;
    const uint32_t nsub = w.nsub;
    const uint32_t gb = stride_grid((units + nsub - 1) / nsub, BIN_BLOCK);
    // the prefill grid holds as many threads as the prefill kernel's own
    dim3 pg = prefill_grid(f);
    pg.x = std::max<uint32_t>(1u, pg.x * 256u / BIN_BLOCK);
    const PrefillK pf{vis, scene_z, pg.x, pg.y};
    hipLaunchKernelGGL(k_bin, dim3(gb + pg.x * pg.y), dim3(BIN_BLOCK), 0, st, 0, w.proj, pos,
                       cams, (const uint8_t *)s.flags, s.scene_off, rk, s.cap, w.tile_cnt,
                       (const uint32_t *)nullptr, w.tile_cur, w.entries, w.long_list, w.counters,
                       nsub, w.segrec, w.saved, (const uint32_t *)nullptr, (uint32_t *)nullptr, 0u,
                       gb, pf);
    plan_items(rk, w, st);
    hipLaunchKernelGGL(k_bin, dim3(gb), dim3(BIN_BLOCK), 0, st, 1, w.proj, pos, cams,
                       (const uint8_t *)s.flags, s.scene_off, rk, s.cap, w.tile_cnt,
                       (const uint32_t *)w.tile_cnt, w.tile_cur, w.entries, w.long_list,
                       w.counters, nsub, w.segrec, w.saved, (const uint32_t *)w.items, w.item_tile,
                       w.max_items, gb, PrefillK{nullptr, nullptr, 1u, 1u});
    draw_tiles(s, cams, p, rk, w, gk, vis, st);
}

// Strand generation that bins as it writes (pass 0 of the binning done by the
// generator's workgroups), then the scatter over the generator's spans and
// the tile raster: the same buffer as generate + raster (single-view frames,
// tiled algorithm with segment ids).  Workspace: the raster's plus one saved
// table per generator workgroup.
size_t gen_raster_workspace(uint32_t n_bundles, const hm_frame &f, uint32_t cap,
                            const hm_raster_params &p)
{
    return raster_workspace(f, cap, p) +
           align_up(sizeof(uint32_t) * (size_t)BIN_SAVE_WORDS * gen_grid(n_bundles, cap));
}

void launch_gen_raster_tiled(const hm_hair_mesh &m, const uint32_t *table,
                             const uint32_t *strand_base, const float *strand_rgb,
                             const hm_gen_params &gp, const hm_strands &s, const hm_camera *cams,
                             const hm_frame &f, const hm_raster_params &p, const float *scene_z,
                             uint64_t *vis, void *ws, hipStream_t st)
{
    const RasterK rk = make_rk(f, p);
    const RasterWs w = carve(ws, f, s.cap, p);
    uint32_t *saved = reinterpret_cast<uint32_t *>((char *)ws + raster_workspace(f, s.cap, p));
    hipLaunchKernelGGL(k_prefill, prefill_grid(f), dim3(256), 0, st, vis, scene_z, cams,
                       f.n_scenes, f.width, f.height, w.tile_cnt, rk.n_tiles + 1, w.counters,
                       64u);
    const BinK bk{rk,         cams,          w.proj,   w.segrec,
                  w.tile_cnt, w.long_list,   w.counters, saved,
                  rk.K < BIN_KMAX ? rk.K : BIN_KMAX};
    launch_generate_bin(m, table, strand_base, strand_rgb, gp, s, bk, st);
    plan_items(rk, w, st);
    hipLaunchKernelGGL(k_bin_spans, dim3(gen_grid(m.n_bundles, s.cap)), dim3(BIN_BLOCK), 0, st,
                       rk, table, m.n_bundles, gen_bundles_per_group(m.n_bundles, s.cap),
                       s.scene_off, s.cap,
                       (const uint32_t *)w.tile_cnt, w.tile_cur, w.entries,
                       (const uint2 *)w.segrec, (const uint32_t *)saved,
                       (const uint32_t *)w.items, w.item_tile, w.max_items);
    const GbK gk{nullptr, reinterpret_cast<const float4 *>(s.rgb)};
    draw_tiles(s, cams, p, rk, w, gk, vis, st);
}

}  // namespace hm


namespace hm {

// LDS of the counting pass: the first-fragment code and one count per layer
// for every pixel of the tile instead of two 64-bit layers.
static uint32_t dom_lds_bytes(uint32_t T, uint32_t n_layers)
{
    return flat_lds_bytes(T, 256u, false, tile_words(T * tile_pitch(T), true, n_layers));
}

// Raster shape of the light view: the defaults, with 16-pixel tiles when the
// counting pass's LDS for 32-pixel tiles would exceed 64 KiB (many layers).
static hm_raster_params dom_raster_params(const hm_frame &lf, const hm_dom_params &p)
{
    hm_raster_params rp;
    raster_defaults(lf, rp);
    rp.r_min = p.r_min;
    if (dom_lds_bytes(rp.tile, p.n_layers) > 65536u) rp.tile = 16;
    return rp;
}

static hm_frame dom_frame(const hm_dom_params &p)
{
    hm_frame f;
    f.n_scenes = 1;
    f.width = p.width;
    f.height = p.height;
    return f;
}

size_t dom_workspace(const hm_frame &lf, uint32_t cap)
{
    hm_raster_params rp;
    raster_defaults(lf, rp);
    return raster_workspace(lf, cap, rp);
}

// The light view is rasterized by the raster path (its bins stay in the
// workspace), then the same work items are walked again by the counting pass
// of the tile kernel, with the completed conservative layer as q0.
void launch_dom_accum(const hm_strands &s, const hm_camera *light, const hm_dom_params &p,
                      uint64_t *light_vis, uint32_t *counts, void *ws, hipStream_t st)
{
    const hm_frame f = dom_frame(p);
    const hm_raster_params rp = dom_raster_params(f, p);
    launch_raster(s, light, f, rp, nullptr, light_vis, ws, st);
    const RasterK rk = make_rk(f, rp);
    RasterWs w = carve(ws, f, s.cap, rp);
    const size_t n = (size_t)p.width * p.height * p.n_layers;
    hipLaunchKernelGGL(k_dom_clear, dim3(stride_grid(n, 256)), dim3(256), 0, st, counts,
                       (uint32_t)n, w.counters);
    const DomK dk{counts, p.layer_codes, p.n_layers};
    const uint32_t lds = dom_lds_bytes(rp.tile, p.n_layers);
    hipLaunchKernelGGL((k_raster_flat<256, true, false>), dim3(256u * 8u), dim3(256), lds, st,
                       (const float4 *)w.proj, (const uint8_t *)s.flags, s.scene_off, light, rk,
                       s.cap, (const uint32_t *)w.tile_cnt, (const uint32_t *)w.items,
                       (const uint32_t *)w.item_tile, (const uint32_t *)w.entries, w.counters,
                       light_vis, dk, GbK{nullptr, nullptr});
    hipLaunchKernelGGL((k_raster_long<true, false>), dim3(256), dim3(256), 0, st,
                       (const float4 *)w.proj, (const uint8_t *)s.flags, s.scene_off, light, rk,
                       s.cap, (const uint32_t *)w.long_list, (const uint32_t *)w.counters,
                       light_vis, dk, GbK{nullptr, nullptr});
}

}  // namespace hm
