// Screen-tile binning shared by the tile raster's binning kernel and the
// generator that bins the strands it writes: the tile grid, segment units,
// the tile box of a segment and its separating-axis tile test, and the LDS
// hash table that aggregates (segment, tile) pairs per workgroup.
#pragma once

#include "hm_device.hpp"

namespace hm {

// One raster call's frame, tile grid and binning parameters (built on the
// host, passed by value).
struct RasterK {
    uint32_t S, W, H;
    float r_min;
    uint32_t T, ntx, nty, n_tiles;
    uint32_t chunk, K;
    uint32_t views;     // 0: scene s draws stream range scene_off[s..s+1];
                        // 1: every scene (view) draws the whole stream
};

// Segment space.  A unit u names (scene, stream control point v); screen
// records, bin entries and long-list entries are indexed by u, keys carry v.
//   views == 0: u = v, scene from the scene offsets;
//   views == 1: u = s * n + v over S views of one stream of n points.
__device__ __forceinline__ uint32_t stream_len(const uint32_t *scene_off, const RasterK &rk,
                                               uint32_t cap)
{
    const uint32_t total = rk.views ? scene_off[1] : scene_off[rk.S];
    return total < cap ? total : cap;
}

__device__ __forceinline__ uint32_t unit_count(uint32_t n, const RasterK &rk)
{
    return rk.views ? n * rk.S : n;
}

__device__ __forceinline__ void unit_map(const uint32_t *scene_off, const RasterK &rk, uint32_t n,
                                         uint32_t u, uint32_t &s, uint32_t &v)
{
    if (rk.views) {
        s = u / n;
        v = u - s * n;
    } else {
        v = u;
        s = scene_of(scene_off, rk.S, u);
    }
}

// Tile-box test: can the segment reach any pixel of tile box [px0, px1) x
// [py0, py1)?  Separating axes x, y and the segment normal on the box widened
// by ra + 1 px (a superset of both predicates' support).
__device__ __forceinline__ bool seg_hits_box(const Seg &sg, float px0, float px1, float py0,
                                             float py1)
{
    const float m = sg.ra + 1.0f;
    const float bx0 = px0 - m, bx1 = px1 + m, by0 = py0 - m, by1 = py1 + m;
    if (!(sg.sxmn <= bx1 && sg.sxmx >= bx0 && sg.symn <= by1 && sg.symx >= by0)) return false;
    const float fa = (bx0 - sg.x0) * sg.dy, fb = (bx1 - sg.x0) * sg.dy;
    const float ga = (by0 - sg.y0) * sg.dx, gb = (by1 - sg.y0) * sg.dx;
    const float lo = fminx(fa, fb) - fmaxx(ga, gb);
    const float hi = fmaxx(fa, fb) - fminx(ga, gb);
    // widen the sign test by a relative slack against rounding
    const float slack = 1e-4f * (fabsf(fa) + fabsf(fb) + fabsf(ga) + fabsf(gb)) + 1e-3f;
    return lo <= slack && hi >= -slack;
}

// Tiles of one segment: the box [tx0, tx1] x [ty0, ty1] of tiles its candidate
// pixels fall in (nt = 0: nothing to draw; nt > K: a long segment).
struct SegTiles {
    Seg sg;
    uint32_t s, tx0, ty0, bw, nt;
};

// Tile box of the segment between screen records a and b (scene s): the
// fields of make_seg that the tile tests read, computed the same way.  False
// when a point lies outside the depth range (w = 0) or the box misses the
// frame.
__device__ __forceinline__ bool seg_tiles_of(float4 a, float4 b, uint32_t s, const RasterK &rk,
                                             SegTiles &st)
{
    st.nt = 0;
    st.s = s;
    if (a.w == 0.0f || b.w == 0.0f) return false;
    Seg &sg = st.sg;
    sg = Seg{};
    sg.x0 = a.x;
    sg.y0 = a.y;
    sg.dx = b.x - a.x;
    sg.dy = b.y - a.y;
    sg.ra = fmaxx(0.5f * fmaxx(a.z, b.z), rk.r_min);
    sg.sxmn = fminx(a.x, b.x); sg.sxmx = fmaxx(a.x, b.x);
    sg.symn = fminx(a.y, b.y); sg.symx = fmaxx(a.y, b.y);
    int i0, i1, j0, j1;
    if (!seg_box(st.sg, rk.W, rk.H, i0, i1, j0, j1)) return false;
    st.tx0 = (uint32_t)i0 / rk.T;
    st.ty0 = (uint32_t)j0 / rk.T;
    st.bw = (uint32_t)i1 / rk.T - st.tx0 + 1;
    st.nt = st.bw * ((uint32_t)j1 / rk.T - st.ty0 + 1);
    return true;
}

// Tile (tx0 + kx, ty0 + ky) of the segment's tile box; returns false when the
// segment cannot reach it.  A box of a single tile needs no test (an extra
// pair would be harmless: the raster tests every pixel exactly).
__device__ __forceinline__ bool seg_tile_at(const SegTiles &st, const RasterK &rk, uint32_t kx,
                                            uint32_t ky, uint32_t &tile)
{
    const uint32_t tx = st.tx0 + kx, ty = st.ty0 + ky;
    tile = (st.s * rk.nty + ty) * rk.ntx + tx;
    if (st.nt == 1u) return true;
    const float px0 = (float)(tx * rk.T), py0 = (float)(ty * rk.T);
    return seg_hits_box(st.sg, px0, px0 + (float)rk.T, py0, py0 + (float)rk.T);
}

constexpr uint32_t BIN_SLOTS = 1024;      // LDS hash slots per workgroup
constexpr uint32_t BIN_FREE = 0xFFFFFFFFu;
constexpr uint32_t BIN_KMAX = 24;         // tile-mask bits in a segment record
constexpr uint32_t BIN_NONE = 0xFFFFFFFFu;

// Slot of `tile` in the workgroup's LDS table (linear probing), -1 if full.
__device__ __forceinline__ int bin_slot(uint32_t *keys, uint32_t tile)
{
    const uint32_t h = (tile * 2654435761u) >> 22;          // 10 bits
    for (uint32_t i = 0; i < BIN_SLOTS; ++i) {
        const uint32_t sl = (h + i) & (BIN_SLOTS - 1);
        const uint32_t prev = atomicCAS(&keys[sl], BIN_FREE, tile);
        if (prev == BIN_FREE || prev == tile) return (int)sl;
    }
    return -1;
}

__device__ __forceinline__ int bin_find(const uint32_t *keys, uint32_t tile)
{
    const uint32_t h = (tile * 2654435761u) >> 22;
    for (uint32_t i = 0; i < BIN_SLOTS; ++i) {
        const uint32_t q = (h + i) & (BIN_SLOTS - 1);
        const uint32_t kq = keys[q];
        if (kq == tile) return (int)q;
        if (kq == BIN_FREE) return -1;
    }
    return -1;
}

// Binning done by the strand generator (single-view streams): where the
// screen records, unit records, tile counts and long list go, and per
// generator workgroup its saved table (count, then (slot, tile, count) of
// each occupied slot) for the scatter pass.
struct BinK {
    RasterK rk;
    const hm_camera *cams;
    float4 *proj;
    uint2 *segrec;
    uint32_t *tile_cnt;
    uint32_t *long_list;
    uint32_t *counters;
    uint32_t *saved;
    uint32_t kmax;
};
constexpr uint32_t BIN_SAVE_WORDS = 1u + 3u * BIN_SLOTS;

// Counting step of one segment unit u (ok: st holds its tile box): a box of
// more than kmax tiles goes to the long list; otherwise each accepted tile is
// counted in the LDS table (in the global counts when the table is full).
// Returns the unit's 8-byte record: the first tile of its box and the box
// width | accepted-tile mask << 8 (BIN_NONE: nothing to scatter).
__device__ __forceinline__ uint2 bin_count(const SegTiles &st, bool ok, uint32_t u,
                                           const RasterK &rk, uint32_t kmax, uint32_t *keys,
                                           uint32_t *cnt, uint32_t *tile_cnt,
                                           uint32_t *long_list, uint32_t *counters)
{
    if (ok && st.nt > kmax) {
        long_list[atomicAdd(&counters[0], 1u)] = u;
        ok = false;
    }
    uint2 rec = make_uint2(BIN_NONE, 0u);
    if (ok) {
        uint32_t mask = 0, tile0 = 0;
        for (uint32_t ky = 0, k = 0; k < st.nt; ++ky)
        for (uint32_t kx = 0; kx < st.bw; ++kx, ++k) {
            uint32_t tile;
            const bool hit = seg_tile_at(st, rk, kx, ky, tile);
            if (k == 0) tile0 = tile;
            if (!hit) continue;
            mask |= 1u << k;
            const int sl = bin_slot(keys, tile);
            if (sl >= 0) atomicAdd(&cnt[sl], 1u);
            else atomicAdd(&tile_cnt[tile], 1u);
        }
        if (mask) rec = make_uint2(tile0, st.bw | (mask << 8));
    }
    return rec;
}

// Scatter step of unit u with record rec: each accepted tile gets u at a rank
// inside the range its table slot reserved (basev), or at a global rank when
// the tile missed the table.
__device__ __forceinline__ void bin_scatter(uint2 rec, uint32_t u, const RasterK &rk,
                                            const uint32_t *keys, uint32_t *cnt,
                                            const uint32_t *basev, const uint32_t *tile_off,
                                            uint32_t *tile_cur, uint32_t *entries)
{
    if (rec.x == BIN_NONE) return;
    const uint32_t bw = rec.y & 0xFFu;
    uint32_t mask = rec.y >> 8;
    while (mask) {
        const uint32_t k = (uint32_t)__builtin_ctz(mask);
        mask &= mask - 1u;
        const uint32_t ky = k / bw, kx = k - ky * bw;
        const uint32_t tile = rec.x + ky * rk.ntx + kx;
        const int sl = bin_find(keys, tile);
        if (sl >= 0) entries[basev[sl] + atomicAdd(&cnt[sl], 1u)] = u;
        else entries[tile_off[tile] + atomicAdd(&tile_cur[tile], 1u)] = u;
    }
}

}  // namespace hm
