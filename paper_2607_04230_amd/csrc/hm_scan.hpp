// Device-wide exclusive prefix sum (three passes: block scans, a single-block
// scan of the block totals, and a fix-up).  out has n + 1 entries; out[n]
// receives the total.  In-place (in == out) is allowed.
#pragma once

#include "hm_device.hpp"

namespace hm {

constexpr uint32_t SCAN_BLOCK = 256;
constexpr uint32_t SCAN_ITEMS = 4;
constexpr uint32_t SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <typename T>
__global__ __launch_bounds__(256) void k_scan_blocks(const T *in, T *out, uint32_t n, T *partials)
{
    __shared__ T lds[SCAN_BLOCK / 64 + 1];
    const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T s = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? in[base + k] : (T)0;
        s += v[k];
    }
    T tot;
    T run = block_exclusive_scan(s, lds, tot);
#pragma unroll
    for (uint32_t k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_partials(T *partials, uint32_t nb, T *total_out)
{
    __shared__ T lds[SCAN_BLOCK / 64 + 1];
    T carry = 0;
    for (uint32_t c0 = 0; c0 < nb; c0 += SCAN_TILE) {
        const uint32_t base = c0 + threadIdx.x * SCAN_ITEMS;
        T v[SCAN_ITEMS];
        T s = 0;
#pragma unroll
        for (uint32_t k = 0; k < SCAN_ITEMS; ++k) {
            v[k] = (base + k < nb) ? partials[base + k] : (T)0;
            s += v[k];
        }
        T tot;
        T run = block_exclusive_scan(s, lds, tot) + carry;
#pragma unroll
        for (uint32_t k = 0; k < SCAN_ITEMS; ++k) {
            if (base + k < nb) partials[base + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_add(T *out, uint32_t n, const T *partials)
{
    const T add = partials[blockIdx.x];
    const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) out[base + k] += add;
}

inline uint32_t scan_blocks(uint32_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

// partials: scan_blocks(n) entries of scratch.
template <typename T>
inline void scan_exclusive(const T *in, T *out, uint32_t n, T *partials, hipStream_t st)
{
    const uint32_t nb = scan_blocks(n) ? scan_blocks(n) : 1;
    hipLaunchKernelGGL(k_scan_blocks<T>, dim3(nb), dim3(SCAN_BLOCK), 0, st, in, out, n, partials);
    hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(SCAN_BLOCK), 0, st, partials, nb, out + n);
    hipLaunchKernelGGL(k_scan_add<T>, dim3(nb), dim3(SCAN_BLOCK), 0, st, out, n,
                       (const T *)partials);
}

}  // namespace hm
