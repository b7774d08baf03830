// Peak-rate microkernels for the raster's rooflines: 64-bit atomic minima in
// LDS (lane-distinct, consecutive addresses, as the tile raster's candidate
// pixels are) and in global memory (addresses spread pseudo-randomly over the
// caller's buffer); and read-only / write-only streams of known size that
// calibrate the profiler's byte counters.  Measurement helpers only; nothing
// on the rendering path calls them.
#include <hip/hip_runtime.h>

#include "hm_bench.h"
#include "hm_device.hpp"
#include "hm_internal.hpp"

namespace hm {

constexpr uint32_t BENCH_LDS_WORDS = 2048;

__global__ __launch_bounds__(256) void k_bench_lds_min(uint32_t iters, unsigned long long *sink)
{
    __shared__ unsigned long long t[BENCH_LDS_WORDS];
    for (uint32_t x = threadIdx.x; x < BENCH_LDS_WORDS; x += blockDim.x) t[x] = ~0ull;
    __syncthreads();
    unsigned long long v = (unsigned long long)(blockIdx.x * blockDim.x + threadIdx.x) *
                           0x9E3779B97F4A7C15ull;
    for (uint32_t i = 0; i < iters; ++i) {
        atomicMin(&t[(threadIdx.x + i * blockDim.x) & (BENCH_LDS_WORDS - 1)], v);
        v = v * 6364136223846793005ull + 1442695040888963407ull;
    }
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = t[blockIdx.x & (BENCH_LDS_WORDS - 1)];
}

__global__ __launch_bounds__(256) void k_bench_global_min(unsigned long long *buf, uint64_t n,
                                                          uint32_t iters)
{
    uint64_t h = (uint64_t)(blockIdx.x * blockDim.x + threadIdx.x) * 0x9E3779B97F4A7C15ull + 1;
    for (uint32_t i = 0; i < iters; ++i) {
        h ^= h >> 33;
        h *= 0xff51afd7ed558ccdull;
        h ^= h >> 29;
        atomicMin(buf + (h % n), (unsigned long long)h);
    }
}

// Known-size memory traffic for calibrating the byte counters of the
// profiler: k_bench_read reads n 16-byte words once (one word per lane per
// step, consecutive lanes on consecutive words) and writes one 32-bit word per
// workgroup; k_bench_write writes n 16-byte words once.
__global__ __launch_bounds__(256) void k_bench_read(const uint4 *buf, uint64_t n, uint32_t *sink)
{
    __shared__ uint32_t red;
    if (threadIdx.x == 0) red = 0u;
    __syncthreads();
    uint32_t acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint4 v = buf[i];
        acc ^= (v.x ^ v.y) ^ (v.z ^ v.w);
    }
    atomicXor(&red, acc);
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = red;
}

__global__ __launch_bounds__(256) void k_bench_write(uint4 *buf, uint64_t n, uint32_t val)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        buf[i] = make_uint4(val, val ^ (uint32_t)i, val, (uint32_t)(i >> 32));
}

// Exceptions of the refined reciprocal: every binary32 bit pattern in [lo, hi)
// is tested against the correctly rounded quotient 1.0f / x (bitwise);
// counts[0] += mismatches, counts[1] += values tested (one add each per
// workgroup).
__global__ __launch_bounds__(256) void k_bench_reciprocal(uint32_t lo, uint32_t hi,
                                                          uint32_t *counts)
{
    __shared__ uint32_t red[2];
    if (threadIdx.x < 2) red[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t bad = 0, seen = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = (uint64_t)lo + blockIdx.x * blockDim.x + threadIdx.x; b < hi; b += stride) {
        const float x = __uint_as_float((uint32_t)b);
        bad += __float_as_uint(rcp_refined(x)) != __float_as_uint(1.0f / x) ? 1u : 0u;
        ++seen;
    }
    atomicAdd(&red[0], bad);
    atomicAdd(&red[1], seen);
    __syncthreads();
    if (threadIdx.x < 2) atomicAdd(counts + threadIdx.x, red[threadIdx.x]);
}

}  // namespace hm

using namespace hm;

extern "C" hm_status hm_bench_reciprocal(uint32_t lo, uint32_t hi, uint32_t *counts,
                                         void *stream)
{
    if (!counts || lo >= hi) return HM_ERR_INVALID;
    hipLaunchKernelGGL(k_bench_reciprocal, dim3(8192), dim3(256), 0, (hipStream_t)stream, lo, hi,
                       counts);
    return hipGetLastError() == hipSuccess ? HM_OK : HM_ERR_HIP;
}

extern "C" hm_status hm_bench_traffic(int32_t kind, void *buf, size_t bytes, uint32_t *sink,
                                      uint32_t grid, void *stream)
{
    if (!buf || bytes == 0 || bytes % 16 != 0 || grid == 0 || grid > 65536)
        return HM_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t n = bytes / 16;
    if (kind == 0) {
        if (!sink) return HM_ERR_INVALID;
        hipLaunchKernelGGL(k_bench_read, dim3(grid), dim3(256), 0, st,
                           reinterpret_cast<const uint4 *>(buf), n, sink);
    } else if (kind == 1) {
        hipLaunchKernelGGL(k_bench_write, dim3(grid), dim3(256), 0, st,
                           reinterpret_cast<uint4 *>(buf), n, 0x5A5A5A5Au);
    } else {
        return HM_ERR_INVALID;
    }
    return hipGetLastError() == hipSuccess ? HM_OK : HM_ERR_HIP;
}

extern "C" hm_status hm_bench_atomics(int32_t kind, uint64_t *buf, size_t n_words, uint32_t iters,
                                      uint32_t grid, void *stream)
{
    if (!buf || iters == 0 || grid == 0 || grid > 65536) return HM_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    if (kind == 0) {
        if (n_words < grid) return HM_ERR_RANGE;
        hipLaunchKernelGGL(k_bench_lds_min, dim3(grid), dim3(256), 0, st, iters,
                           reinterpret_cast<unsigned long long *>(buf));
    } else if (kind == 1) {
        if (n_words == 0) return HM_ERR_RANGE;
        hipLaunchKernelGGL(k_bench_global_min, dim3(grid), dim3(256), 0, st,
                           reinterpret_cast<unsigned long long *>(buf), (uint64_t)n_words, iters);
    } else {
        return HM_ERR_INVALID;
    }
    return hipGetLastError() == hipSuccess ? HM_OK : HM_ERR_HIP;
}
