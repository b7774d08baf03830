/* Measurement helpers of libhm (not part of the rendering method).
 *
 * The tile raster resolves each covered (segment, pixel, layer) pair with one
 * 64-bit atomic minimum in LDS and merges split tiles with 64-bit global
 * atomic minima (Sec. 3.1.2's atomic-min visibility buffer); these kernels
 * measure the device's peak rates of those two operations so that the
 * benchmark can place the raster against them; the known-size streams
 * calibrate the profiler's HBM byte counters. */
#ifndef HM_BENCH_H
#define HM_BENCH_H

#include <stddef.h>
#include <stdint.h>

#include "hm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Enqueue grid workgroups of 256 threads, each thread doing `iters` 64-bit
 * atomic minima, on `stream` (the caller times it).
 * kind 0: in LDS, lane-distinct consecutive addresses; buf (device, at
 *   least grid words) receives one word per workgroup.
 * kind 1: in global memory over buf[n_words] (device, caller-owned, its
 *   contents are overwritten by minima), pseudo-random addresses.
 * Returns HM_ERR_INVALID / HM_ERR_RANGE for bad arguments, HM_ERR_HIP if the
 * launch failed.  Atomics performed: grid * 256 * iters. */
hm_status hm_bench_atomics(int32_t kind, uint64_t *buf, size_t n_words, uint32_t iters,
                           uint32_t grid, void *stream);

/* Enqueue grid workgroups of 256 threads streaming `bytes` (a multiple of 16)
 * of the device buffer buf once, on `stream`:
 * kind 0: read only (16 B per lane per step); sink (device, at least grid
 *   32-bit words) receives one word per workgroup;
 * kind 1: write only, buf is overwritten.
 * Known-size traffic for calibrating the profiler's byte counters (FETCH_SIZE,
 * WRITE_SIZE).  Returns HM_ERR_INVALID for bad arguments, HM_ERR_HIP if the
 * launch failed. */
hm_status hm_bench_traffic(int32_t kind, void *buf, size_t bytes, uint32_t *sink, uint32_t grid,
                           void *stream);

/* Check of the raster's refined reciprocal (the hardware reciprocal plus one
 * Newton step, used for the depth 1/z when the camera's depth range keeps
 * every 1/z within [2^-126, 2^126)): every binary32 bit pattern x in
 * [lo, hi) (lo < hi; the positive normal range is 0x00800000 .. 0x7F800000)
 * is compared bit for bit with the correctly rounded 1.0f / x.  counts
 * (device, two uint32, zeroed by the caller): counts[0] += mismatches,
 * counts[1] += values tested.  Returns HM_ERR_INVALID for bad arguments,
 * HM_ERR_HIP if the launch failed. */
hm_status hm_bench_reciprocal(uint32_t lo, uint32_t hi, uint32_t *counts, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HM_BENCH_H */
