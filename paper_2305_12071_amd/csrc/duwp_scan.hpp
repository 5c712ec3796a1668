// Exclusive scan of per-cell int32 counts into int64 offsets [G+1]:
// tile sums, a one-block scan of the tile sums, then per-tile scans.
// Offsets are clamped to the capacity so later kernels stay in bounds.
#pragma once

#include <hip/hip_runtime.h>

#include "duwp_device.hpp"

namespace duwp {

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_TILE = SCAN_ITEMS * SCAN_BLOCK;

__device__ __forceinline__ int64_t block_exclusive_scan64(int64_t v, int64_t *lds, int64_t *total)
{
    const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int64_t n = __shfl_up(incl, o, WAVE);
        if (lane >= o) incl += n;
    }
    __syncthreads();
    if (lane == WAVE - 1) lds[w] = incl;
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) base += lds[i];
        tot += lds[i];
    }
    *total = tot;
    return base + incl - v;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const int32_t *__restrict__ in, int G,
                                                            int64_t *__restrict__ part)
{
    __shared__ double red[8];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    double s[1] = {0.0};
    int64_t si = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (t0 + i < G) si += in[t0 + i];
    s[0] = (double)si;   // exact: counts stay far below 2^53
    block_sum<1>(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = (int64_t)s[0];
}

__global__ void __launch_bounds__(1024) k_scan_partials(int64_t *part, int n)
{
    __shared__ int64_t lds[16];
    int64_t carry = 0;
    for (int i0 = 0; i0 < n; i0 += blockDim.x) {
        int i = i0 + threadIdx.x;
        int64_t v = i < n ? part[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan64(v, lds, &tot);
        if (i < n) part[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_apply(const int32_t *__restrict__ in, int G,
                                                           const int64_t *__restrict__ part,
                                                           int64_t *__restrict__ out, int64_t cap,
                                                           int64_t *total, int32_t *err)
{
    __shared__ int64_t lds[8];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (t0 + i < G) ? in[t0 + i] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t run = part[blockIdx.x] + block_exclusive_scan64(s, lds, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        // offsets are clamped to the capacity so that later kernels stay in bounds
        if (t0 + i < G) out[t0 + i] = run < cap ? run : cap;
        run += v[i];
        if (t0 + i == G - 1) {
            out[G] = run < cap ? run : cap;
            *total = run;
            if (run > cap) atomicOr(err, ERR_CAPACITY);
        }
    }
}

// Whole scan in one block of 1024 threads when G <= 8 * 1024.
constexpr int SCAN1_ITEMS = 8;
constexpr int SCAN1_MAX = SCAN1_ITEMS * 1024;

__global__ void __launch_bounds__(1024) k_scan_single(const int32_t *__restrict__ in, int G,
                                                      int64_t *__restrict__ out, int64_t cap, int64_t *total,
                                                      int32_t *err)
{
    __shared__ int64_t lds[16];
    const int t0 = threadIdx.x * SCAN1_ITEMS;
    int64_t v[SCAN1_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN1_ITEMS; ++i) {
        v[i] = (t0 + i < G) ? in[t0 + i] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t run = block_exclusive_scan64(s, lds, &tot);
#pragma unroll
    for (int i = 0; i < SCAN1_ITEMS; ++i) {
        if (t0 + i < G) out[t0 + i] = run < cap ? run : cap;
        run += v[i];
        if (t0 + i == G - 1) {
            out[G] = run < cap ? run : cap;
            *total = run;
            if (run > cap) atomicOr(err, ERR_CAPACITY);
        }
    }
}

}  // namespace duwp
