// Device helpers shared by the operator and solver kernels (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "fewha_internal.h"

namespace fewha {

__device__ __forceinline__ int pmod(int a, int m) {
    const int r = a % m;
    return r < 0 ? r + m : r;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Block (kThreads) reduction of NV register values; thread k < NV writes
// part[(slot0 + k) * stride + col].  Fixed shuffle/LDS tree: deterministic.
template <int NV>
__device__ __forceinline__ void block_partials(const double (&v)[NV], double* __restrict__ part, int slot0,
                                               int stride, int col) {
    __shared__ double sh[NV > 0 ? NV : 1][kThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) sh[k][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        part[size_t(slot0 + k) * stride + col] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
    }
    __syncthreads();
}

// Fixed-order sum of `count` (>= 1) consecutive doubles by a whole block (every thread gets
// it).  Four unconditional loads per step (clamped index, zeroed by a factor), so that they
// are in flight together.
__device__ __forceinline__ double block_sum_array(const double* __restrict__ a, int count) {
    __shared__ double sh[kThreads / 64];
    double v = 0;
    for (int b0 = 0; b0 < count; b0 += 4 * kThreads) {
        double x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int b = b0 + k * kThreads + threadIdx.x;
            x[k] = a[b < count ? b : count - 1] * (b < count ? 1.0 : 0.0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) v += x[k];
    }
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// Copies `count` (>= 1) values into LDS with NT threads: every load of a thread is issued,
// unconditionally (clamped index), before its first LDS store, so the global latencies overlap
// instead of adding up (count <= NT * MAXPER).
template <int NT, int MAXPER, typename T, typename Src, typename Dst>
__device__ __forceinline__ void stage_to_lds(int count, Src src, Dst dst) {
    T v[MAXPER];
#pragma unroll
    for (int k = 0; k < MAXPER; ++k) {
        const int e = threadIdx.x + k * NT;
        v[k] = src(e < count ? e : count - 1);
    }
#pragma unroll
    for (int k = 0; k < MAXPER; ++k) {
        const int e = threadIdx.x + k * NT;
        if (e < count) dst(e, v[k]);
    }
}

}  // namespace fewha
