// Device helpers shared by the operator and solver kernels (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "fewha_internal.h"

namespace fewha {

// The value v holds in lane `lane` (wave-uniform), in every lane: a read of that lane's
// register into scalar registers.
__device__ __forceinline__ double lane_value(double v, int lane) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffull), lane));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// v of the lane CTRL's row shift names (DPP row_shr), 0 where the shift leaves the row of 16.
template <int CTRL>
__device__ __forceinline__ double dpp_row_shr(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffull), CTRL, 0xf, 0xf, true));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, true));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// v of the lane that DPP control CTRL names, with every row of 16 lanes enabled (for the row
// rotations: every lane reads a lane of its own row).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffull), CTRL, 0xf, 0xf, false));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, false));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// v of the lane CTRL names (DPP row broadcast) in the rows ROWS selects (bit r: row r of 16
// lanes), 0 in the other rows.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffull), CTRL, ROWS, 0xf, false));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROWS, 0xf, false));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Sum over the 64 lanes of a full wavefront, in every lane, in a fixed order: inclusive sums
// within each row of 16 lanes by data-parallel row shifts of 1, 2, 4 and 8 (lane 15 of a row
// then holds the row's sum), then (row0 + row1) + (row2 + row3).  No LDS traffic.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_row_shr<0x111>(v);
    v += dpp_row_shr<0x112>(v);
    v += dpp_row_shr<0x114>(v);
    v += dpp_row_shr<0x118>(v);
    return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}

// Block (kThreads) reduction of NV register values; thread k < NV writes
// part[(slot0 + k) * stride + col].  Fixed shuffle/LDS tree: deterministic.
// Sum of NW (a power of two) wavefront sums in a fixed pairwise order.
template <int NW>
__device__ __forceinline__ double pairwise_sum(const double* s) {
    if constexpr (NW == 1) return s[0];
    else return pairwise_sum<NW / 2>(s) + pairwise_sum<NW / 2>(s + NW / 2);
}

template <int NV, int NT = kThreads>
__device__ __forceinline__ void block_partials(const double (&v)[NV], double* __restrict__ part, int slot0,
                                               int stride, int col) {
    __shared__ double sh[NV > 0 ? NV : 1][NT / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) sh[k][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        part[size_t(slot0 + k) * stride + col] = pairwise_sum<NT / 64>(sh[k]);
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

}  // namespace fewha
