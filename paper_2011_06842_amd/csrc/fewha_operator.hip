// HIP kernels (gfx950 / CDNA4) of the system operator M = W^-T A^T C^-1 A W^-1 + alpha D
// (Sec. 3) and of the right-hand side b = W^-T A^T C^-1 s.
//
//   W^-1 (synthesis, Sec. 3):  k_idwt_coarse  one workgroup per layer; every level whose block
//                                             fits the coarse block, separable passes in LDS
//                              k_idwt_step    one launch per larger block size; 32x32 output tiles,
//                                             separable passes in LDS from a 36x36 coefficient halo
//   A^T C^-1 A (Sec. 2):       k_data_term    per (sensor, 14x14 node tile), one node of the
//                                             16x16 halo tile per thread: bilinear propagation from
//                                             every layer (NGS shift, LGS cone), Shack-Hartmann
//                                             slopes, noise weights, Shack-Hartmann adjoint; the
//                                             slopes never leave LDS
//                              k_adj_gather   per 8x32 layer tile (k_adj_gather_win: 32x32 for large
//                                             systems, sensor rectangles staged in LDS): exact
//                                             transpose of the bilinear propagation as a gather
//                                             (no atomics, deterministic)
//   W^-T + alpha D:            k_dwt_step / k_dwt_coarse, the mirror images of the synthesis,
//                                             with the prior and an optional (x, Mx) partial fused
//                                             into the final coefficients
#include <hip/hip_runtime.h>

#include <cmath>

#include "fewha_device.h"
#include "fewha_internal.h"

namespace fewha {

namespace {

__device__ __forceinline__ int ilog2i(int v) { return 31 - __clz(v); }

template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

// 16-byte vector of T and its element-wise store.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
    __device__ static void put(float* d, const float4& v) {
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
    }
    __device__ static void store(float* d, const float* v) { *reinterpret_cast<float4*>(d) = float4{v[0], v[1], v[2], v[3]}; }
};
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
    __device__ static void put(double* d, const double2& v) {
        d[0] = v.x;
        d[1] = v.y;
    }
    __device__ static void store(double* d, const double* v) { *reinterpret_cast<double2*>(d) = double2{v[0], v[1]}; }
};

// Workgroup index in an order that gives die x (workgroups x, x + kXcds, ...) a contiguous
// share of the tiles, so that the halos neighbouring tiles share are fetched into one L2.
__device__ __forceinline__ int die_ordered_block() {
    const int g = gridDim.x, b = blockIdx.x;
    return (g % kXcds) ? b : (b % kXcds) * (g / kXcds) + b / kXcds;
}

// Filter taps split by parity, so that every index is a compile-time constant (a tap index
// that varies across lanes would otherwise be fetched from memory inside the loops).
template <typename T>
struct Taps {
    T he[3], ho[3], ge[3], go[3], h[6], g[6];
    __device__ __forceinline__ explicit Taps(const Filt<T>& f) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            he[k] = f.h[2 * k];
            ho[k] = f.h[2 * k + 1];
            ge[k] = f.g[2 * k];
            go[k] = f.g[2 * k + 1];
        }
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            h[t] = f.h[t];
            g[t] = f.g[t];
        }
    }
};

// ------------------------------------------------------------------ wavelet synthesis

// Levels levels..coarse_lev of one layer in LDS.  Every coefficient of those levels lies in
// the top-left (n >> (coarse_lev-1))^2 block of the Mallat pyramid, so the block is loaded
// once; each level then synthesises its top-left block in place (its details are never
// overwritten by coarser levels).  1-D periodic synthesis of a 2m block:
// x_i = sum_{t = i mod 2} h_t a_{((i-t)/2) mod m} + g_t d_{((i-t)/2) mod m}, columns then rows.
template <typename T>
__global__ void __launch_bounds__(kCoarseThreads) k_idwt_coarse(const LayerDev* __restrict__ lays, Filt<T> f,
                                                                 const T* __restrict__ coef, T* __restrict__ ll_out,
                                                                 T* __restrict__ phi, const int32_t* __restrict__ skip) {
    constexpr int CB = CoarseBlock<T>::value;
    __shared__ T A[CB * CB];
    __shared__ T B[CB * CB];
    const LayerDev d = lays[blockIdx.x];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const int n = d.n, lc = d.coarse_lev, levels = d.levels;
    if (levels < lc) return;
    const T* C = coef + d.off;
    const Taps<T> tp(f);
    const int nb0 = n >> (lc - 1), lg0 = ilog2i(nb0);
    // 16-byte chunks of consecutive positions of a row (nb0 >= 8 is a multiple of the chunk)
    using VC = Vec16<T>;
    using V = typename VC::type;
    constexpr int PERC = CB * CB / (VC::n * kCoarseThreads);
    const int nch = nb0 * nb0 / VC::n;
    {
        V v[PERC];
#pragma unroll
        for (int k = 0; k < PERC; ++k) {   // unconditional (clamped) loads
            const int ch0 = threadIdx.x + k * kCoarseThreads, ch = ch0 < nch ? ch0 : 0;
            const int e = ch * VC::n;
            v[k] = *reinterpret_cast<const V*>(C + (e >> lg0) * n + (e & (nb0 - 1)));
        }
#pragma unroll
        for (int k = 0; k < PERC; ++k) {
            const int ch = threadIdx.x + k * kCoarseThreads;
            if (ch < nch) {
                const int e = ch * VC::n;
                VC::put(&A[(e >> lg0) * CB + (e & (nb0 - 1))], v[k]);
            }
        }
    }
    __syncthreads();
    // outputs 2i and 2i + 1 of a line read the same three coefficients of each band, so
    // every pass computes the pair from one read
    for (int lev = levels; lev >= lc; --lev) {
        const int nb = n >> (lev - 1), m = nb >> 1, lg = ilog2i(nb), lgm = lg - 1;
        for (int e = threadIdx.x; e < m * nb; e += kCoarseThreads) {   // rows 2i, 2i + 1
            const int i = e >> lg, x = e & (nb - 1);
            T ev = 0, od = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int ky = (i - k) & (m - 1);
                const T a = A[ky * CB + x], b = A[(m + ky) * CB + x];
                ev += tp.he[k] * a + tp.ge[k] * b;
                od += tp.ho[k] * a + tp.go[k] * b;
            }
            B[(2 * i) * CB + x] = ev;
            B[(2 * i + 1) * CB + x] = od;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nb * m; e += kCoarseThreads) {   // columns 2i, 2i + 1
            const int y = e >> lgm, i = e & (m - 1);
            T ev = 0, od = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int kx = (i - k) & (m - 1);
                const T a = B[y * CB + kx], b = B[y * CB + m + kx];
                ev += tp.he[k] * a + tp.ge[k] * b;
                od += tp.ho[k] * a + tp.go[k] * b;
            }
            A[y * CB + 2 * i] = ev;
            A[y * CB + 2 * i + 1] = od;
        }
        __syncthreads();
    }
    T* out = (lc == 1 ? phi : ll_out) + d.off;
    const T s = lc == 1 ? T(d.inv_delta) : T(1);
    for (int ch = threadIdx.x; ch < nch; ch += kCoarseThreads) {
        const int e = ch * VC::n, r = e >> lg0, c = e & (nb0 - 1);
        T val[VC::n];
#pragma unroll
        for (int j = 0; j < VC::n; ++j) val[j] = A[r * CB + c + j] * s;
        VC::store(out + r * n + c, val);
    }
}

// One synthesis level of block size nbs (> the coarse block) on the listed layers; ST x ST
// output tile per workgroup (the tile size changes no output bit: each output takes the same
// row and column passes).  The LL band comes from the previous step (or from the
// coefficients when this is the layer's coarsest level); the final level writes phi / delta.
template <typename T, int ST>
__global__ void __launch_bounds__(kThreads) k_idwt_step(const LayerDev* __restrict__ lays,
                                                         const int32_t* __restrict__ sl, int nbs,
                                                         Filt<T> f, const T* __restrict__ coef,
                                                         const T* __restrict__ ll_in, T* __restrict__ ll_out,
                                                         T* __restrict__ phi, const int32_t* __restrict__ skip) {
    constexpr int H = ST / 2 + 2;   // coefficient rows (per band) feeding one tile
    __shared__ T R[2 * H][2 * H + 1];
    __shared__ T I[ST][2 * H + 1];
    const int tx = nbs / ST, tiles = tx * tx;
    const int bid = die_ordered_block();
    const int li = bid / tiles, tile = bid - li * tiles;
    const LayerDev d = lays[sl[li]];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const int n = d.n;
    const int lev = ilog2i(n / nbs) + 1;
    const int M = nbs >> 1;
    const int y0 = (tile / tx) * ST, x0 = (tile % tx) * ST;
    const T* C = coef + d.off;
    const T* LL = (lev == d.levels ? coef : ll_in) + d.off;
    const int ky0 = (y0 >> 1) - 2, kx0 = (x0 >> 1) - 2;
    const Taps<T> tp(f);
    // staged in pairs: kx0 is even and M a multiple of 2, so the two coefficients of a pair
    // are adjacent (also across the periodic wrap) and the pair is 2-element aligned
    {
        using V2 = typename Vec2<T>::type;
        constexpr int NP = 2 * H * H, PER = (NP + kThreads - 1) / kThreads;   // pairs (H per row)
        V2 v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {   // unconditional loads (clamped index)
            const int e0 = threadIdx.x + k * kThreads, e = e0 < NP ? e0 : NP - 1;
            const int rr = e / H, cc = 2 * (e - rr * H);
            const int hr = rr >= H, hc = cc >= H;
            const int kr = (ky0 + rr - H * hr) & (M - 1), kc = (kx0 + cc - H * hc) & (M - 1);
            const T* src = (!hr && !hc) ? LL + kr * n + kc : C + (kr + M * hr) * n + kc + M * hc;
            v[k] = *reinterpret_cast<const V2*>(src);
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = threadIdx.x + k * kThreads;
            if (e < NP) {
                const int rr = e / H, cc = 2 * (e - rr * H);
                R[rr][cc] = v[k].x;
                R[rr][cc + 1] = v[k].y;
            }
        }
    }
    __syncthreads();
    // row pass: output rows 2m and 2m + 1 read the same three coefficient rows of each band
    for (int e = threadIdx.x; e < (ST / 2) * 2 * H; e += kThreads) {
        const int m = e / (2 * H), cc = e - m * (2 * H);
        T ev = 0, od = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T a = R[m - k + 2][cc], b = R[H + m - k + 2][cc];
            ev += tp.he[k] * a + tp.ge[k] * b;
            od += tp.ho[k] * a + tp.go[k] * b;
        }
        I[2 * m][cc] = ev;
        I[2 * m + 1][cc] = od;
    }
    __syncthreads();
    // column pass: the pair of outputs (2m, 2m + 1) of a row, stored together
    const T s = T(d.inv_delta);
    for (int e = threadIdx.x; e < ST * (ST / 2); e += kThreads) {
        const int yy = e / (ST / 2), m = e - yy * (ST / 2);
        T ev = 0, od = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T a = I[yy][m - k + 2], b = I[yy][H + m - k + 2];
            ev += tp.he[k] * a + tp.ge[k] * b;
            od += tp.ho[k] * a + tp.go[k] * b;
        }
        const size_t o = size_t(d.off) + size_t(y0 + yy) * n + x0 + 2 * m;   // even: 2-element aligned
        using V2 = typename Vec2<T>::type;
        if (lev == 1)
            *reinterpret_cast<V2*>(phi + o) = V2{ev * s, od * s};
        else
            *reinterpret_cast<V2*>(ll_out + o) = V2{ev, od};
    }
}

// ------------------------------------------------------------------ wavelet analysis

// One analysis level of block size nbs on the listed layers: 16x16 coefficients of every band
// per tile, rows then columns from a 36x36 halo, a_k = sum_t h_t x_{(2k+t) mod nbs}.  Final
// coefficients are scaled by 1/delta.  MODE 1 (inside M x): they get + (alpha D)_i x_i, and the
// partial of (x, out) over them goes to the tile's slot among the layer's partials (tiles of
// finer levels first).  MODE 2 (the right-hand side of a frame): the partial of (out, out)
// goes there instead (its sum tells the frame whether b is finite).  The prior and x operands
// are requested before the halo so that their latency overlaps it.
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) k_dwt_step(const LayerDev* __restrict__ lays,
                                                        const int32_t* __restrict__ sl, int nbs,
                                                        Filt<T> f, const T* __restrict__ img,
                                                        const T* __restrict__ ll_in, T* __restrict__ ll_out,
                                                        T* __restrict__ out, const T* __restrict__ prior_a,
                                                        const T* __restrict__ xprior, double* __restrict__ dotpart,
                                                        const int32_t* __restrict__ skip) {
    constexpr bool PRIOR = MODE == 1;
    constexpr int W = 2 * kAT + 4;
    __shared__ T R[W][W + 1];
    __shared__ T I[W][2 * kAT + 1];
    const int M = nbs >> 1, tx = M / kAT, tiles = tx * tx;
    const int bid = die_ordered_block();
    const int li = bid / tiles, tile = bid - li * tiles;
    const LayerDev d = lays[sl[li]];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const int n = d.n;
    const int lev = ilog2i(n / nbs) + 1;
    const int ky0 = (tile / tx) * kAT, kx0 = (tile % tx) * kAT;
    const int ky = threadIdx.x / kAT, kx = threadIdx.x % kAT;   // 256 threads = 16 x 16
    const int gy = ky0 + ky, gx = kx0 + kx;
    const bool fin_ll = lev == d.levels;
    const size_t base = size_t(d.off);
    const size_t o[4] = {base + size_t(gy) * n + M + gx, base + size_t(M + gy) * n + gx,
                         base + size_t(M + gy) * n + M + gx, base + size_t(gy) * n + gx};
    const int nout = fin_ll ? 4 : 3;
    T pa[4] = {0, 0, 0, 0}, xp[4] = {0, 0, 0, 0};
    if (PRIOR) {   // o[3] (the LL position) is a valid address even when it is not an output
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            pa[k] = prior_a[o[k]];
            xp[k] = xprior[o[k]];
        }
    }
    const T* src = (lev == 1 ? img : ll_in) + d.off;
    const Taps<T> tp(f);
    // staged in 16-byte chunks: 2 kx0 and nbs are multiples of the chunk, so a chunk is
    // contiguous (also across the periodic wrap) and aligned
    {
        using VC = Vec16<T>;
        constexpr int CPR = W / VC::n, NCH = W * CPR, PER = (NCH + kThreads - 1) / kThreads;
        typename VC::type v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {   // unconditional loads (clamped index)
            const int e0 = threadIdx.x + k * kThreads, e = e0 < NCH ? e0 : NCH - 1;
            const int r = e / CPR, q = e - r * CPR;
            v[k] = *reinterpret_cast<const typename VC::type*>(
                src + ((2 * ky0 + r) & (nbs - 1)) * n + ((2 * kx0 + q * VC::n) & (nbs - 1)));
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = threadIdx.x + k * kThreads;
            if (e < NCH) {
                const int r = e / CPR, q = e - r * CPR;
                VC::put(&R[r][q * VC::n], v[k]);
            }
        }
    }
    __syncthreads();
    // row pass: the low- and high-pass outputs of one (row, k) from the same six inputs
    for (int e = threadIdx.x; e < W * kAT; e += kThreads) {
        const int rr = e / kAT, k = e & (kAT - 1);
        T lo = 0, hi = 0;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const T x = R[rr][2 * k + t];
            lo += tp.h[t] * x;
            hi += tp.g[t] * x;
        }
        I[rr][k] = lo;
        I[rr][kAT + k] = hi;
    }
    __syncthreads();
    T ll = 0, yh = 0, xh = 0, hh = 0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const T lo = I[2 * ky + t][kx], hi = I[2 * ky + t][kAT + kx];
        ll += tp.h[t] * lo;
        yh += tp.g[t] * lo;
        xh += tp.h[t] * hi;
        hh += tp.g[t] * hi;
    }
    const T s = T(d.inv_delta);
    const T v[4] = {xh, yh, hh, ll};
    double dot = 0;
    for (int k = 0; k < nout; ++k) {
        T val = v[k] * s;
        if (PRIOR) val += pa[k] * xp[k];
        out[o[k]] = val;
        dot += double(val) * (MODE == 2 ? double(val) : double(xp[k]));   // (x, M x) or (b, b)
    }
    if (!fin_ll) ll_out[o[3]] = ll;
    if (MODE != 0 && dotpart) {
        int slot = d.pq0 + tile;
        for (int j = 1; j < lev; ++j) {
            const int mt = (n >> j) / kAT;
            slot += mt * mt;
        }
        const double vv[1] = {dot};
        block_partials<1>(vv, dotpart, 0, 0, slot);
    }
}

// Levels coarse_lev..levels of one layer in LDS (mirror of k_idwt_coarse).  After the last
// level the block holds the whole coarse Mallat pyramid; it is written once, each thread
// owning fixed positions whose prior and x operands it requested at kernel start.
template <typename T, int MODE>
__global__ void __launch_bounds__(kCoarseThreads) k_dwt_coarse(const LayerDev* __restrict__ lays, Filt<T> f,
                                                                const T* __restrict__ img, const T* __restrict__ ll_in,
                                                                T* __restrict__ out, const T* __restrict__ prior_a,
                                                                const T* __restrict__ xprior,
                                                                double* __restrict__ dotpart, const int32_t* __restrict__ skip) {
    constexpr bool PRIOR = MODE == 1;
    constexpr int CB = CoarseBlock<T>::value;
    __shared__ T A[CB * CB];
    __shared__ T B[CB * CB];
    const LayerDev d = lays[blockIdx.x];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const int n = d.n, lc = d.coarse_lev, levels = d.levels;
    double dot = 0;
    if (levels >= lc) {
        // 16-byte chunks of consecutive positions of a row (nb0 >= 8 is a multiple of the
        // chunk; layer offsets and rows keep chunks aligned)
        using VC = Vec16<T>;
        using V = typename VC::type;
        constexpr int PERC = CB * CB / (VC::n * kCoarseThreads);
        const int nb0 = n >> (lc - 1), lg0 = ilog2i(nb0), nch = nb0 * nb0 / VC::n;
        const T* src = (lc == 1 ? img : ll_in) + d.off;
        const Taps<T> tp(f);
        V pa[PERC], xp[PERC], v[PERC];
#pragma unroll
        for (int k = 0; k < PERC; ++k) {   // unconditional (clamped) loads
            const int ch0 = threadIdx.x + k * kCoarseThreads, ch = ch0 < nch ? ch0 : 0;
            const int e = ch * VC::n, r = e >> lg0, c = e & (nb0 - 1);
            v[k] = *reinterpret_cast<const V*>(src + r * n + c);
            pa[k] = xp[k] = V{};
            if (PRIOR) {
                pa[k] = *reinterpret_cast<const V*>(prior_a + size_t(d.off) + r * n + c);
                xp[k] = *reinterpret_cast<const V*>(xprior + size_t(d.off) + r * n + c);
            }
        }
#pragma unroll
        for (int k = 0; k < PERC; ++k) {
            const int ch = threadIdx.x + k * kCoarseThreads;
            if (ch < nch) {
                const int e = ch * VC::n;
                VC::put(&A[(e >> lg0) * CB + (e & (nb0 - 1))], v[k]);
            }
        }
        __syncthreads();
        for (int lev = lc; lev <= levels; ++lev) {
            const int nb = n >> (lev - 1), m = nb >> 1, lgm = ilog2i(m), lg = lgm + 1;
            for (int e = threadIdx.x; e < nb * m; e += kCoarseThreads) {   // rows: [a | d]
                const int y = e >> lgm, k = e & (m - 1);
                T lo = 0, hi = 0;
#pragma unroll
                for (int t = 0; t < 6; ++t) {
                    const T v = A[y * CB + ((2 * k + t) & (nb - 1))];
                    lo += tp.h[t] * v;
                    hi += tp.g[t] * v;
                }
                B[y * CB + k] = lo;
                B[y * CB + m + k] = hi;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < m * nb; e += kCoarseThreads) {   // columns
                const int k = e >> lg, x = e & (nb - 1);
                T lo = 0, hi = 0;
#pragma unroll
                for (int t = 0; t < 6; ++t) {
                    const T v = B[((2 * k + t) & (nb - 1)) * CB + x];
                    lo += tp.h[t] * v;
                    hi += tp.g[t] * v;
                }
                A[k * CB + x] = lo;
                A[(m + k) * CB + x] = hi;
            }
            __syncthreads();
        }
        const T s = T(d.inv_delta);
#pragma unroll
        for (int k = 0; k < PERC; ++k) {
            const int ch = threadIdx.x + k * kCoarseThreads;
            if (ch < nch) {
                const int e = ch * VC::n, r = e >> lg0, c = e & (nb0 - 1);
                T val[VC::n], a[VC::n], x[VC::n];
                VC::put(a, pa[k]);
                VC::put(x, xp[k]);
#pragma unroll
                for (int j = 0; j < VC::n; ++j) {
                    val[j] = A[r * CB + c + j] * s;
                    if (PRIOR) val[j] += a[j] * x[j];
                    dot += double(val[j]) * (MODE == 2 ? double(val[j]) : double(x[j]));
                }
                VC::store(out + size_t(d.off) + size_t(r) * n + c, val);
            }
        }
    }
    if (MODE != 0 && dotpart) {
        __shared__ double sh[kCoarseThreads / 64];
        const double w = wave_sum(dot);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0;
            for (int k = 0; k < kCoarseThreads / 64; ++k) t += sh[k];
            dotpart[d.pq0 + d.pq_coarse] = t;
        }
    }
}

// ------------------------------------------------------------------ tomography (Sec. 2)

// Sensor owning element e of a concatenation with per-sensor offsets (binary search).
template <typename Off>
__device__ __forceinline__ int find_sensor(const WfsDev* __restrict__ wfs, int G, int64_t e, Off off) {
    int lo = 0, hi = G - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off(wfs[mid]) <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Fused Gamma^T C^-1 Gamma P per sensor tile: wavefront on the tile plus a one-node halo,
// slopes on the (kTile+1)^2 subapertures touching it, adjoint onto the kTile^2 nodes.  The
// halo tile has exactly one node per thread; each thread sums every layer of the sensor's
// instance in order (propagation, Sec. 2) from the bilinear cell tables of the tile's rows and
// columns, staged in LDS; the per-layer scalars are the same for the whole workgroup.
template <typename T>
__global__ void __launch_bounds__(kDataThreads) k_data_term(const WfsDev* __restrict__ wfs,
                                                            const int2* __restrict__ tiles,
                                                            const LayerDev* __restrict__ lays,
                                                            const int32_t* __restrict__ cidx,
                                                            const T* __restrict__ frac, const T* __restrict__ phi,
                                                            const T* __restrict__ w, T* __restrict__ psi,
                                                            const int32_t* __restrict__ skip) {
    constexpr int E = kTile + 2, S1 = kTile + 1;
    static_assert(E * E == kDataThreads, "one halo-tile node per thread");
    static_assert(S1 * S1 <= kDataThreads, "one subaperture per thread");
    static_assert(2 * E == 32, "table entries indexed by shifts");
    __shared__ T sphi[E * E];
    __shared__ T stx[S1 * S1], sty[S1 * S1];
    __shared__ int32_t srow[FEWHA_MAX_LAYERS][E], scol[FEWHA_MAX_LAYERS][E];
    __shared__ T sfy[FEWHA_MAX_LAYERS][E], sfx[FEWHA_MAX_LAYERS][E];
    __shared__ int32_t sn[FEWHA_MAX_LAYERS];
    __shared__ uint32_t soffl[FEWHA_MAX_LAYERS];
    const int2 st = tiles[blockIdx.x];
    if (st.x < 0) return;                                        // padding of the die-ordered grid
    const WfsDev W = wfs[st.x];
    if (skip && skip[W.inst]) return;   // tolerance mode: the instance has converged
    const int ns = W.ns, np = ns + 1;
    const int L = W.nl;
    // the instance's layers follow its first one, at most FEWHA_MAX_LAYERS x 1024^2 values:
    // byte offsets from it fit in 32 bits
    const char* __restrict__ phib = reinterpret_cast<const char*>(phi + lays[W.l0].off);
    const int tl = st.y;
    const int i0 = (tl / W.tiles_x) * kTile, j0 = (tl % W.tiles_x) * kTile;
    // slope weights of this thread's subaperture, requested before anything waits
    const int ls = threadIdx.x / S1, lt = threadIdx.x - ls * S1;
    const int si = i0 - 1 + ls, sj = j0 - 1 + lt;
    const bool sub = threadIdx.x < S1 * S1 && si >= 0 && si < ns && sj >= 0 && sj < ns;
    T wx = 0, wy = 0;
    if (sub) {
        wx = w[W.soff + si * ns + sj];
        wy = w[W.soff + ns * ns + si * ns + sj];
    }
    // the bilinear cells of the tile's rows and columns on each layer: every load is issued
    // before the first LDS store
    constexpr int PER = (FEWHA_MAX_LAYERS * 2 * E + kDataThreads - 1) / kDataThreads;
    const int nent = L * 2 * E;
    int32_t ci[PER];
    T fr[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (k * kDataThreads >= nent) break;                     // uniform: only the L layers
        const int e = threadIdx.x + k * kDataThreads;
        if (e < nent) {
            const int l = e >> 5, q = e & 31, col = q >= E, kk = q - col * E;
            const int node = (col ? j0 : i0) - 1 + kk;
            const int nn = node < 0 ? 0 : (node > ns ? ns : node);   // clamped: halo nodes outside are unused
            const size_t o = size_t(W.fwd0) + size_t(l) * 2 * np + col * np + nn;
            ci[k] = cidx[o];
            fr[k] = frac[o];
        }
    }
    int32_t ln = 0;
    uint32_t loff = 0;
    if (threadIdx.x < L) {
        const LayerDev d = lays[W.l0 + threadIdx.x];
        ln = d.n;
        loff = uint32_t(d.off - lays[W.l0].off) * uint32_t(sizeof(T));
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (k * kDataThreads >= nent) break;
        const int e = threadIdx.x + k * kDataThreads;
        if (e < nent) {
            const int l = e >> 5, q = e & 31, col = q >= E, kk = q - col * E;
            if (col) {
                scol[l][kk] = ci[k];
                sfx[l][kk] = fr[k];
            } else {
                srow[l][kk] = ci[k];
                sfy[l][kk] = fr[k];
            }
        }
    }
    if (threadIdx.x < L) {
        sn[threadIdx.x] = ln;
        soffl[threadIdx.x] = loff;
    }
    __syncthreads();
    {   // this thread's node: the sum over the layers, in layer order
        const int li = threadIdx.x / E, lj = threadIdx.x - li * E;
        const int i = i0 - 1 + li, j = j0 - 1 + lj;
        // layers in chunks of LC whose loads are all issued before the first is used (layers
        // past L read the last one and are not added)
        constexpr int LC = 9;
        T v = 0;
        for (int lb = 0; lb < L; lb += LC) {
            T p[LC][4];
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                const int l = lb + k < L ? lb + k : L - 1;
                const uint32_t n = uint32_t(sn[l]);
                const uint32_t o0 = soffl[l] + (uint32_t(srow[l][li]) * n + uint32_t(scol[l][lj])) * uint32_t(sizeof(T));
                const uint32_t o1 = o0 + n * uint32_t(sizeof(T));
                p[k][0] = *reinterpret_cast<const T*>(phib + o0);
                p[k][1] = *reinterpret_cast<const T*>(phib + o0 + sizeof(T));
                p[k][2] = *reinterpret_cast<const T*>(phib + o1);
                p[k][3] = *reinterpret_cast<const T*>(phib + o1 + sizeof(T));
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                const int l = lb + k < L ? lb + k : L - 1;
                const T fy = sfy[l][li], fx = sfx[l][lj];
                const T r0 = fma(fx, p[k][1], (T(1) - fx) * p[k][0]);
                const T r1 = fma(fx, p[k][3], (T(1) - fx) * p[k][2]);
                const T vn = fma(fy, r1, fma(T(1) - fy, r0, v));
                v = lb + k < L ? vn : v;
            }
        }
        sphi[threadIdx.x] = (i >= 0 && i <= ns && j >= 0 && j <= ns) ? v : T(0);
    }
    __syncthreads();
    if (threadIdx.x < S1 * S1) {   // Shack-Hartmann slopes and noise weights of the subaperture
        T tx = 0, ty = 0;
        if (sub) {
            const T p00 = sphi[ls * E + lt], p01 = sphi[ls * E + lt + 1];
            const T p10 = sphi[(ls + 1) * E + lt], p11 = sphi[(ls + 1) * E + lt + 1];
            const T sx = T(0.5) * ((p01 - p00) + (p11 - p10));
            const T sy = T(0.5) * ((p10 - p00) + (p11 - p01));
            tx = wx * sx;
            ty = wy * sy;
        }
        stx[threadIdx.x] = tx;
        sty[threadIdx.x] = ty;
    }
    __syncthreads();
    if (threadIdx.x < kTile * kTile) {   // Shack-Hartmann adjoint onto the tile's nodes
        const int li = threadIdx.x / kTile, lj = threadIdx.x - li * kTile;
        const int i = i0 + li, j = j0 + lj;
        if (i <= ns && j <= ns) {
            const int A = (li + 1) * S1 + lj + 1, B = (li + 1) * S1 + lj, C = li * S1 + lj + 1, D = li * S1 + lj;
            psi[W.noff + i * np + j] = T(0.5) * ((stx[B] - stx[A]) + (stx[D] - stx[C])) +
                                       T(0.5) * ((sty[C] - sty[A]) + (sty[D] - sty[B]));
        }
    }
}

// Gamma^T (w s) per node (weighted = 1) or Gamma^T (mask s) (weighted = 0, mask = w != 0).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_slopes_adj(const WfsDev* __restrict__ wfs, int G, int64_t V,
                                                          const T* __restrict__ w, const T* __restrict__ s,
                                                          T* __restrict__ psi, int weighted) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= V) return;
    const WfsDev W = wfs[find_sensor(wfs, G, e, [](const WfsDev& w) { return w.noff; })];
    const int ns = W.ns, np = ns + 1;
    const int loc = int(e - W.noff);
    const int i = loc / np, j = loc % np;
    // unconditional loads (clamped index); slopes outside the sensor or of an inactive
    // subaperture (weight 0) are dropped by a select, so that even a non-finite value there is
    // ignored, as the operator ignores inactive subapertures
    auto t = [&](int comp, int si, int sj) -> T {
        const bool ok = si >= 0 && si < ns && sj >= 0 && sj < ns;
        const int64_t o = W.soff + int64_t(comp) * ns * ns + (ok ? si * ns + sj : 0);
        const T ww = w[o], sv = s[o];
        return ok && ww != T(0) ? (weighted ? ww * sv : sv) : T(0);
    };
    psi[e] = T(0.5) * ((t(0, i, j - 1) - t(0, i, j)) + (t(0, i - 1, j - 1) - t(0, i - 1, j))) +
             T(0.5) * ((t(1, i - 1, j) - t(1, i, j)) + (t(1, i - 1, j - 1) - t(1, i, j - 1)));
}

// Gamma P phi per subaperture (operator piece A), zero on inactive subapertures.
template <typename T>
__device__ __forceinline__ T wavefront_node(const WfsDev& W, int i, int j, const LayerDev* __restrict__ lays,
                                            const PairDev* __restrict__ pairs, const int32_t* __restrict__ cidx,
                                            const T* __restrict__ frac, const T* __restrict__ phi) {
    const int np = W.ns + 1;
    T v = 0;
    for (int l = 0; l < W.nl; ++l) {
        const PairDev P = pairs[W.pair0 + l];
        const LayerDev d = lays[W.l0 + l];
        const int n = d.n;
        const int a0 = cidx[P.fwd_off + i], b0 = cidx[P.fwd_off + np + j];
        const T fy = frac[P.fwd_off + i], fx = frac[P.fwd_off + np + j];
        const T* ph = phi + d.off + size_t(a0) * n + b0;
        v += (T(1) - fy) * ((T(1) - fx) * ph[0] + fx * ph[1]) + fy * ((T(1) - fx) * ph[n] + fx * ph[n + 1]);
    }
    return v;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_fwd_slopes(const WfsDev* __restrict__ wfs, int G, int64_t S,
                                                          const LayerDev* __restrict__ lays,
                                                          const PairDev* __restrict__ pairs,
                                                          const int32_t* __restrict__ cidx, const T* __restrict__ frac,
                                                          const T* __restrict__ phi, const T* __restrict__ w,
                                                          T* __restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= S) return;
    const WfsDev W = wfs[find_sensor(wfs, G, e, [](const WfsDev& w) { return w.soff; })];
    const int ns = W.ns;
    const int loc = int(e - W.soff);
    const int comp = loc / (ns * ns), q = loc % (ns * ns), i = q / ns, j = q % ns;
    const T p00 = wavefront_node(W, i, j, lays, pairs, cidx, frac, phi);
    const T p01 = wavefront_node(W, i, j + 1, lays, pairs, cidx, frac, phi);
    const T p10 = wavefront_node(W, i + 1, j, lays, pairs, cidx, frac, phi);
    const T p11 = wavefront_node(W, i + 1, j + 1, lays, pairs, cidx, frac, phi);
    const T v = comp == 0 ? T(0.5) * ((p01 - p00) + (p11 - p10)) : T(0.5) * ((p10 - p00) + (p11 - p01));
    out[e] = w[e] != T(0) ? v : T(0);
}

// sum_g P_g^T psi_g on a layer tile of TR = 8 NRW rows x kGT columns.  Along each axis the
// transpose of the bilinear propagation sends layer row (column) a the sensor rows (columns)
// of its precomputed record, so a layer node sums w_row(i) w_col(j) psi_g(i, j) over at most
// RF x RF sensor nodes per sensor.  The records of the tile's rows and columns are staged in
// LDS (kGatherGroup sensors at a time, all loads issued before the first store); every thread
// then owns NRW nodes of one column and reads their sensor nodes directly (L1/L2), sensors
// summed in order.
template <typename T, int RF, int NRW>
__global__ void __launch_bounds__(kThreads) k_adj_gather(const WfsDev* __restrict__ wfs,
                                                          const LayerDev* __restrict__ lays,
                                                          const int2* __restrict__ tiles,
                                                          const int64_t* __restrict__ recbase,
                                                          const GatherRec<T>* __restrict__ recs,
                                                          const T* __restrict__ psi, T* __restrict__ out,
                                                          const int32_t* __restrict__ skip) {
    constexpr int TR = kGRowStep * NRW;
    constexpr int NR = TR + kGT;                         // records per sensor: tile rows, then columns
    constexpr int PER = (kGatherGroup * NR + kThreads - 1) / kThreads;
    __shared__ int32_t s_start[kGatherGroup][NR], s_cnt[kGatherGroup][NR];
    __shared__ T s_w[kGatherGroup][NR][RF];
    const int2 lt = tiles[blockIdx.x];
    if (lt.x < 0) return;                                // padding of the die-ordered grid
    const LayerDev d = lays[lt.x];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const int n = d.n, tx = (n + kGT - 1) / kGT;
    const int a0 = (lt.y / tx) * TR, b0 = (lt.y % tx) * kGT;
    const int la = threadIdx.x / kGT, lb = threadIdx.x % kGT;
    const int b = b0 + lb;
    const int G = d.ng;
    const WfsDev* __restrict__ wf = wfs + d.g0;
    const int64_t* __restrict__ rb = recbase + d.rb0;
    T acc[NRW];
#pragma unroll
    for (int k = 0; k < NRW; ++k) acc[k] = 0;
    for (int g0 = 0; g0 < G; g0 += kGatherGroup) {
        const int ng = G - g0 < kGatherGroup ? G - g0 : kGatherGroup;
        {   // records of (sensor g0 + gl, tile row / column e)
            GatherRec<T> r[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int f = threadIdx.x + k * kThreads, gl = f / NR, e = f - gl * NR;
                const int node = e < TR ? a0 + e : b0 + e - TR;
                r[k].count = 0;
                if (gl < ng && node < n) r[k] = recs[rb[g0 + gl] + (e < TR ? 0 : n) + node];
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int f = threadIdx.x + k * kThreads, gl = f / NR, e = f - gl * NR;
                if (gl < ng) {
                    s_start[gl][e] = r[k].count > 0 ? r[k].start : 0;
                    s_cnt[gl][e] = r[k].count;
#pragma unroll
                    for (int t = 0; t < RF; ++t) s_w[gl][e][t] = r[k].w[t] * T(t < r[k].count);
                }
            }
        }
        __syncthreads();
        if (b < n) {
            constexpr int GU = RF * RF * NRW <= 16 ? 2 : 1;      // sensors whose loads are in flight together
#pragma unroll GU
            for (int gl = 0; gl < ng; ++gl) {
                const int np = wf[g0 + gl].ns + 1;
                const T* __restrict__ ps = psi + wf[g0 + gl].noff;
                const int jc = s_start[gl][TR + lb], cc = s_cnt[gl][TR + lb];
                T wc[RF];
#pragma unroll
                for (int q = 0; q < RF; ++q) wc[q] = s_w[gl][TR + lb][q];
                T v[NRW][RF][RF];
#pragma unroll
                for (int k = 0; k < NRW; ++k) {
                    const int e = la + k * kGRowStep;
                    const int ir = s_start[gl][e], cr = s_cnt[gl][e];
#pragma unroll
                    for (int r = 0; r < RF; ++r)
#pragma unroll
                        for (int q = 0; q < RF; ++q) {
                            const bool ok = r < cr && q < cc;    // masked entries read node 0 (weight 0)
                            v[k][r][q] = ps[ok ? (ir + r) * np + jc + q : 0];
                        }
                }
#pragma unroll
                for (int k = 0; k < NRW; ++k) {
                    const int e = la + k * kGRowStep;
                    T sum = 0;
#pragma unroll
                    for (int r = 0; r < RF; ++r) {
                        T row = 0;
#pragma unroll
                        for (int q = 0; q < RF; ++q) row += wc[q] * v[k][r][q];
                        sum += s_w[gl][e][r] * row;
                    }
                    acc[k] += sum;
                }
            }
        }
        __syncthreads();
    }
    if (b < n) {
#pragma unroll
        for (int k = 0; k < NRW; ++k) {
            const int a = a0 + la + k * kGRowStep;
            if (a < n) out[d.off + size_t(a) * n + b] = acc[k];
        }
    }
}

// The same sum with the sensor nodes staged in LDS: per (tile, sensor) the setup stores the
// rectangle of sensor nodes the tile's records reach (gwin, extended by RF - 1 rows and
// columns so that every RF x RF window of a record lies inside it; at most 32 x 32).  The
// workgroup loads it with coalesced reads (thread t: column t mod 32, rows t / 32 + 8 k,
// clamped to the sensor grid) into a 32 x 32 LDS image, then every layer node reads its
// RF x RF window at fixed offsets from one base (the weights of entries past a record's
// count are zero; a record the sensor does not see points at the rectangle's origin).  The
// next sensor's rectangle and records are fetched into registers while the current one is
// summed.  Used for large systems, where the per-node reads of k_adj_gather are bound by
// instruction issue.
template <typename T, int RF, int NRW>
__global__ void __launch_bounds__(kThreads) k_adj_gather_win(const WfsDev* __restrict__ wfs,
                                                              const LayerDev* __restrict__ lays,
                                                              const int2* __restrict__ tiles,
                                                              const int64_t* __restrict__ recbase,
                                                              const GatherRec<T>* __restrict__ recs,
                                                              const int4* __restrict__ gwin,
                                                              const T* __restrict__ psi, T* __restrict__ out,
                                                              const int32_t* __restrict__ skip) {
    constexpr int TR = kGRowStep * NRW;
    constexpr int NR = TR + kGT;                         // records per sensor: tile rows, then columns
    constexpr int WP = 32;                               // LDS image pitch (and largest side)
    constexpr int PERW = WP * WP / kThreads;             // image rows per thread (4)
    static_assert(NR <= kThreads, "one record per thread");
    __shared__ int32_t s_base[NR];                       // rows: (start - r0) WP; columns: start - c0
    __shared__ T s_w[NR][RF];
    __shared__ T win[WP * WP];
    const int2 lt = tiles[blockIdx.x];
    if (lt.x < 0) return;                                // padding of the die-ordered grid
    const LayerDev d = lays[lt.x];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const int n = d.n, tx = (n + kGT - 1) / kGT;
    const int a0 = (lt.y / tx) * TR, b0 = (lt.y % tx) * kGT;
    const int la = threadIdx.x / kGT, lb = threadIdx.x % kGT;
    const int b = b0 + lb;
    const int G = d.ng;
    const WfsDev* __restrict__ wf = wfs + d.g0;
    const int64_t* __restrict__ rb = recbase + d.rb0;
    const int4* __restrict__ wt = gwin + d.wb0 + int64_t(lt.y) * G;
    // the thread's record (clamped to a valid one; only threads < NR stage theirs)
    const int re = threadIdx.x < NR ? threadIdx.x : NR - 1;
    const int rnode = re < TR ? a0 + re : b0 + re - TR;
    const bool rvalid = rnode < n;
    const int64_t roff = (re < TR ? 0 : n) + (rvalid ? rnode : 0);
    const int icol = threadIdx.x % WP, irow = threadIdx.x / WP;
    GatherRec<T> rr;
    T wv[PERW];
    int4 wn;
    auto fetch = [&](int gl) {
        wn = wt[gl];
        const int np = wf[gl].ns + 1;
        const T* __restrict__ ps = psi + wf[gl].noff;
        const int cc = min(wn.z + icol, np - 1);
#pragma unroll
        for (int k = 0; k < PERW; ++k) wv[k] = ps[uint32_t(min(wn.x + irow + k * (kThreads / WP), np - 1) * np + cc)];
        rr = recs[rb[gl] + roff];
    };
    T acc[NRW];
#pragma unroll
    for (int k = 0; k < NRW; ++k) acc[k] = 0;
    fetch(0);
    for (int gl = 0; gl < G; ++gl) {
#pragma unroll
        for (int k = 0; k < PERW; ++k) win[threadIdx.x + k * kThreads] = wv[k];
        if (threadIdx.x < NR) {
            const int cnt = rvalid ? rr.count : 0;
            const int st = cnt > 0 ? rr.start : (re < TR ? wn.x : wn.z);
            s_base[threadIdx.x] = re < TR ? (st - wn.x) * WP : st - wn.z;
#pragma unroll
            for (int q = 0; q < RF; ++q) s_w[threadIdx.x][q] = rr.w[q] * T(q < cnt);
        }
        __syncthreads();
        fetch(gl + 1 < G ? gl + 1 : gl);                  // in flight during the sums below
        if (b < n) {
            const int cb = s_base[TR + lb];
            T wc[RF];
#pragma unroll
            for (int q = 0; q < RF; ++q) wc[q] = s_w[TR + lb][q];
#pragma unroll
            for (int k = 0; k < NRW; ++k) {
                const int e = la + k * kGRowStep;
                const T* __restrict__ wp = win + s_base[e] + cb;
                T sum = 0;
#pragma unroll
                for (int r = 0; r < RF; ++r) {
                    T row = 0;
#pragma unroll
                    for (int q = 0; q < RF; ++q) row += wc[q] * wp[r * WP + q];
                    sum += s_w[e][r] * row;
                }
                acc[k] += sum;
            }
        }
        __syncthreads();
    }
    if (b < n) {
#pragma unroll
        for (int k = 0; k < NRW; ++k) {
            const int a = a0 + la + k * kGRowStep;
            if (a < n) out[d.off + size_t(a) * n + b] = acc[k];
        }
    }
}

// The same sum for configurations whose contribution lists exceed kRMax (layer grids much
// coarser than the sensor grids): every node walks its ranges and the bilinear cells.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_adj_gather_wide(const WfsDev* __restrict__ wfs,
                                                               const LayerDev* __restrict__ lays,
                                                               const PairDev* __restrict__ pairs,
                                                               const int32_t* __restrict__ cidx,
                                                               const T* __restrict__ frac,
                                                               const int2* __restrict__ rng,
                                                               const T* __restrict__ psi, T* __restrict__ out,
                                                               const int32_t* __restrict__ skip) {
    const int l = blockIdx.y;
    const LayerDev d = lays[l];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const int n = d.n;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int a = idx / n, b = idx - a * n;
    T acc = 0;
    for (int g = d.g0; g < d.g0 + d.ng; ++g) {
        const WfsDev W = wfs[g];
        const int np = W.ns + 1;
        const PairDev P = pairs[W.pair0 + (l - d.l0)];
        const int2 ra = rng[P.rng_off + a], rb = rng[P.rng_off + n + b];
        for (int ii = 0; ii < ra.y; ++ii) {
            const int i = ra.x + ii;
            const T fy = frac[P.fwd_off + i];
            const T wy = cidx[P.fwd_off + i] == a ? T(1) - fy : fy;
            T row = 0;
            for (int jj = 0; jj < rb.y; ++jj) {
                const int j = rb.x + jj;
                const T fx = frac[P.fwd_off + np + j];
                const T wx = cidx[P.fwd_off + np + j] == b ? T(1) - fx : fx;
                row += wx * psi[W.noff + i * np + j];
            }
            acc += wy * row;
        }
    }
    out[d.off + idx] = acc;
}

template <typename T>
Filt<T> make_filt() {
    // Daubechies' closed form of the orthonormal 6-tap scaling filter; g_m = (-1)^m h_{5-m}
    const double s10 = std::sqrt(10.0), r = std::sqrt(5.0 + 2.0 * s10), k = std::sqrt(2.0) / 32.0;
    const double v[6] = {1 + s10 + r, 5 + s10 + 3 * r, 10 - 2 * s10 + 2 * r,
                         10 - 2 * s10 - 2 * r, 5 + s10 - 3 * r, 1 + s10 - r};
    Filt<T> f;
    for (int m = 0; m < 6; ++m) f.h[m] = T(k * v[m]);
    for (int m = 0; m < 6; ++m) f.g[m] = T(((m & 1) ? -1.0 : 1.0) * k * v[5 - m]);
    return f;
}

inline unsigned cdiv(int64_t a, int64_t b) { return unsigned((a + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------------ profiler

const char* const kKernelNames[KID_COUNT] = {
    "idwt_coarse", "idwt_step", "data_term", "adj_gather", "dwt_step", "dwt_coarse", "slopes_adj", "residual",
    "gram", "gram_solve", "galerkin_apply", "init_dir", "update1", "update2", "finish", "fwd_slopes"};

ProfScope::ProfScope(const Ctx& ctx, int kid, hipStream_t stream) : c(ctx), s(stream) {
    Profiler& p = c.prof;
    if (!p.on) return;
    const size_t j = p.pending.size();
    while (p.pool.size() < 2 * (j + 1)) {
        hipEvent_t e;
        (void)hipEventCreate(&e);
        p.pool.push_back(e);
    }
    p.pending.push_back(kid);
    (void)hipEventRecord(p.pool[2 * j], s);
}

ProfScope::~ProfScope() {
    Profiler& p = c.prof;
    if (!p.on) return;
    (void)hipEventRecord(p.pool[2 * (p.pending.size() - 1) + 1], s);
}

hipError_t profiler_collect(const Ctx& c, hipStream_t s) {
    Profiler& p = c.prof;
    if (p.pending.empty()) return hipSuccess;
    hipError_t e = hipStreamSynchronize(s);
    for (size_t j = 0; j < p.pending.size() && e == hipSuccess; ++j) {
        float ms = 0;
        e = hipEventElapsedTime(&ms, p.pool[2 * j], p.pool[2 * j + 1]);
        p.ms[p.pending[j]] += ms;
        p.launches[p.pending[j]] += 1;
    }
    p.pending.clear();
    return e;
}

// ------------------------------------------------------------------ operator launchers

// A synthesis step with kST x kST tiles, or with tiles of half that side when the large tiles
// would give fewer workgroups than the GPU has compute units (a single small instance): the
// step is then bound by the latency of each workgroup, and four times as many smaller tiles
// finish sooner.
template <typename T>
void launch_idwt_step(const StepInfo& w, const LayerDev* lays, const int32_t* sl, const Filt<T>& f, const T* x,
                      const T* ll_in, T* ll_out, T* phi, hipStream_t s, const int32_t* skip) {
    const int tiles = (w.nb / kST) * (w.nb / kST) * w.nl;
    if (tiles < kSmallTileBelow)
        k_idwt_step<T, kST / 2><<<4 * tiles, kThreads, 0, s>>>(lays, sl + w.loff, w.nb, f, x, ll_in, ll_out, phi, skip);
    else
        k_idwt_step<T, kST><<<tiles, kThreads, 0, s>>>(lays, sl + w.loff, w.nb, f, x, ll_in, ll_out, phi, skip);
}

template <typename T>
void launch_winv(const Ctx& c, const T* x, T* phi, hipStream_t s, const OpBufs* ob, const int32_t* skip) {
    const Filt<T> f = make_filt<T>();
    const OpBufs bb = ob ? *ob : ctx_bufs(c);
    T* buf[2] = {reinterpret_cast<T*>(bb.tmp0), reinterpret_cast<T*>(bb.tmp1)};
    const LayerDev* lays = c.at<LayerDev>(c.lay.layers);
    const int32_t* sl = c.at<int32_t>(c.lay.step_layers);
    {
        ProfScope ps_(c, KID_IDWT_COARSE, s);
        k_idwt_coarse<T><<<c.L, kCoarseThreads, 0, s>>>(lays, f, x, buf[0], phi, skip);
    }
    for (size_t j = 0; j < c.steps.size(); ++j) {
        ProfScope ps_(c, KID_IDWT_STEP, s);
        launch_idwt_step<T>(c.steps[j], lays, sl, f, x, buf[j & 1], buf[(j + 1) & 1], phi, s, skip);
    }
}

template <typename T>
void launch_winvt(const Ctx& c, const T* img, T* y, const T* xprior, double* pq_part, hipStream_t s,
                  const OpBufs* ob, const int32_t* skip) {
    const Filt<T> f = make_filt<T>();
    const OpBufs bb = ob ? *ob : ctx_bufs(c);
    T* buf[2] = {reinterpret_cast<T*>(bb.tmp0), reinterpret_cast<T*>(bb.tmp1)};
    const LayerDev* lays = c.at<LayerDev>(c.lay.layers);
    const int32_t* sl = c.at<int32_t>(c.lay.step_layers);
    const T* pa = c.at<T>(c.lay.prior_a);
    const int J = int(c.steps.size());
    // with xprior: + alpha D x and the (x, y) partials; without it but with pq_part: (y, y)
    const int mode = xprior ? 1 : (pq_part ? 2 : 0);
    for (int j = 0; j < J; ++j) {                 // largest block first
        const StepInfo& w = c.steps[J - 1 - j];
        const int tiles = (w.nb / 2 / kAT) * (w.nb / 2 / kAT);
        ProfScope ps_(c, KID_DWT_STEP, s);
        auto go = [&](auto kern) {
            kern<<<tiles * w.nl, kThreads, 0, s>>>(lays, sl + w.loff, w.nb, f, img, buf[(j + 1) & 1], buf[j & 1], y, pa,
                                                   xprior, pq_part, skip);
        };
        if (mode == 1) go(k_dwt_step<T, 1>);
        else if (mode == 2) go(k_dwt_step<T, 2>);
        else go(k_dwt_step<T, 0>);
    }
    ProfScope ps_(c, KID_DWT_COARSE, s);
    auto go = [&](auto kern) {
        kern<<<c.L, kCoarseThreads, 0, s>>>(lays, f, img, buf[(J - 1) & 1], y, pa, xprior, pq_part, skip);
    };
    if (mode == 1) go(k_dwt_coarse<T, 1>);
    else if (mode == 2) go(k_dwt_coarse<T, 2>);
    else go(k_dwt_coarse<T, 0>);
}

template <typename T>
void launch_data_term(const Ctx& c, const T* phi, T* psi_nodes, hipStream_t s, const int32_t* skip) {
    ProfScope ps_(c, KID_DATA_TERM, s);
    k_data_term<T><<<c.data_grid, kDataThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.at<int2>(c.lay.data_tiles),
                                                        c.at<LayerDev>(c.lay.layers), c.at<int32_t>(c.lay.cellidx),
                                                        c.at<T>(c.lay.frac), phi, c.at<T>(c.lay.weight), psi_nodes,
                                                        skip);
}

template <typename T>
void launch_slopes_adj(const Ctx& c, const T* slopes, T* psi_nodes, int weighted, hipStream_t s) {
    ProfScope ps_(c, KID_SLOPES_ADJ, s);
    k_slopes_adj<T><<<cdiv(c.V, kThreads), kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.G, c.V, c.at<T>(c.lay.weight),
                                                             slopes, psi_nodes, weighted);
}

template <typename T>
void launch_adj_gather(const Ctx& c, const T* psi_nodes, T* psi_layers, hipStream_t s, const int32_t* skip) {
    ProfScope ps_(c, KID_ADJ_GATHER, s);
    if (c.max_rng <= kRMax) {
        auto go = [&](auto kern) {
            kern<<<c.gather_grid, kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.at<LayerDev>(c.lay.layers),
                                                   c.at<int2>(c.lay.gather_tiles), c.at<int64_t>(c.lay.recbase),
                                                   c.at<GatherRec<T>>(c.lay.grecs), psi_nodes, psi_layers, skip);
        };
        const bool wide = c.gather_rows > 1;
        auto gow = [&](auto kern) {
            kern<<<c.gather_grid, kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.at<LayerDev>(c.lay.layers),
                                                   c.at<int2>(c.lay.gather_tiles), c.at<int64_t>(c.lay.recbase),
                                                   c.at<GatherRec<T>>(c.lay.grecs), c.at<int4>(c.lay.gwin),
                                                   psi_nodes, psi_layers, skip);
        };
        // large systems with windows that fit: LDS-staged sensor nodes
        // (rectangles, extended by RF - 1, of at most 32 x 32 sensor nodes)
        if (wide && c.max_rng <= 2 && c.max_gwin_side + 1 <= 32) {
            gow(k_adj_gather_win<T, 2, 4>);
        } else if (wide && c.max_rng <= 3 && c.max_gwin_side + 2 <= 32) {
            gow(k_adj_gather_win<T, 3, 4>);
        } else if (c.max_rng <= 2)
            wide ? go(k_adj_gather<T, 2, 4>) : go(k_adj_gather<T, 2, 1>);
        else if (c.max_rng <= 3)
            wide ? go(k_adj_gather<T, 3, 4>) : go(k_adj_gather<T, 3, 1>);
        else
            wide ? go(k_adj_gather<T, kRMax, 4>) : go(k_adj_gather<T, kRMax, 1>);
    } else {
        const dim3 grid(cdiv(int64_t(c.max_n) * c.max_n, kThreads), c.L);
        k_adj_gather_wide<T><<<grid, kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.at<LayerDev>(c.lay.layers),
                                                       c.at<PairDev>(c.lay.pairs), c.at<int32_t>(c.lay.cellidx),
                                                       c.at<T>(c.lay.frac), c.at<int2>(c.lay.ranges), psi_nodes,
                                                       psi_layers, skip);
    }
}

template <typename T>
void launch_fwd_slopes(const Ctx& c, const T* phi, T* slopes, hipStream_t s) {
    ProfScope ps_(c, KID_FWD_SLOPES, s);
    k_fwd_slopes<T><<<cdiv(c.S, kThreads), kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.G, c.S,
                                                             c.at<LayerDev>(c.lay.layers), c.at<PairDev>(c.lay.pairs),
                                                             c.at<int32_t>(c.lay.cellidx), c.at<T>(c.lay.frac), phi,
                                                             c.at<T>(c.lay.weight), slopes);
}

template <typename T>
void launch_apply_M(const Ctx& c, const T* x, T* y, double* pq_part, hipStream_t s, const OpBufs* ob,
                    const int32_t* skip) {
    const OpBufs bb = ob ? *ob : ctx_bufs(c);
    T* phi = reinterpret_cast<T*>(bb.nodal);
    T* psi_n = reinterpret_cast<T*>(bb.psi_nodes);
    T* psi_l = reinterpret_cast<T*>(bb.psi_layers);
    launch_winv<T>(c, x, phi, s, &bb, skip);
    launch_data_term<T>(c, phi, psi_n, s, skip);
    launch_adj_gather<T>(c, psi_n, psi_l, s, skip);
    launch_winvt<T>(c, psi_l, y, x, pq_part, s, &bb, skip);
}

// slopes NULL: the weighted slope adjoint is already in the sensor-node buffer (the graphed
// frame launches it outside the graph, on the caller's slopes).  bb_part (may be NULL): the
// analysis tiles' partials of (b, b), in the slots of the (p, q) partials.
template <typename T>
void launch_rhs(const Ctx& c, const T* slopes, T* b, hipStream_t s, double* bb_part) {
    T* psi_n = c.at<T>(c.lay.psi_nodes);
    T* psi_l = c.at<T>(c.lay.psi_layers);
    if (slopes) launch_slopes_adj<T>(c, slopes, psi_n, 1, s);
    launch_adj_gather<T>(c, psi_n, psi_l, s);
    launch_winvt<T>(c, psi_l, b, static_cast<const T*>(nullptr), bb_part, s);
}

// Launches one operator kernel with the arguments it has inside M x (input: the coefficient
// vector c; intermediates: the context buffers).  step selects the tiled wavelet level.
template <typename T>
static hipError_t launch_one(const Ctx& c, int kid, int step, hipStream_t s) {
    const Filt<T> f = make_filt<T>();
    const LayerDev* lays = c.at<LayerDev>(c.lay.layers);
    const int32_t* sl = c.at<int32_t>(c.lay.step_layers);
    T* buf[2] = {c.at<T>(c.lay.tmp0), c.at<T>(c.lay.tmp1)};
    const T* x = c.at<T>(c.lay.c);
    T* y = c.at<T>(c.lay.vy);
    const int J = int(c.steps.size());
    switch (kid) {
        case KID_IDWT_COARSE:
            k_idwt_coarse<T><<<c.L, kCoarseThreads, 0, s>>>(lays, f, x, buf[0], c.at<T>(c.lay.nodal), nullptr);
            break;
        case KID_IDWT_STEP: {
            if (step < 0 || step >= J) return hipErrorInvalidValue;
            launch_idwt_step<T>(c.steps[step], lays, sl, f, x, buf[step & 1], buf[(step + 1) & 1],
                                c.at<T>(c.lay.nodal), s, nullptr);
            break;
        }
        case KID_DATA_TERM:
            launch_data_term<T>(c, c.at<T>(c.lay.nodal), c.at<T>(c.lay.psi_nodes), s);
            break;
        case KID_ADJ_GATHER:
            launch_adj_gather<T>(c, c.at<T>(c.lay.psi_nodes), c.at<T>(c.lay.psi_layers), s);
            break;
        case KID_DWT_STEP: {
            if (step < 0 || step >= J) return hipErrorInvalidValue;
            const StepInfo& w = c.steps[step];
            const int j = J - 1 - step;
            k_dwt_step<T, 1><<<(w.nb / 2 / kAT) * (w.nb / 2 / kAT) * w.nl, kThreads, 0, s>>>(
                lays, sl + w.loff, w.nb, f, c.at<T>(c.lay.psi_layers), buf[(j + 1) & 1], buf[j & 1], y,
                c.at<T>(c.lay.prior_a), x, c.at<double>(c.lay.pq_part), nullptr);
            break;
        }
        case KID_DWT_COARSE:
            k_dwt_coarse<T, 1><<<c.L, kCoarseThreads, 0, s>>>(lays, f, c.at<T>(c.lay.psi_layers), buf[(J - 1) & 1],
                                                                 y, c.at<T>(c.lay.prior_a), x,
                                                                 c.at<double>(c.lay.pq_part), nullptr);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Average duration of one operator kernel: `reps` launches captured into one graph, replayed
// between two events on stream s (the graph keeps the gaps between launches small).
template <typename T>
hipError_t time_operator_kernel(Ctx& c, int kid, int step, int reps, hipStream_t s, float* ms) {
    if (reps < 1 || !ms) return hipErrorInvalidValue;
    const bool prof_on = c.prof.on;     // no profiler events inside the captured graph
    c.prof.on = false;
    hipStream_t cs = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        for (int r = 0; r < reps && le == hipSuccess; ++r) le = launch_one<T>(c, kid, step, cs);
        e = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipGraphLaunch(ge, s);            // warm-up replay
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = hipGraphLaunch(ge, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess) *ms = t / reps;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    if (cs) (void)hipStreamDestroy(cs);
    c.prof.on = prof_on;
    return e;
}

#define FEWHA_INSTANTIATE_OP(T)                                                                           \
    template void launch_winv<T>(const Ctx&, const T*, T*, hipStream_t, const OpBufs*, const int32_t*);   \
    template void launch_winvt<T>(const Ctx&, const T*, T*, const T*, double*, hipStream_t, const OpBufs*, \
                                  const int32_t*);                                                        \
    template void launch_data_term<T>(const Ctx&, const T*, T*, hipStream_t, const int32_t*);             \
    template void launch_slopes_adj<T>(const Ctx&, const T*, T*, int, hipStream_t);                       \
    template void launch_adj_gather<T>(const Ctx&, const T*, T*, hipStream_t, const int32_t*);            \
    template void launch_fwd_slopes<T>(const Ctx&, const T*, T*, hipStream_t);                            \
    template void launch_apply_M<T>(const Ctx&, const T*, T*, double*, hipStream_t, const OpBufs*,        \
                                    const int32_t*);                                                      \
    template void launch_rhs<T>(const Ctx&, const T*, T*, hipStream_t, double*);                                   \
    template hipError_t time_operator_kernel<T>(Ctx&, int, int, int, hipStream_t, float*);

FEWHA_INSTANTIATE_OP(float)
FEWHA_INSTANTIATE_OP(double)

}  // namespace fewha
