// HIP kernels (gfx950 / CDNA4) of the system operator M = W^-T A^T C^-1 A W^-1 + alpha D
// (Sec. 3) and of the right-hand side b = W^-T A^T C^-1 s.
//
//   W^-1 (synthesis, Sec. 3):  k_idwt         one launch: per 32x32 (or 16x16) image tile, the
//                                             windows of every level the tile depends on, loaded
//                                             at once and synthesised coarsest first in LDS
//   A^T C^-1 A (Sec. 2):       k_data_term    per (sensor, 14x14 node tile), one node of the
//                                             16x16 halo tile per thread: bilinear propagation from
//                                             every layer (NGS shift, LGS cone), Shack-Hartmann
//                                             slopes, noise weights, Shack-Hartmann adjoint; the
//                                             slopes never leave LDS
//                              k_adj_gather   per 8x32 layer tile (k_adj_gather_win: 32x32 for large
//                                             systems, sensor rectangles staged in LDS): exact
//                                             transpose of the bilinear propagation as a gather
//                                             (no atomics, deterministic)
//   W^-T + alpha D:            k_dwt_tiles    up to three levels per launch and tile from one input
//                                             window, then k_dwt_coarse (the levels whose block
//                                             fits 32x32, one workgroup per layer); the prior and
//                                             an optional (x, Mx) partial fused into the final
//                                             coefficients
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

// Tiled analysis launches of at most kAnaWideItems tiles (a single instance: the GPU is far
// from full, and the longest tiles set the launch's duration) run kAnaWide-thread workgroups;
// larger ones keep kThreads, which fit more tiles per compute unit.
inline bool ana_wide(int items) { return items <= kAnaWideItems; }

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

// One workgroup computes one ST x ST tile (n x n when the layer is smaller) of a layer's image
// phi = W^-1 c / delta in a single launch.  Output rows [a, a + w) of a synthesis level read the
// coefficient rows [floor(a/2) - 2, floor((a + w - 1)/2)] of each band (periodic), so the
// tile depends on a window of every level that shrinks to about six coefficients at the coarse
// end; the workgroup loads those windows of every level at once and synthesises them from the
// coarsest level down, each level's LL window staying in LDS.  Neighbouring tiles recompute
// the overlapping coarse windows, which costs a few hundred values per tile; no intermediate
// goes through global memory and every output takes exactly the row and column passes of the
// level-by-level transform: x_i = sum_{t = i mod 2} h_t a_{(i-t)/2} + g_t d_{(i-t)/2}, rows
// (the vertical pass) then columns.  Every loop runs over the compile-time bound of its
// window (valid entries masked), so no index needs a run-time division.
constexpr int kMaxLevels = 10;   // layers are at most 1024 x 1024

// Bound of the window side at level l of an st-wide output tile: (st - 1)/2 + 3 at the first
// level (tiles start at even positions), then half of the previous side plus 3.
constexpr int syn_window(int st, int l) {
    int w = st;
    for (int j = 1; j <= l; ++j) w = (j == 1 ? (w - 1) / 2 : w / 2) + 3;
    return w;
}
// LDS offset of level l's buffer (2 W rows of 2 W + 1; quadrant rows and columns at W)
constexpr int syn_boff(int st, int l) {
    int s = 0;
    for (int j = 1; j < l; ++j) s += 2 * syn_window(st, j) * (2 * syn_window(st, j) + 1);
    return s;
}
constexpr int cdiv_c(int a, int b) { return (a + b - 1) / b; }
// loads per thread of all levels' windows (four quadrants per level at the bound)
constexpr int syn_loads(int st) {
    int s = 0;
    for (int l = 1; l <= kMaxLevels; ++l) s += cdiv_c(4 * syn_window(st, l) * syn_window(st, l), kThreads);
    return s;
}

template <typename T, int ST>
struct SynTile {
    // the windows of levels 0..kMaxLevels of one tile: start and side per direction
    int ay[kMaxLevels + 1], wy[kMaxLevels + 1], ax[kMaxLevels + 1], wx[kMaxLevels + 1];

    // quadrant loads of level l (Q = 4 W^2 slots, q = slot / W^2: 0 LL, 1 top right, 2 bottom
    // left, 3 bottom right of the Mallat block), into v starting at index k0
    template <int l>
    __device__ __forceinline__ void load(const T* __restrict__ C, int n, int L, T* v, int* dst, int k0) const {
        constexpr int W = syn_window(ST, l), Q = 4 * W * W, P = cdiv_c(Q, kThreads), SB = 2 * W + 1;
        const int m = n >> l;
        if (l > L) {   // uniform: levels the layer does not have
#pragma unroll
            for (int k = 0; k < P; ++k) dst[k0 + k] = -1;
            return;
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int e = threadIdx.x + k * kThreads;
            const int q = e / (W * W), rem = e - q * (W * W), rr = rem / W, cc = rem - rr * W;
            const int hr = q >> 1, hc = q & 1;
            const bool ok = l <= L && e < Q && rr < wy[l] && cc < wx[l] && (q > 0 || l == L);
            const int kr = (ay[l] + rr) & (m - 1), kc = (ax[l] + cc) & (m - 1);
            v[k0 + k] = C[ok ? (kr + m * hr) * n + kc + m * hc : 0];
            dst[k0 + k] = ok ? syn_boff(ST, l) + (hr * W + rr) * SB + hc * W + cc : -1;
        }
    }

    // synthesis of level l: level l - 1's LL window (the image tile at l = 1)
    template <int l>
    __device__ __forceinline__ void level(T* __restrict__ buf, T* __restrict__ I, const Taps<T>& tp, T* __restrict__ phi,
                                          size_t off, int n, T inv_delta) const {
        constexpr int W = syn_window(ST, l), SB = 2 * W + 1, W2 = syn_window(ST, l - 1);
        const T* B = buf + syn_boff(ST, l);
        const int a2 = ay[l - 1], h2 = wy[l - 1], b2 = ax[l - 1], v2 = wx[l - 1], wxl = wx[l];
        if constexpr (l == 1) {
            // the finest level: the tile starts at even rows and columns, so outputs 2i and 2i + 1
            // read the same three coefficients of each band (base = i + 2) and are formed as a
            // pair, with the same arithmetic as one at a time
            using V2 = typename Vec2<T>::type;
            for (int e = threadIdx.x; e < (ST / 2) * 2 * W; e += kThreads) {   // vertical pass
                const int i = e / (2 * W), col = e - i * (2 * W);
                const int cc = col >= W ? col - W : col;
                if (2 * i < h2 && cc < wxl) {
                    T ev = 0, od = 0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const T a = B[(i + 2 - k) * SB + col], b = B[(W + i + 2 - k) * SB + col];
                        ev += tp.he[k] * a + tp.ge[k] * b;
                        od += tp.ho[k] * a + tp.go[k] * b;
                    }
                    I[(2 * i) * SB + col] = ev;
                    I[(2 * i + 1) * SB + col] = od;
                }
            }
            __syncthreads();
            for (int e = threadIdx.x; e < ST * (ST / 2); e += kThreads) {   // horizontal pass
                const int i = e / (ST / 2), j = e - i * (ST / 2);
                if (i < h2 && 2 * j < v2) {
                    T ev = 0, od = 0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const T a = I[i * SB + j + 2 - k], b = I[i * SB + W + j + 2 - k];
                        ev += tp.he[k] * a + tp.ge[k] * b;
                        od += tp.ho[k] * a + tp.go[k] * b;
                    }
                    *reinterpret_cast<V2*>(phi + off + size_t(ay[0] + i) * n + ax[0] + 2 * j) =
                        V2{ev * inv_delta, od * inv_delta};
                }
            }
            __syncthreads();
            return;
        }
        // vertical pass: the rows of level l - 1's window, both column halves (I: rows of SB)
        for (int e = threadIdx.x; e < W2 * 2 * W; e += kThreads) {
            const int i = e / (2 * W), col = e - i * (2 * W);
            const int cc = col >= W ? col - W : col;
            if (i < h2 && cc < wxl) {
                const int ai = a2 + i, odd = ai & 1, base = (ai >> 1) - (a2 >> 1) + 2;
                T v = 0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const T a = B[(base - k) * SB + col], b = B[(W + base - k) * SB + col];
                    v += (odd ? tp.ho[k] : tp.he[k]) * a + (odd ? tp.go[k] : tp.ge[k]) * b;
                }
                I[i * SB + col] = v;
            }
        }
        __syncthreads();
        // horizontal pass: into level l - 1's LL quadrant, or the image
        for (int e = threadIdx.x; e < W2 * W2; e += kThreads) {
            const int i = e / W2, j = e - i * W2;
            if (i < h2 && j < v2) {
                const int aj = b2 + j, odd = aj & 1, base = (aj >> 1) - (b2 >> 1) + 2;
                T v = 0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const T a = I[i * SB + base - k], b = I[i * SB + W + base - k];
                    v += (odd ? tp.ho[k] : tp.he[k]) * a + (odd ? tp.go[k] : tp.ge[k]) * b;
                }
                if constexpr (l > 1)
                    buf[syn_boff(ST, l - 1) + i * (2 * W2 + 1) + j] = v;
                else
                    phi[off + size_t(ay[0] + i) * n + ax[0] + j] = v * inv_delta;
            }
        }
        __syncthreads();
    }
};

template <typename T, int ST, int l>
__device__ __forceinline__ void syn_load_all(const SynTile<T, ST>& tl, const T* C, int n, int L, T* v, int* dst, int k0) {
    if constexpr (l <= kMaxLevels) {
        tl.template load<l>(C, n, L, v, dst, k0);
        syn_load_all<T, ST, l + 1>(tl, C, n, L, v, dst, k0 + cdiv_c(4 * syn_window(ST, l) * syn_window(ST, l), kThreads));
    }
}

template <typename T, int ST, int l>
__device__ __forceinline__ void syn_levels(const SynTile<T, ST>& tl, T* buf, T* I, const Taps<T>& tp, T* phi, size_t off,
                                           int n, int L, T inv_delta) {
    if constexpr (l >= 1) {
        if (l <= L) tl.template level<l>(buf, I, tp, phi, off, n, inv_delta);
        syn_levels<T, ST, l - 1>(tl, buf, I, tp, phi, off, n, L, inv_delta);
    }
}

template <typename T, int ST>
__global__ void __launch_bounds__(kThreads) k_idwt(const LayerDev* __restrict__ lays, const int2* __restrict__ items,
                                                    Filt<T> f, const T* __restrict__ coef, T* __restrict__ phi,
                                                    const int32_t* __restrict__ skip) {
    constexpr int W1 = syn_window(ST, 1);
    constexpr int PER = syn_loads(ST);
    __shared__ T buf[syn_boff(ST, kMaxLevels + 1)];
    __shared__ T I[ST * (2 * W1 + 1)];
    const int2 it = items[die_ordered_block()];
    if (it.x < 0) return;               // padding of the die-ordered grid
    const LayerDev d = lays[it.x];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const int n = d.n, L = d.levels;
    const int ts = n < ST ? n : ST, tx = n / ts;
    const int ty = it.y / tx;
    SynTile<T, ST> tl;
    tl.ay[0] = ty * ts;
    tl.wy[0] = ts;
    tl.ax[0] = (it.y - ty * tx) * ts;
    tl.wx[0] = ts;
#pragma unroll
    for (int l = 1; l <= kMaxLevels; ++l) {   // >> of a negative start: floor
        tl.wy[l] = ((tl.ay[l - 1] + tl.wy[l - 1] - 1) >> 1) - (tl.ay[l - 1] >> 1) + 3;
        tl.wx[l] = ((tl.ax[l - 1] + tl.wx[l - 1] - 1) >> 1) - (tl.ax[l - 1] >> 1) + 3;
        tl.ay[l] = (tl.ay[l - 1] >> 1) - 2;
        tl.ax[l] = (tl.ax[l - 1] >> 1) - 2;
    }
    {
        T v[PER];
        int dst[PER];
        syn_load_all<T, ST, 1>(tl, coef + d.off, n, L, v, dst, 0);
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (dst[k] >= 0) buf[dst[k]] = v[k];
    }
    __syncthreads();
    const Taps<T> tp(f);
    syn_levels<T, ST, kMaxLevels>(tl, buf, I, tp, phi, size_t(d.off), n, L, T(d.inv_delta));
}

// ------------------------------------------------------------------ wavelet analysis

// K consecutive analysis levels l1 .. l1 + K - 1 of one layer for one tile (item: layer, tile,
// l1 | K << 8 | T << 16, partial slot), T = 16 >> (K - 1): from an input window of
// v0 = (T << K) + 4 ((1 << K) - 1) values per side (a_k = sum_t h_t x_{2k+t} reads 2 v + 4
// inputs for v outputs) down to a T x T tile of the K-th level.  The workgroup loads its
// input window once (the image, or the LL band of a previous launch), then per level a row
// pass (low and high pass of every input row) and a column pass; the LL window of each level
// stays in LDS for the next.  Its outputs at level j are the T 2^(K-1-j) square block of
// positions its tile covers (every position of a level belongs to exactly one tile; 16 x 16
// at the first level); the rest of each LL window is the halo the next level reads.  Final
// coefficients are scaled by 1/delta; MODE 1 (inside M x) adds (alpha D)_i x_i and sums
// (x, out) over the tile's outputs into its partial slot, MODE 2 (the right-hand side) sums
// (out, out) there.  The last level's LL band goes to ll_out for the next launch or the coarse
// kernel, or is a coefficient when it is the layer's coarsest.  Every thread owns at most one
// output position per level, so the prior and x operands of its outputs are requested before
// the window.  FP32 runs up to three levels per launch, FP64 up to two (LDS).
constexpr int ana_v0(int K) { return ((16 >> (K - 1)) << K) + 4 * ((1 << K) - 1); }
template <typename T> struct AnaMaxLevels;
template <> struct AnaMaxLevels<float> { static constexpr int value = 3; };
template <> struct AnaMaxLevels<double> { static constexpr int value = 2; };

template <typename T, int MODE, int K, int NT>
__device__ __forceinline__ void dwt_tiles_body(const LayerDev& d, int4 it, const Taps<T>& tp, const T* __restrict__ img,
                                               const T* __restrict__ ll_in, T* __restrict__ ll_out, T* __restrict__ out,
                                               const T* __restrict__ prior_a, const T* __restrict__ xprior, T* A, T* Bf,
                                               double& dot) {
    constexpr bool PRIOR = MODE == 1;
    constexpr int TT = 16 >> (K - 1), V0 = ana_v0(K), SA = V0 + 1;
    const int n = d.n, l1 = it.z & 0xff;
    const int nb_in = n >> (l1 - 1);
    const int mt = (nb_in >> K) / TT;
    const int ty = it.y / mt, tx = it.y - ty * mt;
    const bool fin = l1 + K - 1 == d.levels;
    const size_t base = size_t(d.off);
    // the first NT threads of the workgroup do the work; the others (NT below the launch
    // width) take no item but join the barriers
    const int t = int(threadIdx.x) < NT ? int(threadIdx.x) : (1 << 20);
    T pa[K][4], xp[K][4];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int own = TT << (K - 1 - j);
#pragma unroll
        for (int b = 0; b < 4; ++b) pa[j][b] = xp[j][b] = T(0);
        if (PRIOR && t < own * own) {   // o[3] (the LL position) is a valid address even when it is not an output
            const int m = n >> (l1 + j), r = t / own, c = t - r * own;
            const int gy = ty * own + r, gx = tx * own + c;
            const size_t o[4] = {base + size_t(gy) * n + m + gx, base + size_t(m + gy) * n + gx,
                                 base + size_t(m + gy) * n + m + gx, base + size_t(gy) * n + gx};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                pa[j][b] = prior_a[o[b]];
                xp[j][b] = xprior[o[b]];
            }
        }
    }
    // input window in 16-byte chunks: its start (a multiple of T 2^K >= 16) and the block
    // side are multiples of the chunk, so a chunk is contiguous across the periodic wrap
    {
        using VC = Vec16<T>;
        constexpr int CPR = V0 / VC::n, NCH = V0 * CPR, PER = cdiv_c(NCH, NT);
        const T* src = (l1 == 1 ? img : ll_in) + d.off;
        const int sy = (ty * TT) << K, sx = (tx * TT) << K;
        typename VC::type v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {   // unconditional loads (clamped index)
            const int e0 = t + k * NT, e = e0 < NCH ? e0 : NCH - 1;
            const int r = e / CPR, q = e - r * CPR;
            v[k] = *reinterpret_cast<const typename VC::type*>(src + ((sy + r) & (nb_in - 1)) * n +
                                                               ((sx + q * VC::n) & (nb_in - 1)));
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = t + k * NT;
            if (e < NCH) {
                const int r = e / CPR, q = e - r * CPR;
                VC::put(&A[r * SA + q * VC::n], v[k]);
            }
        }
    }
    __syncthreads();
    const T s = T(d.inv_delta);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int vin = (TT << (K - j)) + 4 * ((1 << (K - j)) - 1);   // compile-time after unrolling
        const int vo = (vin - 4) >> 1, sb = 2 * vo + 1;
        // row pass: low- and high-pass outputs of one (row, k) from the same six inputs
        for (int e = t; e < vin * vo; e += NT) {
            const int rr = e / vo, k = e - rr * vo;
            T lo = 0, hi = 0;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const T x = A[rr * SA + 2 * k + q];
                lo += tp.h[q] * x;
                hi += tp.g[q] * x;
            }
            Bf[rr * sb + k] = lo;
            Bf[rr * sb + vo + k] = hi;
        }
        __syncthreads();
        // column pass: the tile's own positions (item t is thread t's), then the halo rows and
        // columns the next level reads
        const int own = TT << (K - 1 - j);
        const int m = n >> (l1 + j);
        const bool last = j == K - 1;
        for (int e = t; e < vo * vo; e += NT) {
            int r, c;
            if (e < own * own) {
                r = e / own;
                c = e - r * own;
            } else {
                const int e2 = e - own * own;   // halo: rows [0, own) x columns [own, vo), then rows [own, vo)
                if (e2 < own * (vo - own)) {
                    r = e2 / (vo - own);
                    c = own + e2 - r * (vo - own);
                } else {
                    const int e3 = e2 - own * (vo - own);
                    r = own + e3 / vo;
                    c = e3 - (e3 / vo) * vo;
                }
            }
            T ll = 0, yh = 0, xh = 0, hh = 0;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const T lo = Bf[(2 * r + q) * sb + c], hi = Bf[(2 * r + q) * sb + vo + c];
                ll += tp.h[q] * lo;
                yh += tp.g[q] * lo;
                xh += tp.h[q] * hi;
                hh += tp.g[q] * hi;
            }
            A[r * SA + c] = ll;
            if (e < own * own) {
                const int gy = ty * own + r, gx = tx * own + c;
                const size_t o[4] = {base + size_t(gy) * n + m + gx, base + size_t(m + gy) * n + gx,
                                     base + size_t(m + gy) * n + m + gx, base + size_t(gy) * n + gx};
                const T v4[4] = {xh, yh, hh, ll};
                const int nout = last && fin ? 4 : 3;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if (b < nout) {
                        T val = v4[b] * s;
                        if (PRIOR) val += pa[j][b] * xp[j][b];
                        out[o[b]] = val;
                        dot += double(val) * (MODE == 2 ? double(val) : double(xp[j][b]));   // (x, M x) or (b, b)
                    }
                }
                if (last && !fin) ll_out[o[3]] = ll;
            }
        }
        __syncthreads();
    }
}

// Levels coarse_lev..levels of one layer in LDS (the coarse block, in A and B).  After the
// last level the block holds the whole coarse Mallat pyramid; it is written once, each thread
// owning fixed positions whose prior and x operands it requested first.  Returns the thread's
// share of the partial ((x, out) for MODE 1, (out, out) for MODE 2).
template <typename T, int MODE>
__device__ __forceinline__ double dwt_coarse_body(const LayerDev& d, const Filt<T>& f, const T* __restrict__ img,
                                                  const T* __restrict__ ll_in, T* __restrict__ out,
                                                  const T* __restrict__ prior_a, const T* __restrict__ xprior,
                                                  T* __restrict__ A, T* __restrict__ B) {
    constexpr bool PRIOR = MODE == 1;
    constexpr int CB = CoarseBlock<T>::value;
    const int n = d.n, lc = d.coarse_lev, levels = d.levels;
    double dot = 0;
    if (levels >= lc) {
        // 16-byte chunks of consecutive positions of a row (nb0 >= 8 is a multiple of the
        // chunk; layer offsets and rows keep chunks aligned)
        using VC = Vec16<T>;
        using V = typename VC::type;
        constexpr int PERC = CB * CB / (VC::n * kThreads);
        const int nb0 = n >> (lc - 1), lg0 = ilog2i(nb0), nch = nb0 * nb0 / VC::n;
        const T* src = (lc == 1 ? img : ll_in) + d.off;
        const Taps<T> tp(f);
        V pa[PERC], xp[PERC], v[PERC];
#pragma unroll
        for (int k = 0; k < PERC; ++k) {   // unconditional (clamped) loads
            const int ch0 = threadIdx.x + k * kThreads, ch = ch0 < nch ? ch0 : 0;
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
            const int ch = threadIdx.x + k * kThreads;
            if (ch < nch) {
                const int e = ch * VC::n;
                VC::put(&A[(e >> lg0) * CB + (e & (nb0 - 1))], v[k]);
            }
        }
        __syncthreads();
        for (int lev = lc; lev <= levels; ++lev) {
            const int nb = n >> (lev - 1), m = nb >> 1, lgm = ilog2i(m), lg = lgm + 1;
            for (int e = threadIdx.x; e < nb * m; e += kThreads) {   // rows: [a | d]
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
            for (int e = threadIdx.x; e < m * nb; e += kThreads) {   // columns
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
            const int ch = threadIdx.x + k * kThreads;
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
    return dot;
}

// The coarse levels of every layer, one workgroup per layer.  (A fused variant, in which the
// workgroup that finishes a layer's last tile runs them, needs device-scope fences around a
// counter; on gfx950 those cost more than this launch.)
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) k_dwt_coarse(const LayerDev* __restrict__ lays, Filt<T> f,
                                                          const T* __restrict__ img, const T* __restrict__ ll_in,
                                                          T* __restrict__ out, const T* __restrict__ prior_a,
                                                          const T* __restrict__ xprior, double* __restrict__ dotpart,
                                                          const int32_t* __restrict__ skip) {
    constexpr int CB = CoarseBlock<T>::value;
    __shared__ T A[CB * CB];
    __shared__ T B[CB * CB];
    const LayerDev d = lays[blockIdx.x];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const double dot = dwt_coarse_body<T, MODE>(d, f, img, ll_in, out, prior_a, xprior, A, B);
    if (MODE != 0 && dotpart) {
        const double vv[1] = {dot};
        block_partials<1>(vv, dotpart, 0, 0, d.pq0 + d.pq_coarse);
    }
}

// LW: workgroup width, kThreads or kAnaWide (the wide one only where the launch has few tiles:
// it gives the three-level tiles, the longest, twice the threads; every tile computes the same
// values and partial either way).
template <typename T, int MODE, int LW>
__global__ void __launch_bounds__(LW) k_dwt_tiles(const LayerDev* __restrict__ lays, const int4* __restrict__ items,
                                                         Filt<T> f, const T* __restrict__ img, const T* __restrict__ ll_in,
                                                         T* __restrict__ ll_out, T* __restrict__ out,
                                                         const T* __restrict__ prior_a, const T* __restrict__ xprior,
                                                         double* __restrict__ dotpart, const int32_t* __restrict__ skip) {
    constexpr int KM = AnaMaxLevels<T>::value, V0 = ana_v0(KM), V1 = (V0 - 4) / 2;
    __shared__ T A[V0 * (V0 + 1)];
    __shared__ T Bf[V0 * (2 * V1 + 1)];
    const int4 it = items[die_ordered_block()];
    if (it.x < 0) return;               // padding of the die-ordered grid
    const LayerDev d = lays[it.x];
    if (skip && skip[d.inst]) return;   // tolerance mode: the instance has converged
    const Taps<T> tp(f);
    const int K = (it.z >> 8) & 0xff;
    double dot = 0;
    // three-level tiles (the largest windows) over the whole workgroup, the others over four
    // wavefronts
    if (KM >= 3 && K == 3)
        dwt_tiles_body<T, MODE, KM >= 3 ? 3 : 1, LW>(d, it, tp, img, ll_in, ll_out, out, prior_a, xprior, A, Bf, dot);
    else if (K == 2)
        dwt_tiles_body<T, MODE, 2, kThreads>(d, it, tp, img, ll_in, ll_out, out, prior_a, xprior, A, Bf, dot);
    else
        dwt_tiles_body<T, MODE, 1, kThreads>(d, it, tp, img, ll_in, ll_out, out, prior_a, xprior, A, Bf, dot);
    if (MODE != 0 && dotpart) {
        const double vv[1] = {dot};
        block_partials<1, LW>(vv, dotpart, 0, 0, d.pq0 + it.w);
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
                                                            const int32_t* __restrict__ skip, const T* __restrict__ xw,
                                                            T* __restrict__ wsl) {
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
    T wx = 0, wy = 0, wc = 0;
    if (sub) {
        wx = w[W.soff + si * ns + sj];
        wy = w[W.soff + ns * ns + si * ns + sj];
        if (xw) wc = xw[W.soff / 2 + si * ns + sj];   // off-diagonal of the subaperture's 2x2 block
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
            if (xw) {   // C_eta^-1 block [[wx, wc], [wc, wy]]
                tx = wx * sx + wc * sy;
                ty = wc * sx + wy * sy;
            } else {
                tx = wx * sx;
                ty = wy * sy;
            }
            // a tip/tilt-filtered sensor keeps its weighted slopes for the rank-2 correction
            // (each subaperture written by the tile that owns its first node)
            if (wsl && W.tt && si >= i0 && si < i0 + kTile && sj >= j0 && sj < j0 + kTile) {
                wsl[W.soff + si * ns + sj] = tx;
                wsl[W.soff + ns * ns + si * ns + sj] = ty;
            }
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
// With the 2x2 noise blocks (xw) the weighted slope pair of a subaperture is
// [[wx, wc], [wc, wy]] (sx, sy), zero on an inactive subaperture (wx = wy = 0).  The weighted
// slopes of a tip/tilt-filtered sensor also go to wsl (node (i, j) writes subaperture (i, j)).
// The node's sensor is found from the sensor of the block's first node (a setup table), so
// that it costs one or two dependent loads instead of a binary search over all sensors.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_slopes_adj(const WfsDev* __restrict__ wfs, int G, int64_t V,
                                                          const T* __restrict__ w, const T* __restrict__ s,
                                                          T* __restrict__ psi, int weighted, const T* __restrict__ xw,
                                                          T* __restrict__ wsl, const int32_t* __restrict__ node_sensor) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= V) return;
    int g = node_sensor[blockIdx.x];
    while (g + 1 < G && wfs[g + 1].noff <= e) ++g;
    const WfsDev W = wfs[g];
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
    auto tb = [&](int comp, int si, int sj) -> T {   // the block form
        const bool ok = si >= 0 && si < ns && sj >= 0 && sj < ns;
        const int64_t q = ok ? si * ns + sj : 0;
        const int64_t ox = W.soff + q, oy = W.soff + int64_t(ns) * ns + q;
        const T wx = w[ox], wy = w[oy], wc = xw[W.soff / 2 + q], sx = s[ox], sy = s[oy];
        const bool act = ok && (wx != T(0) || wy != T(0));
        const T v = comp == 0 ? wx * sx + wc * sy : wc * sx + wy * sy;
        return act ? v : T(0);
    };
    if (weighted && xw)
        psi[e] = T(0.5) * ((tb(0, i, j - 1) - tb(0, i, j)) + (tb(0, i - 1, j - 1) - tb(0, i - 1, j))) +
                 T(0.5) * ((tb(1, i - 1, j) - tb(1, i, j)) + (tb(1, i - 1, j - 1) - tb(1, i, j - 1)));
    else
        psi[e] = T(0.5) * ((t(0, i, j - 1) - t(0, i, j)) + (t(0, i - 1, j - 1) - t(0, i - 1, j))) +
                 T(0.5) * ((t(1, i - 1, j) - t(1, i, j)) + (t(1, i - 1, j - 1) - t(1, i, j - 1)));
    if (weighted && wsl && W.tt && i < ns && j < ns) {
        wsl[W.soff + i * ns + j] = xw ? tb(0, i, j) : t(0, i, j);
        wsl[W.soff + int64_t(ns) * ns + i * ns + j] = xw ? tb(1, i, j) : t(1, i, j);
    }
}

// Tip/tilt filter of a sensor's C_eta^-1 (B - B T (T^T B T)^-1 T^T B): the sensor-node vector
// Gamma^T B y already holds the B part; this subtracts m_x v_x + m_y v_y, v_k = Gamma^T B T e_k
// (precomputed) and m = (T^T B T)^-1 T^T B y, whose two sums over the weighted slopes B y (wsl)
// are taken in FP64 in a fixed order.  One workgroup per sensor.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_tt_correct(const WfsDev* __restrict__ wfs, const T* __restrict__ wsl,
                                                          const T* __restrict__ ttv, int64_t V, T* __restrict__ psi,
                                                          const int32_t* __restrict__ skip) {
    const WfsDev W = wfs[blockIdx.x];
    if (!W.tt) return;
    if (skip && skip[W.inst]) return;   // tolerance mode: the instance has converged
    const int n2 = W.ns * W.ns, nv = (W.ns + 1) * (W.ns + 1);
    double v[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < n2; k += kThreads) {
        v[0] += double(wsl[W.soff + k]);
        v[1] += double(wsl[W.soff + n2 + k]);
    }
    __shared__ double sh[2][kThreads / 64];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double w = wave_sum(v[c]);
        if ((threadIdx.x & 63) == 0) sh[c][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    const double tx = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    const double ty = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    const double mx = W.tg[0] * tx + W.tg[1] * ty, my = W.tg[1] * tx + W.tg[2] * ty;
    for (int k = threadIdx.x; k < nv; k += kThreads) {
        const int64_t o = W.noff + k;
        psi[o] = T(double(psi[o]) - mx * double(ttv[o]) - my * double(ttv[V + o]));
    }
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
    "idwt", "data_term", "adj_gather", "dwt_tiles", "dwt_coarse", "slopes_adj", "residual", "gram", "gram_solve",
    "galerkin_apply", "init_dir", "update1", "update2", "finish", "fwd_slopes", "tt_correct"};

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

template <typename T>
inline Filt<float> f32_filt(const Filt<T>& f) {
    Filt<float> g;
    for (int t = 0; t < 6; ++t) {
        g.h[t] = float(f.h[t]);
        g.g[t] = float(f.g[t]);
    }
    return g;
}

// The synthesis in one launch: kSynTile x kSynTile output tiles, or tiles of half that side
// when the large ones would give fewer workgroups than kSmallTileBelow (a single small
// instance): the launch is then bound by the latency of each workgroup, and four times as many
// smaller tiles finish sooner.  The tile side changes no output bit.
template <typename T>
void launch_winv(const Ctx& c, const T* x, T* phi, hipStream_t s, const OpBufs* /*ob*/, const int32_t* skip) {
    const Filt<T> f = make_filt<T>();
    const LayerDev* lays = c.at<LayerDev>(c.lay.layers);
    const int2* items = c.at<int2>(c.lay.syn_items);
    ProfScope ps_(c, KID_IDWT, s);
    if (c.syn_tile == kSynTile / 2 || (c.syn_tile == 0 && c.syn_large < kSmallTileBelow))
        k_idwt<T, kSynTile / 2><<<c.syn_small, kThreads, 0, s>>>(lays, items, f, x, phi, skip);
    else if (c.syn_tile == 2 * kSynTile && sizeof(T) == 4)   // 64 x 64 tiles: FP32 only (LDS)
        k_idwt<float, 2 * kSynTile><<<c.syn_huge, kThreads, 0, s>>>(lays, items + c.syn_small + c.syn_large, f32_filt(f),
                                                                     reinterpret_cast<const float*>(x),
                                                                     reinterpret_cast<float*>(phi), skip);
    else
        k_idwt<T, kSynTile><<<c.syn_large, kThreads, 0, s>>>(lays, items + c.syn_small, f, x, phi, skip);
}

// The analysis: the tiled launches (finest levels first), each LL band handed to the next
// launch through the two scratch vectors, then the coarse kernel.
template <typename T>
void launch_winvt(const Ctx& c, const T* img, T* y, const T* xprior, double* pq_part, hipStream_t s,
                  const OpBufs* ob, const int32_t* skip) {
    const Filt<T> f = make_filt<T>();
    const OpBufs bb = ob ? *ob : ctx_bufs(c);
    T* buf[2] = {reinterpret_cast<T*>(bb.tmp0), reinterpret_cast<T*>(bb.tmp1)};
    const LayerDev* lays = c.at<LayerDev>(c.lay.layers);
    const int4* items = c.at<int4>(c.lay.ana_items);
    const T* pa = c.at<T>(c.lay.prior_a);
    const int J = int(c.steps.size());
    // with xprior: + alpha D x and the (x, y) partials; without it but with pq_part: (y, y)
    const int mode = xprior ? 1 : (pq_part ? 2 : 0);
    for (int j = 0; j < J; ++j) {
        const StepInfo& w = c.steps[j];
        ProfScope ps_(c, KID_DWT_TILES, s);
        auto go = [&](auto kern, int lw) {
            kern<<<w.ni, lw, 0, s>>>(lays, items + w.loff, f, img, buf[(j + 1) & 1], buf[j & 1], y, pa, xprior,
                                     pq_part, skip);
        };
        const bool wide = ana_wide(w.ni);
        if (mode == 1) wide ? go(k_dwt_tiles<T, 1, kAnaWide>, kAnaWide) : go(k_dwt_tiles<T, 1, kThreads>, kThreads);
        else if (mode == 2) wide ? go(k_dwt_tiles<T, 2, kAnaWide>, kAnaWide) : go(k_dwt_tiles<T, 2, kThreads>, kThreads);
        else wide ? go(k_dwt_tiles<T, 0, kAnaWide>, kAnaWide) : go(k_dwt_tiles<T, 0, kThreads>, kThreads);
    }
    ProfScope ps_(c, KID_DWT_COARSE, s);
    auto go = [&](auto kern) {
        kern<<<c.L, kCoarseThreads, 0, s>>>(lays, f, img, buf[(J + 1) & 1], y, pa, xprior, pq_part, skip);
    };
    if (mode == 1) go(k_dwt_coarse<T, 1>);
    else if (mode == 2) go(k_dwt_coarse<T, 2>);
    else go(k_dwt_coarse<T, 0>);
}

// The rank-2 tip/tilt correction of the filtered sensors (after the data term or the slope
// adjoint wrote the weighted slopes to wsl).
template <typename T>
void launch_tt_correct(const Ctx& c, T* psi_nodes, const T* wsl, hipStream_t s, const int32_t* skip) {
    if (!c.any_tt) return;
    ProfScope ps_(c, KID_TT_CORRECT, s);
    k_tt_correct<T><<<c.G, kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), wsl, c.at<T>(c.lay.ttv), c.V, psi_nodes, skip);
}

template <typename T>
void launch_data_term(const Ctx& c, const T* phi, T* psi_nodes, hipStream_t s, const int32_t* skip, T* wsl) {
    if (!wsl) wsl = c.at<T>(c.lay.wslopes);
    {
        ProfScope ps_(c, KID_DATA_TERM, s);
        k_data_term<T><<<c.data_grid, kDataThreads, 0, s>>>(
            c.at<WfsDev>(c.lay.wfs), c.at<int2>(c.lay.data_tiles), c.at<LayerDev>(c.lay.layers),
            c.at<int32_t>(c.lay.cellidx), c.at<T>(c.lay.frac), phi, c.at<T>(c.lay.weight), psi_nodes, skip,
            c.any_cross ? c.at<T>(c.lay.xweight) : nullptr, c.any_tt ? wsl : nullptr);
    }
    launch_tt_correct<T>(c, psi_nodes, wsl, s, skip);
}

// weighted = 1: Gamma^T C_eta^-1 s without the tip/tilt correction (launch_tt_correct follows
// where the frame needs it); weighted = 0: Gamma^T (mask s).
template <typename T>
void launch_slopes_adj(const Ctx& c, const T* slopes, T* psi_nodes, int weighted, hipStream_t s) {
    ProfScope ps_(c, KID_SLOPES_ADJ, s);
    k_slopes_adj<T><<<cdiv(c.V, kThreads), kThreads, 0, s>>>(
        c.at<WfsDev>(c.lay.wfs), c.G, c.V, c.at<T>(c.lay.weight), slopes, psi_nodes, weighted,
        weighted && c.any_cross ? c.at<T>(c.lay.xweight) : nullptr, weighted && c.any_tt ? c.at<T>(c.lay.wslopes) : nullptr,
        c.at<int32_t>(c.lay.node_sensor));
}

template <typename T>
void launch_adj_gather(const Ctx& c, const T* psi_nodes, T* psi_layers, hipStream_t s, const int32_t* skip) {
    ProfScope ps_(c, KID_ADJ_GATHER, s);
    if (c.max_rng <= kRMax) {
        const bool wide = c.gather_rows > 1;
        const int grid = wide ? c.gather_grid4 : c.gather_grid1;
        const int2* tiles = c.at<int2>(c.lay.gather_tiles) + (wide ? c.gather_grid1 : 0);
        auto go = [&](auto kern) {
            kern<<<grid, kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.at<LayerDev>(c.lay.layers),
                                                   tiles, c.at<int64_t>(c.lay.recbase),
                                                   c.at<GatherRec<T>>(c.lay.grecs), psi_nodes, psi_layers, skip);
        };
        auto gow = [&](auto kern) {
            kern<<<grid, kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.at<LayerDev>(c.lay.layers),
                                                   tiles, c.at<int64_t>(c.lay.recbase),
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
    launch_data_term<T>(c, phi, psi_n, s, skip, reinterpret_cast<T*>(bb.wslopes));
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
    launch_tt_correct<T>(c, psi_n, c.at<T>(c.lay.wslopes), s, nullptr);
    launch_adj_gather<T>(c, psi_n, psi_l, s);
    launch_winvt<T>(c, psi_l, b, static_cast<const T*>(nullptr), bb_part, s);
}

// Launches one operator kernel with the arguments it has inside M x (input: the coefficient
// vector c; intermediates: the context buffers).  step selects the tiled wavelet level.
template <typename T>
static hipError_t launch_one(const Ctx& c, int kid, int step, hipStream_t s) {
    const Filt<T> f = make_filt<T>();
    const LayerDev* lays = c.at<LayerDev>(c.lay.layers);
    T* buf[2] = {c.at<T>(c.lay.tmp0), c.at<T>(c.lay.tmp1)};
    const T* x = c.at<T>(c.lay.c);
    T* y = c.at<T>(c.lay.vy);
    const int J = int(c.steps.size());
    switch (kid) {
        case KID_APPLY:   // all of M x
            launch_apply_M<T>(c, x, y, nullptr, s, nullptr, nullptr);
            break;
        case KID_IDWT:
            launch_winv<T>(c, x, c.at<T>(c.lay.nodal), s, nullptr, nullptr);
            break;
        case KID_DATA_TERM:
            launch_data_term<T>(c, c.at<T>(c.lay.nodal), c.at<T>(c.lay.psi_nodes), s, nullptr, nullptr);
            break;
        case KID_ADJ_GATHER:
            launch_adj_gather<T>(c, c.at<T>(c.lay.psi_nodes), c.at<T>(c.lay.psi_layers), s);
            break;
        case KID_DWT_TILES: {
            if (step < 0 || step >= J) return hipErrorInvalidValue;
            const StepInfo& w = c.steps[step];
            auto go = [&](auto kern, int lw) {
                kern<<<w.ni, lw, 0, s>>>(lays, c.at<int4>(c.lay.ana_items) + w.loff, f, c.at<T>(c.lay.psi_layers),
                                         buf[(step + 1) & 1], buf[step & 1], y, c.at<T>(c.lay.prior_a), x,
                                         c.at<double>(c.lay.pq_part), nullptr);
            };
            if (ana_wide(w.ni)) go(k_dwt_tiles<T, 1, kAnaWide>, kAnaWide);
            else go(k_dwt_tiles<T, 1, kThreads>, kThreads);
            break;
        }
        case KID_DWT_COARSE:
            k_dwt_coarse<T, 1><<<c.L, kCoarseThreads, 0, s>>>(lays, f, c.at<T>(c.lay.psi_layers), buf[(J + 1) & 1],
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
    template void launch_data_term<T>(const Ctx&, const T*, T*, hipStream_t, const int32_t*, T*);         \
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
