// HIP kernels (gfx950 / CDNA4) of the augmented-FEWHA frame solve.
//
// Operator M = W^-T A^T C^-1 A W^-1 + alpha D (Sec. 3) as a chain of HBM-streaming kernels:
//   k_idwt_level   per level, all layers: periodic db3 synthesis (W^-1 = DWT^T / delta_l)
//   k_data_term    per (sensor, 16x16 node tile): bilinear propagation from every layer
//                  (Sec. 2, NGS shift / LGS cone), Shack-Hartmann slopes, noise weights and
//                  the Shack-Hartmann adjoint, all in LDS -- the slopes never leave the chip
//   k_adj_gather   per layer node: the exact transpose of the bilinear propagation written as
//                  a gather over the sensor nodes touching the node (no atomics, deterministic)
//   k_dwt_level    per level, all layers: periodic db3 analysis (W^-T = DWT / delta_l), the
//                  prior alpha D x fused into the final coefficients
// Solver (Alg. 1, Alg. 2, Alg. 3 residual update): vector kernels on a fixed 512-block grid
// that write per-block FP64 partial inner products, and single-block kernels that reduce
// them in a fixed order and compute every scalar (alpha, beta, mu, the k x k Gram solve)
// on the device.  No float atomics anywhere: results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fewha_internal.h"

namespace fewha {

namespace {

__device__ __forceinline__ int pmod(int a, int m) {
    const int r = a % m;
    return r < 0 ? r + m : r;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Block (256 threads) reduction of NV values; thread 0..NV-1 write part[k * kVecBlocks + block].
template <int NV>
__device__ __forceinline__ void block_partials(const double (&v)[NV], double* __restrict__ part, int slot0) {
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
        part[size_t(slot0 + k) * kVecBlocks + blockIdx.x] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
    }
}

// Same for a run-time count nv <= 2 kKMax + 2.
__device__ __forceinline__ void block_partials_dyn(const double* v, int nv, double* __restrict__ part, int slot0) {
    __shared__ double sh[2 * kKMax + 2][kThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < nv; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) sh[k][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        const int k = threadIdx.x;
        part[size_t(slot0 + k) * kVecBlocks + blockIdx.x] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
    }
}

// Fixed-order sum of one partial slot by a whole block; result valid in every thread.
__device__ double block_total(const double* __restrict__ part, int slot) {
    __shared__ double sh[kThreads / 64];
    __shared__ double res;
    double v = 0;
    for (int b = threadIdx.x; b < kVecBlocks; b += blockDim.x) v += part[size_t(slot) * kVecBlocks + b];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) res = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    const double r = res;
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ wavelet levels (Sec. 3)

// One synthesis level on every layer with at least `lev` levels: the 2m x 2m block from its
// four m x m bands.  1-D periodic synthesis x_i = sum_k a_k h_{(i-2k) mod 2m} + d_k g_{(i-2k) mod 2m}
// applied along y and x (the transpose of the rows-then-columns analysis).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_idwt_level(const LayerDev* __restrict__ lays, int lev, Filt<T> f,
                                                          const T* __restrict__ coef, const T* __restrict__ src,
                                                          T* __restrict__ dst, T* __restrict__ out_final) {
    const LayerDev d = lays[blockIdx.y];
    if (lev > d.levels) return;
    const int n = d.n, nb = n >> (lev - 1), m = nb >> 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nb * nb) return;
    const int y = idx / nb, x = idx - y * nb;
    const T* C = coef + d.off;
    const T* LL = (lev == d.levels) ? C : src + d.off;
    T acc = 0;
    for (int ty = y & 1; ty < 6; ty += 2) {
        const int ky = pmod((y - ty) >> 1, m);
        T lo = 0, hi = 0;
        for (int tx = x & 1; tx < 6; tx += 2) {
            const int kx = pmod((x - tx) >> 1, m);
            lo += f.h[tx] * LL[ky * n + kx] + f.g[tx] * C[ky * n + m + kx];
            hi += f.h[tx] * C[(m + ky) * n + kx] + f.g[tx] * C[(m + ky) * n + m + kx];
        }
        acc += f.h[ty] * lo + f.g[ty] * hi;
    }
    if (lev == 1)
        out_final[d.off + y * n + x] = acc * T(d.inv_delta);
    else
        dst[d.off + y * n + x] = acc;
}

// One analysis level: rows then columns of the current 2m x 2m block,
// a_k = sum_t h_t x_{(2k+t) mod 2m}, d_k = sum_t g_t x_{(2k+t) mod 2m}.  Final coefficients
// are scaled by 1/delta_l and, when xprior is given, receive + (alpha D)_i xprior_i.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_dwt_level(const LayerDev* __restrict__ lays, int lev, Filt<T> f,
                                                         const T* __restrict__ src, T* __restrict__ dst_ll,
                                                         T* __restrict__ out, const T* __restrict__ prior_a,
                                                         const T* __restrict__ xprior) {
    const LayerDev d = lays[blockIdx.y];
    if (lev > d.levels) return;
    const int n = d.n, nb = n >> (lev - 1), m = nb >> 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * m) return;
    const int ky = idx / m, kx = idx - ky * m;
    const T* I = src + d.off;
    T ll = 0, xh = 0, yh = 0, hh = 0;
    for (int ty = 0; ty < 6; ++ty) {
        const int row = (2 * ky + ty) & (nb - 1);
        T rl = 0, rh = 0;
        for (int tx = 0; tx < 6; ++tx) {
            const T v = I[row * n + ((2 * kx + tx) & (nb - 1))];
            rl += f.h[tx] * v;
            rh += f.g[tx] * v;
        }
        ll += f.h[ty] * rl;
        xh += f.h[ty] * rh;
        yh += f.g[ty] * rl;
        hh += f.g[ty] * rh;
    }
    const T s = T(d.inv_delta);
    auto fin = [&](int r, int c, T v) {
        const size_t o = size_t(d.off) + size_t(r) * n + c;
        T val = v * s;
        if (xprior) val += prior_a[o] * xprior[o];
        out[o] = val;
    };
    fin(ky, m + kx, xh);
    fin(m + ky, kx, yh);
    fin(m + ky, m + kx, hh);
    if (lev == d.levels)
        fin(ky, kx, ll);
    else
        dst_ll[d.off + ky * n + kx] = ll;
}

// ------------------------------------------------------------------ tomography (Sec. 2)

__device__ __forceinline__ int find_sensor(const WfsDev* __restrict__ wfs, int G, int tile) {
    int g = 0;
    while (g + 1 < G && wfs[g + 1].tile_off <= tile) ++g;
    return g;
}

// Wavefront of sensor g at node (i, j): sum over layers of the bilinear interpolant.
template <typename T>
__device__ __forceinline__ T wavefront_node(int g, int i, int j, int np, int L, const LayerDev* __restrict__ lays,
                                            const PairDev* __restrict__ pairs, const int32_t* __restrict__ cidx,
                                            const T* __restrict__ frac, const T* __restrict__ phi) {
    T v = 0;
    for (int l = 0; l < L; ++l) {
        const PairDev P = pairs[g * L + l];
        const int n = lays[l].n;
        const int a0 = cidx[P.fwd_off + i], b0 = cidx[P.fwd_off + np + j];
        const T fy = frac[P.fwd_off + i], fx = frac[P.fwd_off + np + j];
        const T* ph = phi + lays[l].off + size_t(a0) * n + b0;
        v += (T(1) - fy) * ((T(1) - fx) * ph[0] + fx * ph[1]) + fy * ((T(1) - fx) * ph[n] + fx * ph[n + 1]);
    }
    return v;
}

// Fused Gamma^T C^-1 Gamma P per sensor tile.  Tile of kTile x kTile output nodes; the
// wavefront is formed on the tile plus a one-node halo, slopes on the (kTile+1)^2
// subapertures touching the tile.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_data_term(const WfsDev* __restrict__ wfs, int G,
                                                         const LayerDev* __restrict__ lays, int L,
                                                         const PairDev* __restrict__ pairs,
                                                         const int32_t* __restrict__ cidx, const T* __restrict__ frac,
                                                         const T* __restrict__ phi, const T* __restrict__ w,
                                                         T* __restrict__ psi) {
    constexpr int E = kTile + 2, S1 = kTile + 1;
    __shared__ T sphi[E * E];
    __shared__ T stx[S1 * S1], sty[S1 * S1];
    const int g = find_sensor(wfs, G, blockIdx.x);
    const WfsDev W = wfs[g];
    const int ns = W.ns, np = ns + 1;
    const int tl = blockIdx.x - W.tile_off;
    const int i0 = (tl / W.tiles_x) * kTile, j0 = (tl % W.tiles_x) * kTile;
    for (int e = threadIdx.x; e < E * E; e += blockDim.x) {
        const int i = i0 - 1 + e / E, j = j0 - 1 + e % E;
        T v = 0;
        if (i >= 0 && i <= ns && j >= 0 && j <= ns) v = wavefront_node(g, i, j, np, L, lays, pairs, cidx, frac, phi);
        sphi[e] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < S1 * S1; e += blockDim.x) {
        const int ls = e / S1, lt = e % S1;
        const int si = i0 - 1 + ls, sj = j0 - 1 + lt;
        T tx = 0, ty = 0;
        if (si >= 0 && si < ns && sj >= 0 && sj < ns) {
            const T p00 = sphi[ls * E + lt], p01 = sphi[ls * E + lt + 1];
            const T p10 = sphi[(ls + 1) * E + lt], p11 = sphi[(ls + 1) * E + lt + 1];
            const T sx = T(0.5) * ((p01 - p00) + (p11 - p10));
            const T sy = T(0.5) * ((p10 - p00) + (p11 - p01));
            tx = w[W.soff + si * ns + sj] * sx;
            ty = w[W.soff + ns * ns + si * ns + sj] * sy;
        }
        stx[e] = tx;
        sty[e] = ty;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
        const int li = e / kTile, lj = e % kTile;
        const int i = i0 + li, j = j0 + lj;
        if (i > ns || j > ns) continue;
        const int A = (li + 1) * S1 + lj + 1, B = (li + 1) * S1 + lj, C = li * S1 + lj + 1, D = li * S1 + lj;
        psi[W.noff + i * np + j] = T(0.5) * ((stx[B] - stx[A]) + (stx[D] - stx[C])) +
                                   T(0.5) * ((sty[C] - sty[A]) + (sty[D] - sty[B]));
    }
}

// Gamma^T (w s) per node (weighted = 1) or Gamma^T (mask s) (weighted = 0, mask = w != 0).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_slopes_adj(const WfsDev* __restrict__ wfs, int G, int64_t V,
                                                          const T* __restrict__ w, const T* __restrict__ s,
                                                          T* __restrict__ psi, int weighted) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= V) return;
    int g = 0;
    while (g + 1 < G && wfs[g + 1].noff <= e) ++g;
    const WfsDev W = wfs[g];
    const int ns = W.ns, np = ns + 1;
    const int loc = int(e - W.noff);
    const int i = loc / np, j = loc % np;
    auto t = [&](int comp, int si, int sj) -> T {
        if (si < 0 || si >= ns || sj < 0 || sj >= ns) return T(0);
        const int64_t o = W.soff + int64_t(comp) * ns * ns + si * ns + sj;
        const T ww = w[o];
        return weighted ? ww * s[o] : (ww != T(0) ? s[o] : T(0));
    };
    psi[e] = T(0.5) * ((t(0, i, j - 1) - t(0, i, j)) + (t(0, i - 1, j - 1) - t(0, i - 1, j))) +
             T(0.5) * ((t(1, i - 1, j) - t(1, i, j)) + (t(1, i - 1, j - 1) - t(1, i, j - 1)));
}

// Gamma P phi per subaperture (operator piece A), zero on inactive subapertures.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_fwd_slopes(const WfsDev* __restrict__ wfs, int G, int64_t S,
                                                          const LayerDev* __restrict__ lays, int L,
                                                          const PairDev* __restrict__ pairs,
                                                          const int32_t* __restrict__ cidx, const T* __restrict__ frac,
                                                          const T* __restrict__ phi, const T* __restrict__ w,
                                                          T* __restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= S) return;
    int g = 0;
    while (g + 1 < G && wfs[g + 1].soff <= e) ++g;
    const WfsDev W = wfs[g];
    const int ns = W.ns, np = ns + 1;
    const int loc = int(e - W.soff);
    const int comp = loc / (ns * ns), q = loc % (ns * ns), i = q / ns, j = q % ns;
    const T p00 = wavefront_node(g, i, j, np, L, lays, pairs, cidx, frac, phi);
    const T p01 = wavefront_node(g, i, j + 1, np, L, lays, pairs, cidx, frac, phi);
    const T p10 = wavefront_node(g, i + 1, j, np, L, lays, pairs, cidx, frac, phi);
    const T p11 = wavefront_node(g, i + 1, j + 1, np, L, lays, pairs, cidx, frac, phi);
    const T v = comp == 0 ? T(0.5) * ((p01 - p00) + (p11 - p10)) : T(0.5) * ((p10 - p00) + (p11 - p01));
    out[e] = w[e] != T(0) ? v : T(0);
}

// sum_g P_g^T psi_g at every layer node, as a gather: node (a, b) of layer l collects the
// sensor nodes whose bilinear cell has (a, b) as a corner, with the same weights as P_g.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_adj_gather(const WfsDev* __restrict__ wfs, int G,
                                                          const LayerDev* __restrict__ lays, int L,
                                                          const PairDev* __restrict__ pairs,
                                                          const int32_t* __restrict__ cidx, const T* __restrict__ frac,
                                                          const int2* __restrict__ rng, const T* __restrict__ psi,
                                                          T* __restrict__ out) {
    const int l = blockIdx.y;
    const LayerDev d = lays[l];
    const int n = d.n;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int a = idx / n, b = idx - a * n;
    T acc = 0;
    for (int g = 0; g < G; ++g) {
        const WfsDev W = wfs[g];
        const int np = W.ns + 1;
        const PairDev P = pairs[g * L + l];
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

// ------------------------------------------------------------------ solver vector kernels

// Partial-slot map (rows of the partials buffer, kVecBlocks columns each).
enum : int { P_RZ = 0, P_BB = 1, P_PQ = 2, P_RR = 3, P_RZ1 = 4, P_PROJ = 8 };

struct SlotList { int32_t s[kKMax]; };

template <typename T>
__global__ void __launch_bounds__(kThreads) k_residual(int64_t N, const T* __restrict__ b, T* __restrict__ b_prev,
                                                        T* __restrict__ r, const T* __restrict__ mc, double* part) {
    // first frame: r = b - M c; later frames: r = (b - b_prev) + r (Alg. 3 residual update).
    double bb = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
        const double bi = double(b[i]);
        if (mc)
            r[i] = T(bi - double(mc[i]));
        else
            r[i] = T((bi - double(b_prev[i])) + double(r[i]));
        b_prev[i] = b[i];
        bb += bi * bi;
    }
    const double v[1] = {bb};
    block_partials<1>(v, part, P_BB);
}

// Gram pass: X_ab = (U_a, Q_b) (a, b < m) and v_a = (U_a, r), staged through LDS in
// chunks of 64 elements; thread t owns dot products t, t+256, ...
template <typename T>
__global__ void __launch_bounds__(kThreads) k_gram(int64_t N, int m, SlotList sl, const T* __restrict__ ring_u,
                                                    const T* __restrict__ ring_q, const T* __restrict__ r,
                                                    double* part) {
    constexpr int CH = 64;
    __shared__ double su[kKMax][CH], sq[kKMax][CH], sr[CH];
    const int ndot = m * m + m;
    double acc[(kKMax * kKMax + kKMax + kThreads - 1) / kThreads];
    constexpr int NA = (kKMax * kKMax + kKMax + kThreads - 1) / kThreads;
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[k] = 0;
    for (int64_t base = int64_t(blockIdx.x) * CH; base < N; base += int64_t(gridDim.x) * CH) {
        const int cnt = int(N - base < CH ? N - base : CH);
        for (int e = threadIdx.x; e < (2 * m + 1) * CH; e += blockDim.x) {
            const int v = e / CH, q = e % CH;
            double val = 0;
            if (q < cnt) {
                if (v < m)
                    val = double(ring_u[size_t(sl.s[v]) * N + base + q]);
                else if (v < 2 * m)
                    val = double(ring_q[size_t(sl.s[v - m]) * N + base + q]);
                else
                    val = double(r[base + q]);
            }
            if (v < m)
                su[v][q] = val;
            else if (v < 2 * m)
                sq[v - m][q] = val;
            else
                sr[q] = val;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int t = threadIdx.x + k * kThreads;
            if (t < ndot) {
                double s = 0;
                if (t < m * m) {
                    const int a = t / m, bq = t % m;
                    for (int q = 0; q < CH; ++q) s += su[a][q] * sq[bq][q];
                } else {
                    const int a = t - m * m;
                    for (int q = 0; q < CH; ++q) s += su[a][q] * sr[q];
                }
                acc[k] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int t = threadIdx.x + k * kThreads;
        if (t < ndot) part[size_t(P_PROJ + t) * kVecBlocks + blockIdx.x] = acc[k];
    }
}

// Galerkin step c += U y, r -= Q y; then z = J^-1 r and partials of (Q_a, z).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_galerkin_apply(int64_t N, int m, SlotList sl,
                                                              const T* __restrict__ ring_u, const T* __restrict__ ring_q,
                                                              const Scalars* __restrict__ sc, T* __restrict__ c,
                                                              T* __restrict__ r, T* __restrict__ z,
                                                              const T* __restrict__ jinv, double* part) {
    double acc[kKMax];
    for (int a = 0; a < m; ++a) acc[a] = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
        double ci = double(c[i]), ri = double(r[i]);
        for (int a = 0; a < m; ++a) {
            const double y = sc->y[a];
            ci += y * double(ring_u[size_t(sl.s[a]) * N + i]);
            ri -= y * double(ring_q[size_t(sl.s[a]) * N + i]);
        }
        c[i] = T(ci);
        const T rt = T(ri);
        r[i] = rt;
        const T zt = jinv[i] * rt;
        z[i] = zt;
        for (int a = 0; a < m; ++a) acc[a] += double(ring_q[size_t(sl.s[a]) * N + i]) * double(zt);
    }
    block_partials_dyn(acc, m, part, P_PROJ);
}

// Initial direction p_0 = z - U y2 (m > 0) or p_0 = J^-1 r (m = 0; z stays untouched);
// partial of (r, p_0) (equal to (r, z_0) of the projected z_0).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_init_dir(int64_t N, int m, SlotList sl, const T* __restrict__ ring_u,
                                                        const Scalars* __restrict__ sc, const T* __restrict__ z,
                                                        const T* __restrict__ r, const T* __restrict__ jinv,
                                                        T* __restrict__ p, double* part) {
    double rz = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
        T pt;
        if (m == 0) {
            pt = jinv[i] * r[i];
        } else {
            double pi = double(z[i]);
            for (int a = 0; a < m; ++a) pi -= sc->y2[a] * double(ring_u[size_t(sl.s[a]) * N + i]);
            pt = T(pi);
        }
        p[i] = pt;
        rz += double(r[i]) * double(pt);
    }
    const double v[1] = {rz};
    block_partials<1>(v, part, P_RZ);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_dot(int64_t N, const T* __restrict__ x, const T* __restrict__ y,
                                                   double* part, int slot) {
    double s = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x)
        s += double(x[i]) * double(y[i]);
    const double v[1] = {s};
    block_partials<1>(v, part, slot);
}

// c += alpha p, r -= alpha q; unless last: z = J^-1 r and partials (r, z), (Q_a, z), (U_a, r)
// over the in-loop projection set; always the partial (r, r).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_update1(int64_t N, int mp, SlotList pl, const T* __restrict__ ring_u,
                                                       const T* __restrict__ ring_q, const Scalars* __restrict__ sc,
                                                       const T* __restrict__ p, const T* __restrict__ q,
                                                       T* __restrict__ c, T* __restrict__ r, T* __restrict__ z,
                                                       const T* __restrict__ jinv, int last, double* part) {
    const double alpha = sc->alpha;
    double acc[2 * kKMax + 2];
    const int nv = last ? 1 : 2 + 2 * mp;
    for (int k = 0; k < nv; ++k) acc[k] = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
        c[i] = T(double(c[i]) + alpha * double(p[i]));
        const T rt = T(double(r[i]) - alpha * double(q[i]));
        r[i] = rt;
        const double rd = double(rt);
        acc[0] += rd * rd;
        if (!last) {
            const T zt = jinv[i] * rt;
            z[i] = zt;
            const double zd = double(zt);
            acc[1] += rd * zd;
            for (int a = 0; a < mp; ++a) {
                acc[2 + a] += double(ring_q[size_t(pl.s[a]) * N + i]) * zd;
                acc[2 + mp + a] += double(ring_u[size_t(pl.s[a]) * N + i]) * rd;
            }
        }
    }
    block_partials_dyn(acc, nv, part, P_RR);
}

// p_next = z - sum_a y3_a U_a + beta p.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_update2(int64_t N, int mp, SlotList pl, const T* __restrict__ ring_u,
                                                       const Scalars* __restrict__ sc, const T* __restrict__ z,
                                                       const T* __restrict__ p, T* __restrict__ pn) {
    const double beta = sc->beta;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
        double v = double(z[i]) + beta * double(p[i]);
        for (int a = 0; a < mp; ++a) v -= sc->y2[a] * double(ring_u[size_t(pl.s[a]) * N + i]);
        pn[i] = T(v);
    }
}

// ------------------------------------------------------------------ single-block scalar kernels

enum : int { ST_GRAM = 0, ST_DIR = 1, ST_RZ = 2, ST_ALPHA = 3, ST_BETA = 4, ST_FINISH = 5 };

__device__ void chol_drop(Scalars* sc, const double* X, int m) {
    // G_ab = X_ab for a <= b (mirrored); upper factor R with G = R^T R, columns processed in
    // order, column j dropped when its pivot is <= 1e-14 max diag G.
    double dmax = 0;
    for (int j = 0; j < m; ++j) dmax = fmax(dmax, X[j * m + j]);
    const double thr = 1e-14 * dmax;
    int dropped = 0;
    for (int i = 0; i < m * m; ++i) sc->R[i] = 0;
    for (int j = 0; j < m; ++j) {
        double d = X[j * m + j];
        for (int i = 0; i < j; ++i) d -= sc->R[i * m + j] * sc->R[i * m + j];
        if (!(d > thr)) {
            sc->keep[j] = 0;
            ++dropped;
            continue;
        }
        sc->keep[j] = 1;
        const double rjj = sqrt(d);
        sc->R[j * m + j] = rjj;
        for (int k = j + 1; k < m; ++k) {
            double s = X[j * m + k];
            for (int i = 0; i < j; ++i) s -= sc->R[i * m + j] * sc->R[i * m + k];
            sc->R[j * m + k] = s / rjj;
        }
    }
    sc->dropped = dropped;
}

__device__ void chol_solve(const Scalars* sc, int m, const double* v, double* y) {
    double t[kKMax];
    for (int j = 0; j < m; ++j) {
        t[j] = 0;
        if (!sc->keep[j]) continue;
        double s = v[j];
        for (int i = 0; i < j; ++i) s -= sc->R[i * m + j] * t[i];
        t[j] = s / sc->R[j * m + j];
    }
    for (int j = m - 1; j >= 0; --j) {
        y[j] = 0;
        if (!sc->keep[j]) continue;
        double s = t[j];
        for (int k = j + 1; k < m; ++k) s -= sc->R[j * m + k] * y[k];
        y[j] = s / sc->R[j * m + j];
    }
}

// stage-dependent reduction + scalar work.  sl: the active recycled slots (oldest first);
// lastslot: slot of the most recent recycled direction; pslot: slot of the current p.
__global__ void __launch_bounds__(kThreads) k_scalars(int stage, int m, int mode, int project_all, SlotList sl,
                                                       int pslot, Scalars* sc, const double* part,
                                                       fewha_solve_info* info, fewha_solve_info* info_user,
                                                       int iters) {
    __shared__ double X[kKMax * kKMax + kKMax];
    if (stage == ST_GRAM || stage == ST_DIR) {
        const int nd = stage == ST_GRAM ? m * m + m : m;
        for (int t = 0; t < nd; ++t) {
            const double s = block_total(part, P_PROJ + t);
            if (threadIdx.x == 0) X[t] = s;
        }
        __syncthreads();
        if (threadIdx.x != 0) return;
        if (stage == ST_GRAM) {
            // X holds (U_a, Q_b) row-major then (U_a, r)
            const double* v = X + m * m;
            if (mode == FEWHA_RECYCLE_PAPER) {
                // sequential sigma_j with the running residual: (r, p_j) = sigma_j g_j + sum_{i<j} sigma_i (q_i, p_j)
                for (int j = 0; j < m; ++j) {
                    double s = v[j];
                    for (int i = 0; i < j; ++i) s -= sc->y[i] * X[j * m + i];
                    sc->y[j] = s / sc->gam[sl.s[j]];
                }
                // keep the Gram for the initial-direction step
                for (int i = 0; i < m * m; ++i) sc->R[i] = X[i];
                sc->dropped = 0;
            } else {
                chol_drop(sc, X, m);
                double y[kKMax];
                chol_solve(sc, m, v, y);
                for (int j = 0; j < m; ++j) sc->y[j] = y[j];
            }
            sc->used = m;
        } else {
            // X holds (Q_a, z)
            if (mode == FEWHA_RECYCLE_PAPER) {
                // sequential tau_j with the running z: (z, q_j) = tau_j g_j + sum_{i<j} tau_i (p_i, q_j)
                for (int j = 0; j < m; ++j) {
                    double s = X[j];
                    for (int i = 0; i < j; ++i) s -= sc->y2[i] * sc->R[i * m + j];
                    sc->y2[j] = s / sc->gam[sl.s[j]];
                }
            } else {
                double y[kKMax];
                chol_solve(sc, m, X, y);
                for (int j = 0; j < m; ++j) sc->y2[j] = y[j];
            }
        }
        return;
    }
    if (stage == ST_RZ) {
        const double rz = block_total(part, P_RZ);
        const double bb = block_total(part, P_BB);
        if (threadIdx.x == 0) {
            sc->rz = rz;
            sc->bb = bb;
            sc->flags = 0;
            if (m == 0) {
                sc->used = 0;
                sc->dropped = 0;
            }
        }
        return;
    }
    if (stage == ST_ALPHA) {
        const double pq = block_total(part, P_PQ);
        if (threadIdx.x == 0) {
            sc->pq = pq;
            sc->gam[pslot] = pq;
            double alpha = sc->rz / pq;
            if (sc->flags || !(pq > 0) || !isfinite(alpha)) {
                sc->flags |= 1;
                alpha = 0;
            }
            sc->alpha = alpha;
        }
        return;
    }
    if (stage == ST_BETA) {
        // m here is the size of the in-loop projection set
        const double rz1 = block_total(part, P_RZ1);
        for (int t = 0; t < 2 * m; ++t) {
            const double s = block_total(part, P_RZ1 + 1 + t);
            if (threadIdx.x == 0) X[t] = s;
        }
        __syncthreads();
        if (threadIdx.x != 0) return;
        // X[0..m): (Q_a, z); X[m..2m): (U_a, r)
        double y3[kKMax];
        if (m == 0) {
        } else if (project_all) {
            chol_solve(sc, m, X, y3);
        } else {
            y3[0] = X[0] / sc->gam[sl.s[0]];
        }
        double rzn = rz1;
        for (int a = 0; a < m; ++a) {
            rzn -= y3[a] * X[m + a];
            sc->y2[a] = y3[a];
        }
        double beta = sc->rz != 0 ? rzn / sc->rz : 0.0;
        if (sc->flags || !isfinite(beta)) {
            sc->flags |= 1;
            beta = 0;
        }
        sc->beta = beta;
        sc->mu = m ? y3[0] : 0.0;
        sc->rz = rzn;
        return;
    }
    if (stage == ST_FINISH) {
        const double rr = block_total(part, P_RR);
        if (threadIdx.x == 0) {
            fewha_solve_info in;
            in.iters = iters;
            in.recycle_used = sc->used;
            in.dropped = sc->dropped;
            in.flags = sc->flags;
            in.rel_res = sc->bb > 0 ? sqrt(rr / sc->bb) : 0.0;
            *info = in;
            if (info_user) *info_user = in;
        }
        return;
    }
}

template <typename T>
Filt<T> make_filt() {
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

// ------------------------------------------------------------------ launchers

template <typename T>
void launch_winv(const Ctx& c, const T* x, T* phi, hipStream_t s) {
    const Filt<T> f = make_filt<T>();
    T* buf[2] = {c.at<T>(c.lay.tmp0), c.at<T>(c.lay.tmp1)};
    for (int lev = c.max_levels; lev >= 1; --lev) {
        const int64_t nb = c.max_n >> (lev - 1);
        dim3 grid(cdiv(nb * nb, kThreads), c.L);
        k_idwt_level<T><<<grid, kThreads, 0, s>>>(c.at<LayerDev>(c.lay.layers), lev, f, x, buf[(lev + 1) & 1],
                                                  buf[lev & 1], phi);
    }
}

template <typename T>
void launch_winvt(const Ctx& c, const T* phi, T* y, const T* xprior, hipStream_t s) {
    const Filt<T> f = make_filt<T>();
    T* buf[2] = {c.at<T>(c.lay.tmp0), c.at<T>(c.lay.tmp1)};
    for (int lev = 1; lev <= c.max_levels; ++lev) {
        const int64_t m = c.max_n >> lev;
        dim3 grid(cdiv(m * m, kThreads), c.L);
        k_dwt_level<T><<<grid, kThreads, 0, s>>>(c.at<LayerDev>(c.lay.layers), lev, f,
                                                 lev == 1 ? phi : buf[(lev - 1) & 1], buf[lev & 1], y,
                                                 c.at<T>(c.lay.prior_a), xprior);
    }
}

template <typename T>
void launch_data_term(const Ctx& c, const T* phi, T* psi_nodes, hipStream_t s) {
    k_data_term<T><<<c.fwd_tiles, kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.G, c.at<LayerDev>(c.lay.layers), c.L,
                                                    c.at<PairDev>(c.lay.pairs), c.at<int32_t>(c.lay.cellidx),
                                                    c.at<T>(c.lay.frac), phi, c.at<T>(c.lay.weight), psi_nodes);
}

template <typename T>
void launch_slopes_adj(const Ctx& c, const T* slopes, T* psi_nodes, int weighted, hipStream_t s) {
    k_slopes_adj<T><<<cdiv(c.V, kThreads), kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.G, c.V, c.at<T>(c.lay.weight),
                                                             slopes, psi_nodes, weighted);
}

template <typename T>
void launch_adj_gather(const Ctx& c, const T* psi_nodes, T* psi_layers, hipStream_t s) {
    dim3 grid(cdiv(int64_t(c.max_n) * c.max_n, kThreads), c.L);
    k_adj_gather<T><<<grid, kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.G, c.at<LayerDev>(c.lay.layers), c.L,
                                              c.at<PairDev>(c.lay.pairs), c.at<int32_t>(c.lay.cellidx),
                                              c.at<T>(c.lay.frac), c.at<int2>(c.lay.ranges), psi_nodes, psi_layers);
}

template <typename T>
void launch_fwd_slopes(const Ctx& c, const T* phi, T* slopes, hipStream_t s) {
    k_fwd_slopes<T><<<cdiv(c.S, kThreads), kThreads, 0, s>>>(c.at<WfsDev>(c.lay.wfs), c.G, c.S,
                                                             c.at<LayerDev>(c.lay.layers), c.L,
                                                             c.at<PairDev>(c.lay.pairs), c.at<int32_t>(c.lay.cellidx),
                                                             c.at<T>(c.lay.frac), phi, c.at<T>(c.lay.weight), slopes);
}

template <typename T>
void launch_apply_M(const Ctx& c, const T* x, T* y, hipStream_t s) {
    T* phi = c.at<T>(c.lay.nodal);
    T* psi_n = c.at<T>(c.lay.psi_nodes);
    T* psi_l = c.at<T>(c.lay.psi_layers);
    launch_winv<T>(c, x, phi, s);
    launch_data_term<T>(c, phi, psi_n, s);
    launch_adj_gather<T>(c, psi_n, psi_l, s);
    launch_winvt<T>(c, psi_l, y, x, s);
}

template <typename T>
void launch_rhs(const Ctx& c, const T* slopes, T* b, hipStream_t s) {
    T* psi_n = c.at<T>(c.lay.psi_nodes);
    T* psi_l = c.at<T>(c.lay.psi_layers);
    launch_slopes_adj<T>(c, slopes, psi_n, 1, s);
    launch_adj_gather<T>(c, psi_n, psi_l, s);
    launch_winvt<T>(c, psi_l, b, static_cast<const T*>(nullptr), s);
}

template <typename T>
void launch_solve_frame(Ctx& c, const T* slopes, T* c_out, fewha_solve_info* info_user, hipStream_t s) {
    const int64_t N = c.N;
    const int K = c.slots;
    T* b = c.at<T>(c.lay.b);
    T* bp = c.at<T>(c.lay.b_prev);
    T* r = c.at<T>(c.lay.r);
    T* z = c.at<T>(c.lay.z);
    T* cv = c.at<T>(c.lay.c);
    T* vx = c.at<T>(c.lay.vx);
    T* U = c.at<T>(c.lay.ring_u);
    T* Q = c.at<T>(c.lay.ring_q);
    const T* jinv = c.at<T>(c.lay.jinv);
    double* part = c.at<double>(c.lay.partials);
    Scalars* sc = c.at<Scalars>(c.lay.scalars);
    fewha_solve_info* info = c.at<fewha_solve_info>(c.lay.info);
    const dim3 vb(kVecBlocks), vt(kThreads);

    // a1: right-hand side
    launch_rhs<T>(c, slopes, b, s);
    // a2: residual
    int m = 0;
    if (c.first) {
        launch_apply_M<T>(c, cv, vx, s);
        k_residual<T><<<vb, vt, 0, s>>>(N, b, bp, r, vx, part);
    } else {
        k_residual<T><<<vb, vt, 0, s>>>(N, b, bp, r, nullptr, part);
        if (c.k > 0) m = c.mode == FEWHA_RECYCLE_PAPER ? std::min(c.last_iters, c.k) : std::min(c.count, c.k);
    }
    SlotList act{};
    for (int j = 0; j < m; ++j) act.s[j] = ((c.head - m + j) % K + K) % K;
    const int lastslot = ((c.head - 1) % K + K) % K;
    // a3 + a4: Galerkin step and initial direction
    T* p0 = U + size_t(c.head) * N;
    if (m > 0) {
        k_gram<T><<<vb, vt, 0, s>>>(N, m, act, U, Q, r, part);
        k_scalars<<<1, vt, 0, s>>>(ST_GRAM, m, c.mode, c.project_all, act, 0, sc, part, info, nullptr, 0);
        k_galerkin_apply<T><<<vb, vt, 0, s>>>(N, m, act, U, Q, sc, cv, r, z, jinv, part);
        k_scalars<<<1, vt, 0, s>>>(ST_DIR, m, c.mode, c.project_all, act, 0, sc, part, info, nullptr, 0);
    }
    k_init_dir<T><<<vb, vt, 0, s>>>(N, m, act, U, sc, z, r, jinv, p0, part);
    k_scalars<<<1, vt, 0, s>>>(ST_RZ, m, c.mode, c.project_all, act, 0, sc, part, info, nullptr, 0);
    // in-loop projection set: all of U (project_all) or the most recent direction
    SlotList pl{};
    int mp = 0;
    if (m > 0) {
        if (c.project_all) {
            pl = act;
            mp = m;
        } else {
            pl.s[0] = lastslot;
            mp = 1;
        }
    }
    // a5 + a6: iterations
    for (int it = 0; it < c.max_iter; ++it) {
        const int ps = (c.head + it) % K;
        T* p = U + size_t(ps) * N;
        T* q = Q + size_t(ps) * N;
        launch_apply_M<T>(c, p, q, s);
        k_dot<T><<<vb, vt, 0, s>>>(N, p, q, part, P_PQ);
        k_scalars<<<1, vt, 0, s>>>(ST_ALPHA, m, c.mode, c.project_all, act, ps, sc, part, info, nullptr, 0);
        const int last = it == c.max_iter - 1;
        k_update1<T><<<vb, vt, 0, s>>>(N, mp, pl, U, Q, sc, p, q, cv, r, z, jinv, last, part);
        if (!last) {
            k_scalars<<<1, vt, 0, s>>>(ST_BETA, mp, c.mode, c.project_all, pl, ps, sc, part, info, nullptr, 0);
            T* pn = U + size_t((c.head + it + 1) % K) * N;
            k_update2<T><<<vb, vt, 0, s>>>(N, mp, pl, U, sc, z, p, pn);
        }
    }
    k_scalars<<<1, vt, 0, s>>>(ST_FINISH, m, c.mode, c.project_all, act, 0, sc, part, info, info_user, c.max_iter);
    if (c_out) (void)hipMemcpyAsync(c_out, cv, sizeof(T) * N, hipMemcpyDeviceToDevice, s);
    // a7: ring bookkeeping (the fixed iteration count makes it host-known)
    c.head = (c.head + c.max_iter) % K;
    c.count = std::min(c.count + c.max_iter, K);
    c.last_iters = c.max_iter;
    c.first = false;
}

#define FEWHA_INSTANTIATE(T)                                                                         \
    template void launch_winv<T>(const Ctx&, const T*, T*, hipStream_t);                            \
    template void launch_winvt<T>(const Ctx&, const T*, T*, const T*, hipStream_t);                 \
    template void launch_data_term<T>(const Ctx&, const T*, T*, hipStream_t);                       \
    template void launch_slopes_adj<T>(const Ctx&, const T*, T*, int, hipStream_t);                 \
    template void launch_adj_gather<T>(const Ctx&, const T*, T*, hipStream_t);                      \
    template void launch_fwd_slopes<T>(const Ctx&, const T*, T*, hipStream_t);                      \
    template void launch_apply_M<T>(const Ctx&, const T*, T*, hipStream_t);                         \
    template void launch_rhs<T>(const Ctx&, const T*, T*, hipStream_t);                             \
    template void launch_solve_frame<T>(Ctx&, const T*, T*, fewha_solve_info*, hipStream_t);

FEWHA_INSTANTIATE(float)
FEWHA_INSTANTIATE(double)

}  // namespace fewha
