// HIP kernels (gfx950 / CDNA4) of the frame update of the augmented wavelet reconstructor:
// Alg. 3 residual update, the Galerkin projection and initial direction of Alg. 2 (Sec. 4.1),
// and the PCG iterations of Alg. 1 / Alg. 2.
//
// Every inner product is reduced in FP64 in two fixed-order stages: each vector workgroup
// writes one partial per inner product; the consumer kernel -- every workgroup of it,
// redundantly -- sums its instance's partials in the same order and derives the scalars it
// needs (alpha, beta, mu, the in-loop projection).  Every workgroup therefore holds
// bit-identical scalars without an extra single-block launch between iterations, and results
// are reproducible run to run.  Workgroup 0 of an instance records its scalars in device
// memory for the next kernels and for the frame statistics.  The frame start's k x k solves
// (Galerkin and initial-direction coefficients) run once per instance in k_gram_solve.
//
// A batch of independent instances runs through the same kernels: a workgroup's instance,
// element range and partial column come from the workgroup table (absent for a single
// instance, where the launch itself defines them).  An instance's workgroup count depends on
// its own size only, so it gets the same bits alone or in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fewha_device.h"
#include "fewha_internal.h"
#include "../../include/fewha_unet.h"

namespace fewha {

namespace {

// Rows of the partial buffer (one column per vector workgroup of the batch).
enum : int { P_RZ = 0, P_BB = 1, P_RR = 2, P_RZ1 = 3, P_PROJ = 4 };

struct SlotList { int32_t s[kKMax]; };

// Work of one vector workgroup (see VecBlk).
struct Seg {
    int64_t off;
    int n, local, nb, inst, col, pq0, npq;
};

__device__ __forceinline__ Seg seg_of(const VecBlk* __restrict__ vb, int64_t N, int npq) {
    if (!vb) return Seg{0, int(N), int(blockIdx.x), int(gridDim.x), 0, int(blockIdx.x), 0, npq};
    const VecBlk v = vb[blockIdx.x];
    return Seg{v.off, v.n, v.local, v.nb, v.inst, v.col, v.pq0, v.npq};
}

// Sums NV rows (row0..row0+nrows-1, nrows <= NV) of the instance's partial columns at once.
template <int NV>
__device__ __forceinline__ void block_row_sums(const double* __restrict__ part, int pstride, const Seg& sg, int row0,
                                               int nrows, double (&out)[NV]) {
    __shared__ double sh[NV][kThreads / 64];
    const int c0 = sg.col - sg.local;
    double v[NV];
    // every load is unconditional (a clamped index, zeroed by a factor): loads behind
    // conditions would each be waited for before the next one is issued
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        v[k] = 0;
        const int kr = k < nrows ? k : 0;
        const double fk = k < nrows ? 1.0 : 0.0;
#pragma unroll
        for (int j = 0; j < kVecBlocksMax / kThreads; ++j) {
            const int b = threadIdx.x + j * kThreads;
            const int bc = b < sg.nb ? b : sg.nb - 1;
            v[k] += part[size_t(row0 + kr) * pstride + c0 + bc] * (b < sg.nb ? fk : 0.0);
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) sh[k][wv] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
    __syncthreads();
}

// Small dense algebra of the recycle space on one wavefront (m <= kKMax = 32, all 64 lanes active).
// This runs once per frame on a single wavefront, where every step of a dependency chain costs
// its full latency (a broadcast, a multiply-add: tens of cycles each), so the forms below are
// chosen for short chains rather than few operations.

// 1 / p for a positive normal p: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - p r), within an ulp or two (a correctly rounded division takes about twice as
// many dependent steps, and each pivot's reciprocal is on the elimination's critical path).
__device__ __forceinline__ double recip(double p) {
    double r = __builtin_amdgcn_rcp(p);
    r = fma(r, fma(-p, r, 1.0), r);
    r = fma(r, fma(-p, r, 1.0), r);
    return r;
}

// The Galerkin system G y = v by Gauss-Jordan elimination in place (G symmetric positive
// semi-definite: pivots in order, no exchanges).  Lane c < m holds column c of G in a[0..m-1],
// lane m the right-hand side v; rows m..MB-1 and the other lanes are zero.  Step j broadcasts
// column j (its row j is the pivot p: G_jj after the earlier steps, the Schur complement, which
// is the square of the Cholesky pivot); row j is divided by p and eliminated from every other
// row, and column j becomes column j of the inverse.  Index j is dropped when p <= thr: its
// step then runs with 1/p replaced by 0, which leaves the other columns as they are and zeroes
// row j and column j.  Lanes c < m end with the columns of G+ (the inverse of G restricted to
// the kept indices, zero rows and columns for the dropped ones) and lane m with y = G+ v.
// Returns the mask of kept indices.  Every step is the same straight-line code (no branch on
// the pivot): one broadcast of a column and two multiply-adds per entry, so the compiler can
// overlap a step's entry updates with the next pivot's reciprocal.
template <int MB>
__device__ __forceinline__ unsigned wave_gauss_jordan(double (&a)[MB], int m, double thr) {
    const int c = threadIdx.x & 63;
    bool mine = false;   // lane c < m: pivot c was kept
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        if (j < m) {
            // column j, read before lane j rewrites it (all at once where the scalar registers
            // hold it, so that the reads overlap the reciprocal)
            constexpr bool HOIST = MB <= 24;
            double f[HOIST ? MB : 1];
            if constexpr (HOIST)
#pragma unroll
                for (int i = 0; i < MB; ++i) f[i] = lane_value(a[i], j);
            const double p = HOIST ? f[j < (HOIST ? MB : 1) ? j : 0] : lane_value(a[j], j);
            const bool kj = p > thr;
            if (c == j) mine = kj;
            const double ip = kj ? recip(p) : 0.0;
            const double nj = c == j ? 0.0 : 1.0;
            const double rj = (c == j ? 1.0 : a[j]) * ip;
#pragma unroll
            for (int i = 0; i < MB; ++i)
                if (i != j) {
                    const double fi = HOIST ? f[i < (HOIST ? MB : 1) ? i : 0] : lane_value(a[i], j);
                    a[i] = a[i] * nj - fi * rj;
                }
            a[j] = rj;
        }
    }
    const unsigned kept = unsigned(__ballot(mine && c < m));
#pragma unroll
    for (int i = 0; i < MB; ++i)
        if ((c < m && !mine) || !((kept >> i) & 1u)) a[i] = 0.0;
    return kept;
}

// Sequential single-vector projections as a triangular solve: x_j = (v_j - sum_{i<j} x_i L(j, i)) / d_j,
// L(j, i) = Mx[j * ldr + i * ldc] (LDS), column-oriented: after x_j, lanes k > j subtract
// x_j L(k, j).  Lane k passes v_k, gets x_k.
__device__ double wave_forward_sub(const double* Mx, int ldr, int ldc, const double* diag, int m, double v) {
    const int k = threadIdx.x & 63;
    const bool on = k < m;
    // a recycled direction with (p, q) = 0 is the zero vector (stored by a frame whose residual
    // was exactly zero): its coefficient is zero.  Lane k holds 1 / d_k (0 for such a direction).
    const double inv = (on && diag[k] > 0) ? 1.0 / diag[k] : 0.0;
    double nx = (on && k > 0) ? Mx[k * ldr] : 0.0;
#pragma unroll 1
    for (int j = 0; j < m; ++j) {
        const double lkj = nx;
        nx = (on && k > j + 1) ? Mx[k * ldr + (j + 1) * ldc] : 0.0;
        const double xj = lane_value(inv != 0.0 ? v * inv : 0.0, j);
        if (k == j) v = xj;
        else if (k > j) v -= xj * lkj;
    }
    return on ? v : 0.0;
}

// ------------------------------------------------------------------ frame start

// First frame: r = b - M c; later frames: r = (b - b_prev) + r (Alg. 3 residual update).
// b_prev = b; partial (b, b).  Block 0 resets the frame's flags.  Every workgroup first sums
// the analysis tiles' partials of (b, b): when that is not finite (non-finite or overflowing
// slopes) the frame is not solved -- r and b_prev keep their values (a first frame sets
// r = b_prev - M c, so that the next residual update gives b - M c) and the frame is flagged
// (bits 0 and 3), so that every later kernel of the frame leaves c and r alone.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_residual(int64_t N, const VecBlk* __restrict__ vb, int pstride,
                                                        const T* __restrict__ b, T* __restrict__ b_prev,
                                                        T* __restrict__ r, const T* __restrict__ mc,
                                                        double* __restrict__ part, Scalars* __restrict__ scs, int m,
                                                        int npq, const double* __restrict__ bb_part,
                                                        int32_t* __restrict__ done) {
    const Seg sg = seg_of(vb, N, npq);
    const double bb_all = block_sum_array(bb_part + sg.pq0, sg.npq);
    const bool bad = !isfinite(bb_all);
    double bb = 0;
    for (int64_t j = int64_t(sg.local) * kThreads + threadIdx.x; j < sg.n; j += int64_t(sg.nb) * kThreads) {
        const int64_t i = sg.off + j;
        if (bad) {
            if (mc) r[i] = T(double(b_prev[i]) - double(mc[i]));
            continue;
        }
        const double bi = double(b[i]);
        if (mc)
            r[i] = T(bi - double(mc[i]));
        else
            r[i] = T((bi - double(b_prev[i])) + double(r[i]));
        b_prev[i] = b[i];
        bb += bi * bi;
    }
    const double v[1] = {bb};
    block_partials<1>(v, part, P_BB, pstride, sg.col);
    if (sg.local == 0 && threadIdx.x == 0) {
        Scalars* sc = scs + sg.inst;
        sc->flags = bad ? (kFlagBreakdown | kFlagBadRhs) : 0;
        sc->used = m;
        sc->dropped = 0;
        sc->conv_iter = 0;
        sc->ws_state = 0;
        if (done) done[sg.inst] = 0;
    }
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Four consecutive elements (16-byte aligned) as doubles times a factor, as vector loads.
__device__ __forceinline__ void load4(const float* p, double (&v)[4], double f) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    v[0] = double(x.x) * f;
    v[1] = double(x.y) * f;
    v[2] = double(x.z) * f;
    v[3] = double(x.w) * f;
}
// Four consecutive elements as loaded (the FP64 conversion comes later, so that the loads of
// a step are all issued before the first one is waited for).
template <typename T>
struct Raw4;
template <>
struct Raw4<float> {
    float4 a;
    __device__ __forceinline__ void load(const float* p) { a = *reinterpret_cast<const float4*>(p); }
    __device__ __forceinline__ void to(double (&v)[4], double f) const {
        v[0] = double(a.x) * f;
        v[1] = double(a.y) * f;
        v[2] = double(a.z) * f;
        v[3] = double(a.w) * f;
    }
};
template <>
struct Raw4<double> {
    double2 a, b;
    __device__ __forceinline__ void load(const double* p) {
        a = reinterpret_cast<const double2*>(p)[0];
        b = reinterpret_cast<const double2*>(p)[1];
    }
    __device__ __forceinline__ void to(double (&v)[4], double f) const {
        v[0] = a.x * f;
        v[1] = a.y * f;
        v[2] = b.x * f;
        v[3] = b.y * f;
    }
};

__device__ __forceinline__ void load4(const double* p, double (&v)[4], double f) {
    const double2 x = reinterpret_cast<const double2*>(p)[0], y = reinterpret_cast<const double2*>(p)[1];
    v[0] = x.x * f;
    v[1] = x.y * f;
    v[2] = y.x * f;
    v[3] = y.y * f;
}

// Gram pass: X_ab = (U_a, Q_b) (a, b < m) and X_{a,m} = (U_a, r), entry e = a (m+1) + b, and
// the same products of J^-1 Q_a: Y_ab = (J^-1 Q_a, Q_b), Y_{a,m} = (J^-1 Q_a, r), entry
// m (m+1) + a (m+1) + b (with them the Galerkin step knows (Q_a, J^-1 r_new) before it runs,
// so it also forms the initial direction).  Dense m x N by N x (m+1) contractions on the FP64
// matrix cores.  Block (x, y) owns the 16x16 tiles y of X and Y over its share of the
// elements; each wavefront feeds v_mfma_f64_16x16x4 with 16 elements per step (lane l:
// row/column l mod 16, elements 4 (l / 16) .. +3; on a diagonal tile the row vector Q_a of Y
// is the lane's own column operand), the four wavefronts' tiles are summed in LDS in a fixed
// order and written as one partial each.
//
// BLK4 (GALERKIN, m <= 11, one tile): only the upper triangles are needed, so the products run
// on v_mfma_f64_4x4x4 instead, which takes its four 4x4 blocks' A and B operands from the same
// lanes as the 16x16 form (lane 16 k + 4 b + i: row or column 4 b + i at depth k) and gives
// block b's entry (i, j) to lane 16 i + 4 b + j.  With B rotated by 4 d lanes within each row of
// 16, block b pairs rows 4 b.. with columns 4 (b + d).., so d = 0 .. ND - 1 (ND = ceil((m + 1) / 4)
// <= 3) covers every block on or above the diagonal: ND instructions of 16 cycles per matrix
// and depth step instead of one of 64.  Only entries on or above the diagonal are written.
template <typename T, bool ONE_TILE, bool BLK4 = false>
__global__ void __launch_bounds__(kGramThreads) k_gram(int64_t N, const GramBlk* __restrict__ gt, int m, SlotList sl,
                                                        const T* __restrict__ U, const T* __restrict__ Q,
                                                        const T* __restrict__ r, const T* __restrict__ jinv,
                                                        double* __restrict__ gpart) {
    static_assert(!BLK4 || ONE_TILE, "the small-block form covers one tile");
    constexpr int NW = kGramThreads / 64;          // wavefronts per workgroup
    __shared__ double sh[NW][256];
    GramBlk g;
    if (gt) {
        g = gt[blockIdx.x];
    } else {
        g.off = 0;
        g.n = int(N);
        g.local = blockIdx.x;
        g.nb = gridDim.x;
        g.gbase = 0;
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tb_count = (m + 1 + 15) / 16;
    const int ta = blockIdx.y / tb_count, tb = blockIdx.y - ta * tb_count;
    const int ar = 16 * ta + (lane & 15), bc = 16 * tb + (lane & 15), kq = lane >> 4;
    // rows / columns outside the tile read a valid vector and are zeroed by a factor (loads
    // behind a condition would each be waited for before the next)
    const T* pa = U + size_t(sl.s[ar < m ? ar : 0]) * N + g.off;
    const T* pb = (bc < m ? Q + size_t(sl.s[bc]) * N : r) + g.off;
    const T* pq = Q + size_t(sl.s[ar < m ? ar : 0]) * N + g.off;   // rows of Y off the diagonal
    const T* pj = jinv + g.off;
    const double ma = ar < m ? 1.0 : 0.0, mb = bc <= m ? 1.0 : 0.0;
    f64x4 c = {0.0, 0.0, 0.0, 0.0}, c2 = {0.0, 0.0, 0.0, 0.0};
    double x4[3] = {0.0, 0.0, 0.0}, y4[3] = {0.0, 0.0, 0.0};   // BLK4: block diagonal d of X and Y
    const int nd = (m + 1 + 3) / 4;
    // one 16-element chunk per step: its three (four) loads issued together; the next chunk's
    // loads are in flight while this one is converted and fed to the matrix cores
    const int64_t step = int64_t(g.nb) * NW * 16;
    const int64_t n = g.n;
    int64_t base = (int64_t(g.local) * NW + wv) * 16;   // n % 16 == 0
    Raw4<T> ra, rb, rj, rq;
    if (base < n) {
        const int64_t e0 = base + 4 * kq;
        ra.load(pa + e0);
        rb.load(pb + e0);
        rj.load(pj + e0);
        if (!ONE_TILE) rq.load(pq + e0);
    }
    while (base < n) {
        const int64_t nx = base + step;
        Raw4<T> na, nb, nj, nq;
        if (nx < n) {
            const int64_t e0 = nx + 4 * kq;
            na.load(pa + e0);
            nb.load(pb + e0);
            nj.load(pj + e0);
            if (!ONE_TILE) nq.load(pq + e0);
        }
        double av[4], bv[4], jq[4];                // jq: J^-1 Q_a, the row operand of Y
        ra.to(av, ma);
        rb.to(bv, mb);
        rj.to(jq, 1.0);
        if (ONE_TILE) {   // m < 16: the only tile is diagonal, Q_a is the lane's column operand
#pragma unroll
            for (int j = 0; j < 4; ++j) jq[j] *= bv[j];
        } else {
            double qa[4];
            rq.to(qa, ma);
#pragma unroll
            for (int j = 0; j < 4; ++j) jq[j] *= qa[j];
        }
        if constexpr (BLK4) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // B of columns 4 (b + d) + j in the lanes of block b: a left rotation by 4 d
                // within each row of 16 (data-parallel row rotate right by 16 - 4 d)
                const double b1 = dpp_f64<0x12C>(bv[j]), b2 = dpp_f64<0x128>(bv[j]);
                x4[0] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[j], bv[j], x4[0], 0, 0, 0);
                y4[0] = __builtin_amdgcn_mfma_f64_4x4x4f64(jq[j], bv[j], y4[0], 0, 0, 0);
                if (nd > 1) {
                    x4[1] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[j], b1, x4[1], 0, 0, 0);
                    y4[1] = __builtin_amdgcn_mfma_f64_4x4x4f64(jq[j], b1, y4[1], 0, 0, 0);
                }
                if (nd > 2) {
                    x4[2] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[j], b2, x4[2], 0, 0, 0);
                    y4[2] = __builtin_amdgcn_mfma_f64_4x4x4f64(jq[j], b2, y4[2], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], bv[j], c, 0, 0, 0);
                c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(jq[j], bv[j], c2, 0, 0, 0);
            }
        }
        ra = na;
        rb = nb;
        rj = nj;
        if (!ONE_TILE) rq = nq;
        base = nx;
    }
    // lane l, register v holds tile entry (row 4 v + l / 16, column l mod 16); the NW tiles are
    // summed by the first 256 threads, one entry each, in a fixed pairwise order
    const int t = threadIdx.x, row = 16 * ta + (t >> 4), col = 16 * tb + (t & 15);
    const bool wr = t < 256 && row < m && col <= m;
    auto tile_sum = [&]() {
        double v[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) v[w] = sh[w][t & 255];
#pragma unroll
        for (int h = NW / 2; h > 0; h >>= 1)
#pragma unroll
            for (int w = 0; w < h; ++w) v[w] = v[w] + v[w + h];
        return v[0];
    };
    if constexpr (BLK4) {
        // lane 16 i + 4 b + j holds entry (4 b + i, 4 ((b + d) & 3) + j) of diagonal d; entries no
        // diagonal covers stay zero (and only those on or above the diagonal are written)
        const int bi = (lane & 15) >> 2, ei = 4 * bi + (lane >> 4);
        const bool wu = wr && row <= col;
        auto put = [&](const double (&acc)[3]) {
#pragma unroll
            for (int v = 0; v < 4; ++v) sh[wv][v * 64 + lane] = 0.0;
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (d < nd) sh[wv][ei * 16 + 4 * ((bi + d) & 3) + (lane & 3)] = acc[d];
        };
        put(x4);
        __syncthreads();
        if (wu) gpart[size_t(g.gbase) + size_t(row * (m + 1) + col) * g.nb + g.local] = tile_sum();
        __syncthreads();
        put(y4);
        __syncthreads();
        if (wu) gpart[size_t(g.gbase) + size_t(m * (m + 1) + row * (m + 1) + col) * g.nb + g.local] = tile_sum();
        return;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sh[wv][(4 * v + (lane >> 4)) * 16 + (lane & 15)] = c[v];
    __syncthreads();
    if (wr) gpart[size_t(g.gbase) + size_t(row * (m + 1) + col) * g.nb + g.local] = tile_sum();
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) sh[wv][(4 * v + (lane >> 4)) * 16 + (lane & 15)] = c2[v];
    __syncthreads();
    if (wr) gpart[size_t(g.gbase) + size_t(m * (m + 1) + row * (m + 1) + col) * g.nb + g.local] = tile_sum();
}

// Sums of the Gram partials of one instance: entry e (< ne) of X is the sum of its ngb
// block partials gp[e * ngb + j].  A row of 16 lanes takes one entry (each load of a wavefront
// reads four 128-byte runs, one per row); wavefront wv takes 4 EB consecutive entries per pass,
// entry e0 + 4 b + row.  Lane c of a row adds the partials j = c + 16 q in increasing j, QB of
// them per round; the row's 16 sums are then added by DPP row shifts (lane 15 of the row ends
// with the entry's sum).  Loads outside the partials are clamped and their values dropped.
// emap (LDS, may be NULL): the t-th entry reduced is emap[t] (ne entries in the map).
template <int EB, int QB>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ gp, int ngb, int ne, int wv, int lane,
                                                double* __restrict__ X, const int16_t* __restrict__ emap) {
    constexpr int NWS = kSolveThreads / 64;
    const int row = lane >> 4, c = lane & 15;
    for (int e0 = wv * 4 * EB; e0 < ne; e0 += NWS * 4 * EB) {
        int ent[EB];
#pragma unroll
        for (int b = 0; b < EB; ++b) {
            const int t = e0 + 4 * b + row;
            ent[b] = emap ? emap[t < ne ? t : 0] : t;
        }
        double s[EB];
#pragma unroll
        for (int b = 0; b < EB; ++b) s[b] = 0.0;
        for (int j0 = 0; j0 < ngb; j0 += 16 * QB) {
            double v[EB][QB];
#pragma unroll
            for (int b = 0; b < EB; ++b)
#pragma unroll
                for (int q = 0; q < QB; ++q) {
                    const int j = j0 + 16 * q + c;
                    const bool ok = e0 + 4 * b + row < ne && j < ngb;
                    v[b][q] = gp[ok ? size_t(ent[b]) * ngb + j : 0];
                }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int b = 0; b < EB; ++b)
#pragma unroll
                for (int q = 0; q < QB; ++q)
                    s[b] += (e0 + 4 * b + row < ne && j0 + 16 * q + c < ngb) ? v[b][q] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < EB; ++b) s[b] += dpp_row_shr<0x111>(s[b]);
#pragma unroll
        for (int b = 0; b < EB; ++b) s[b] += dpp_row_shr<0x112>(s[b]);
#pragma unroll
        for (int b = 0; b < EB; ++b) s[b] += dpp_row_shr<0x114>(s[b]);
#pragma unroll
        for (int b = 0; b < EB; ++b) s[b] += dpp_row_shr<0x118>(s[b]);
        if (c == 15) {
#pragma unroll
            for (int b = 0; b < EB; ++b)
                if (e0 + 4 * b + row < ne) X[ent[b]] = s[b];
        }
    }
}

// Reduce the Gram partials and solve for the Galerkin coefficients y (Sec. 4.1).
// GALERKIN: G_ab = X_ab (a <= b, mirrored), eliminated in order, index j dropped when its pivot
// is <= 1e-14 max diag G; y = G^-1 U^T r.  MB: m rounded up to the register blocking.
// PAPER: sequential sigma_j with the running residual, (r, p_j) = sigma_j g_j +
// sum_{i<j} sigma_i (q_i, p_j); X is kept for the initial-direction step.
template <int MB>
__global__ void __launch_bounds__(kSolveThreads) k_gram_solve(int m, int mode, SlotList sl,
                                                               Scalars* __restrict__ scs,
                                                               const InstDev* __restrict__ insts, int ke,
                                                               const double* __restrict__ gpart, int tol_mode) {
    __shared__ double X[2 * kKMax * (kKMax + 1)];     // X, then Y (see k_gram)
    __shared__ double gm[kKMax];
    const InstDev I = insts[blockIdx.x];               // one workgroup per instance
    Scalars* __restrict__ sc = scs + blockIdx.x;
    // the (p, q) of the recycled directions, requested first: their latency overlaps the
    // partial sums
    const double gam = threadIdx.x < m ? sc->gam[sl.s[threadIdx.x]] : 0.0;
    const double* __restrict__ gp = gpart + size_t(I.gb0) * ke;
    const int ngb = I.ngb;
    const int W = m + 1;
    // GALERKIN uses the upper triangles of X and Y with their r column (both matrices are
    // symmetric in their first m columns): only those m (m + 3) entries are reduced, and the
    // lower triangles are read through the upper ones.  PAPER reads both triangles of X.
    __shared__ int16_t emap[kKMax * (kKMax + 3)];
    const bool upper = mode != FEWHA_RECYCLE_PAPER;
    const int nh = m * (m + 3) / 2;
    const int ne = upper ? 2 * nh : 2 * m * W;
    if (upper) {
        for (int t = threadIdx.x; t < 2 * nh; t += kSolveThreads) {
            const int half = t >= nh ? 1 : 0;
            int rem = t - half * nh, a = 0;
            while (rem >= W - a) {   // row a holds columns a .. m
                rem -= W - a;
                ++a;
            }
            emap[t] = int16_t(half * m * W + a * W + a + rem);
        }
        __syncthreads();
    }
    {   // 32 loads per lane requested at once (16 where there are at most 16 partials)
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int16_t* em = upper ? emap : nullptr;
        if (ngb <= 16) reduce_partials<16, 1>(gp, ngb, ne, wv, lane, X, em);
        else if (ngb <= 64) reduce_partials<8, 4>(gp, ngb, ne, wv, lane, X, em);
        else reduce_partials<4, 8>(gp, ngb, ne, wv, lane, X, em);
    }
    if (threadIdx.x < m) gm[threadIdx.x] = gam;
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int k = threadIdx.x;
    // tolerance mode: only the last `avail` slots of the window hold this instance's real
    // directions (an instance that stopped early has fewer); the others are made zero rows and
    // columns, which both variants skip (zero pivot / zero (p, q)), and are not reported
    const int hide = tol_mode ? m - min(m, sc->avail) : 0;
    if (hide > 0) {
        for (int e = k; e < 2 * m * W; e += 64) {
            const int row = (e % (m * W)) / W, col = e % W;
            if (row < hide || col < hide) X[e] = 0.0;
        }
        if (k < hide) gm[k] = 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    }
    const double v = k < m ? X[k * W + m] : 0.0;   // (U_k, r)
    // entry (a, b) of the upper-triangle store (GALERKIN), for lanes k < m
    auto sym = [&](const double* M, int a, int b) { return M[min(a, b) * W + max(a, b)]; };
    // Initial direction (condition 1 of Alg. 2): its coefficients solve the same system with
    // the right-hand side (Q_k, z), z = J^-1 r_new, r_new = r - Q y, that is
    // w_k = (J^-1 Q_k, r) - sum_b (J^-1 Q_k, Q_b) y_b, accumulated from its first term
    const double* Y = X + m * W;
    double w = k < m ? Y[k * W + m] : 0.0;
    double y, y2, a[MB];
    if (mode == FEWHA_RECYCLE_PAPER) {
        // (r, p_j) = sigma_j g_j + sum_{i<j} sigma_i (q_i, p_j),  (q_i, p_j) = X[j][i]
        y = wave_forward_sub(X, W, 1, gm, m, v);
        if (k < m)
            for (int b = 0; b < m; ++b) sc->R[k * m + b] = X[k * W + b];
        if (k == 0) sc->dropped = 0;
    } else {
#pragma unroll
        for (int i = 0; i < MB; ++i)
            a[i] = i >= m ? 0.0 : k < m ? sym(X, i, k) : k == m ? X[i * W + m] : 0.0;
        double dmax = k < m ? X[k * W + k] : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
        // rows k of G and Y, read before the elimination so that their LDS latency is hidden
        // there (at most 16 entries each: more would not stay in registers beside the columns)
        constexpr bool PRE = MB <= 16;
        constexpr int YB = PRE ? MB : 1;
        double grow[YB], yrow[YB];
#pragma unroll
        for (int i = 0; i < YB; ++i) {
            grow[i] = (PRE && i < m && k < m) ? sym(X, k, i) : 0.0;
            yrow[i] = (PRE && i < m && k < m) ? sym(Y, k, i) : 0.0;
        }
        auto g_ki = [&](int i) { return PRE ? grow[i < YB ? i : 0] : ((i < m && k < m) ? sym(X, k, i) : 0.0); };
        auto y_ki = [&](int i) { return PRE ? yrow[i < YB ? i : 0] : ((i < m && k < m) ? sym(Y, k, i) : 0.0); };
        const unsigned kept = wave_gauss_jordan<MB>(a, m, 1e-14 * dmax);
        const bool kk = k < m && ((kept >> k) & 1u);
        // One step of iterative refinement (residual in FP64, correction through G+) for each of
        // the two solves: a product with the explicit inverse alone carries the inverse's
        // rounding error times the condition number, where the solve it replaces does not.
        // x <- x + G+ (rhs - G x), on the kept indices (G+ is zero on the others).
        auto refine = [&](double x, double rhs) {
            double res = rhs;
#pragma unroll
            for (int i = 0; i < MB; ++i)
                if (i < m) res -= g_ki(i) * lane_value(x, i);
            res = kk ? res : 0.0;
            double dx = 0.0;
#pragma unroll
            for (int i = 0; i < MB; ++i)
                if (i < m) dx += a[i] * lane_value(res, i);
            return kk ? x + dx : x;
        };
        // y from lane m to every lane; G+ (symmetric: lane k's column is its row k) to the
        // scalars for the in-loop projections
        y = 0.0;
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const double yi = lane_value(a[i], m);
            if (i == k) y = yi;
        }
        y = refine(y, v);
#pragma unroll
        for (int i = 0; i < MB; ++i)
            if (i < m) w -= y_ki(i) * lane_value(y, i);
        // y2 = G+ w, row k of G+ being lane k's column, then refined as y was
        y2 = 0.0;
#pragma unroll
        for (int i = 0; i < MB; ++i)
            if (i < m) y2 += a[i] * lane_value(w, i);
        y2 = refine(y2, w);
        if (k < m)
#pragma unroll
            for (int i = 0; i < MB; ++i)
                if (i < m) sc->R[i * m + k] = a[i];
        if (k < m) sc->keep[k] = (kept >> k) & 1u;
        if (k == 0) sc->dropped = (m - __builtin_popcount(kept)) - hide;
    }
    if (k < m) sc->y[k] = y;
    if (k == 0) sc->used = m - hide;
    if (mode == FEWHA_RECYCLE_PAPER) {
#pragma unroll 1
        for (int b = 0; b < m; ++b) w -= (k < m ? Y[k * W + b] : 0.0) * lane_value(y, b);
        // (z, q_j) = tau_j g_j + sum_{i<j} tau_i (p_i, q_j),  (p_i, q_j) = X[i][j]
        y2 = wave_forward_sub(X, 1, W, gm, m, w);
    }
    if (k < m) sc->y2[k] = y2;
    // a non-finite projection coefficient is a breakdown: the Galerkin pass then leaves the frame
    if (__any(k < m && !(isfinite(y) && isfinite(y2))) && k == 0) sc->flags |= kFlagBreakdown;
}

// Galerkin step and initial direction in one pass (Sec. 4.1, Alg. 2): c += U y, r -= Q y,
// z = J^-1 r, p_0 = z - U y_2 with y and y_2 from the Gram solve; partial (r, p_0).
template <typename T, int MB>
__global__ void __launch_bounds__(kThreads) k_galerkin_apply(int64_t N, const VecBlk* __restrict__ vb, int pstride,
                                                              int m, SlotList sl, const T* __restrict__ U,
                                                              const T* __restrict__ Q, const Scalars* __restrict__ scs,
                                                              T* __restrict__ c, T* __restrict__ r, T* __restrict__ p,
                                                              const T* __restrict__ jinv, double* __restrict__ part) {
    const Seg sg = seg_of(vb, N, 0);
    const Scalars* __restrict__ sc = scs + sg.inst;
    if (sc->flags != 0) {   // broken frame: c and r stay, the direction is the zero vector
        for (int64_t j = int64_t(sg.local) * kThreads + threadIdx.x; j < sg.n; j += int64_t(sg.nb) * kThreads)
            p[sg.off + j] = T(0);
        const double vz[1] = {0.0};
        block_partials<1>(vz, part, P_RZ, pstride, sg.col);
        return;
    }
    // slots a >= m of the list repeat slot 0 with coefficient 0 (unconditional loads)
    double y[MB], y2[MB];
#pragma unroll
    for (int a = 0; a < MB; ++a) {
        y[a] = sc->y[a] * (a < m ? 1.0 : 0.0);
        y2[a] = sc->y2[a] * (a < m ? 1.0 : 0.0);
    }
    double rz = 0;
    for (int64_t j = int64_t(sg.local) * kThreads + threadIdx.x; j < sg.n; j += int64_t(sg.nb) * kThreads) {
        const int64_t i = sg.off + j;
        double ci = double(c[i]), ri = double(r[i]);
        double uv[MB];
#pragma unroll
        for (int a = 0; a < MB; ++a) {
            uv[a] = double(U[size_t(sl.s[a]) * N + i]);
            ci += y[a] * uv[a];
            ri -= y[a] * double(Q[size_t(sl.s[a]) * N + i]);
        }
        c[i] = T(ci);
        const T rt = T(ri);
        r[i] = rt;
        double pi = double(jinv[i] * rt);
#pragma unroll
        for (int a = 0; a < MB; ++a) pi -= y2[a] * uv[a];
        const T pt = T(pi);
        p[i] = pt;
        rz += double(rt) * double(pt);
    }
    const double vv[1] = {rz};
    block_partials<1>(vv, part, P_RZ, pstride, sg.col);
}

// Without recycled directions p_0 = z = J^-1 r (Alg. 1).  Partial of (r, p_0).  (With them the
// Galerkin kernel above forms p_0.)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_init_dir(int64_t N, const VecBlk* __restrict__ vb, int pstride,
                                                        const T* __restrict__ r, const T* __restrict__ jinv,
                                                        T* __restrict__ p, double* __restrict__ part,
                                                        const Scalars* __restrict__ scs) {
    const Seg sg = seg_of(vb, N, 0);
    const T on = scs[sg.inst].flags != 0 ? T(0) : T(1);   // broken frame: the zero direction
    double rz = 0;
    for (int64_t j = int64_t(sg.local) * kThreads + threadIdx.x; j < sg.n; j += int64_t(sg.nb) * kThreads) {
        const int64_t i = sg.off + j;
        const T pt = on * jinv[i] * r[i];
        p[i] = pt;
        rz += double(r[i]) * double(pt);
    }
    const double vv[1] = {rz};
    block_partials<1>(vv, part, P_RZ, pstride, sg.col);
}

// ------------------------------------------------------------------ PCG iteration

// alpha = (r, z) / (p, q) from the analysis partials of (p, q) = (p, Mp) and the (r, z) of
// this iteration; c += alpha p, r -= alpha q; unless last: z = J^-1 r with partials of (r, z)
// and, over the in-loop projection set, (Q_a, z) and (U_a, r); always the partial (r, r).
// Breakdown (a non-finite value, or (p, q) <= 0 with (r, z) != 0; or a flag from earlier in
// the frame): c and r keep their values, and this iteration's ring slot (p, q) and z become
// zero vectors with (p, q) = 0, so that later projections give them no weight.
template <typename T, int MP>
__global__ void __launch_bounds__(kThreads) k_update1(int64_t N, const VecBlk* __restrict__ vb, int pstride, int it,
                                                       int mp, SlotList pl, const T* __restrict__ U,
                                                       const T* __restrict__ Q, Scalars* __restrict__ scs,
                                                       T* __restrict__ p, T* __restrict__ q,
                                                       T* __restrict__ c, T* __restrict__ r, T* __restrict__ z,
                                                       const T* __restrict__ jinv, int last, int npq,
                                                       const double* __restrict__ pq_part, double* __restrict__ part,
                                                       int pslot, const int32_t* __restrict__ skip) {
    const Seg sg = seg_of(vb, N, npq);
    if (skip && skip[sg.inst]) return;   // tolerance mode: the instance has stopped
    Scalars* __restrict__ sc = scs + sg.inst;
    constexpr int MP1 = MP > 0 ? MP : 1;
    // UN elements per step with every operand requested first (clamped indices, so that no
    // load waits behind a condition); the first step's are requested before the sums of the
    // (p, q) and (r, z) partials below, so that their latencies overlap.  Elements are visited,
    // and summed, in increasing j as one at a time.
    constexpr int UN = 2;
    const int64_t stride = int64_t(sg.nb) * kThreads;
    const int64_t j0 = int64_t(sg.local) * kThreads + threadIdx.x;
    T cv[UN], pv[UN], rv[UN], qv[UN], jv[UN], Qv[UN][MP1], Uv[UN][MP1];
    auto fetch = [&](int64_t jb) {
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int64_t jj = jb + u * stride;
            const int64_t i = sg.off + (jj < sg.n ? jj : int64_t(sg.n) - 1);
            cv[u] = c[i];
            pv[u] = p[i];
            rv[u] = r[i];
            qv[u] = q[i];
            jv[u] = T(0);
#pragma unroll
            for (int a = 0; a < MP1; ++a) Qv[u][a] = Uv[u][a] = T(0);
            if (!last) {
                jv[u] = jinv[i];
#pragma unroll
                for (int a = 0; a < MP; ++a) {
                    Qv[u][a] = Q[size_t(pl.s[a]) * N + i];
                    Uv[u][a] = U[size_t(pl.s[a]) * N + i];
                }
            }
        }
    };
    fetch(j0);
    const double pq = block_sum_array(pq_part + sg.pq0, sg.npq);
    double rz;
    if (it == 0) {
        double t[1];
        block_row_sums<1>(part, pstride, sg, P_RZ, 1, t);
        rz = t[0];
    } else {
        rz = sc->rzb[it & 1];
    }
    // (p, q) = 0 with (r, z) = 0 is exact convergence (a zero residual), not a breakdown
    const bool ok = isfinite(pq) && isfinite(rz) && (pq > 0 ? isfinite(rz / pq) : (pq == 0 && rz == 0));
    const bool broken = sc->flags != 0 || !ok;
    const double alpha = !broken && pq > 0 ? rz / pq : 0.0;
    if (sg.local == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->gam[pslot] = broken ? 0.0 : pq;
        sc->alpha = alpha;
        if (it == 0) sc->rzb[0] = rz;
        if (broken) sc->flags |= kFlagBreakdown;
    }
    constexpr int NV = 2 + 2 * MP;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0;
    // one element: the update and its partial-sum terms, from loaded operands
    auto element = [&](int64_t i, T cv, T pv, T rv, T qv, T jv, const T* Qv, const T* Uv) {
        if (broken) {   // keep c and r; the slot and z become zero vectors
            const double rd = double(rv);
            acc[0] += rd * rd;
            p[i] = T(0);
            q[i] = T(0);
            if (!last) z[i] = T(0);
            return;
        }
        c[i] = T(double(cv) + alpha * double(pv));
        const T rt = T(double(rv) - alpha * double(qv));
        r[i] = rt;
        const double rd = double(rt);
        acc[0] += rd * rd;
        if (!last) {
            const T zt = jv * rt;
            z[i] = zt;
            const double zd = double(zt);
            acc[1] += rd * zd;
#pragma unroll
            for (int a = 0; a < MP; ++a) {   // slots a >= mp repeat slot 0; their sums are unused
                acc[2 + a] += double(Qv[a]) * zd;
                acc[2 + MP + a] += double(Uv[a]) * rd;
            }
        }
    };
    for (int64_t jb = j0; jb < sg.n; jb += UN * stride) {
        T c0[UN], p0[UN], r0[UN], q0[UN], jz[UN], Q0[UN][MP1], U0[UN][MP1];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            c0[u] = cv[u];
            p0[u] = pv[u];
            r0[u] = rv[u];
            q0[u] = qv[u];
            jz[u] = jv[u];
#pragma unroll
            for (int a = 0; a < MP1; ++a) {
                Q0[u][a] = Qv[u][a];
                U0[u][a] = Uv[u][a];
            }
        }
        if (jb + UN * stride < sg.n) fetch(jb + UN * stride);   // the next step's operands in flight
#pragma unroll
        for (int u = 0; u < UN; ++u)
            if (jb + u * stride < sg.n) element(sg.off + jb + u * stride, c0[u], p0[u], r0[u], q0[u], jz[u], Q0[u], U0[u]);
    }
    __shared__ double sh[NV][kThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) sh[k][wv] = s;
    }
    __syncthreads();
    // rows: P_RR, P_RZ1, P_PROJ + a (Q_a, z), P_PROJ + MP + a (U_a, r)
    const int k = threadIdx.x;
    if (k < (last ? 1 : NV)) {
        const int row = k == 0 ? P_RR : (k == 1 ? P_RZ1 : P_PROJ + (k - 2));
        part[size_t(row) * pstride + sg.col] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
    }
}

// Projection coefficients y3 of the new z against the in-loop set (the most recent recycled
// direction: mu = (z, q_m) / (p_m, q_m); or all of U through the Gram factor), the projected
// (r, z) = (r, z) - sum_a y3_a (U_a, r) and beta; p_next = z - U y3 + beta p.
template <typename T, int MP>
__global__ void __launch_bounds__(kThreads) k_update2(int64_t N, const VecBlk* __restrict__ vb, int pstride, int it,
                                                       int mp, int project_all, SlotList pl, const T* __restrict__ U,
                                                       Scalars* __restrict__ scs, const T* __restrict__ z,
                                                       const T* __restrict__ p, T* __restrict__ pn,
                                                       const double* __restrict__ part, double tol,
                                                       int32_t* __restrict__ done) {
    constexpr int NV = 1 + 2 * MP;
    constexpr int MP1 = MP > 0 ? MP : 1;
    const Seg sg = seg_of(vb, N, 0);
    if (done && done[sg.inst]) return;   // tolerance mode: the instance has stopped
    // four elements per step with every operand requested first (clamped indices); the first
    // step's are requested before the partial sums below, so that their latencies overlap
    const int64_t stride = int64_t(sg.nb) * kThreads;
    const int64_t j0 = int64_t(sg.local) * kThreads + threadIdx.x;
    T zv[4], pv[4], uv[4][MP1];
    auto fetch = [&](int64_t jb) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t jj = jb + u * stride;
            const int64_t i = sg.off + (jj < sg.n ? jj : int64_t(sg.n) - 1);
            zv[u] = z[i];
            pv[u] = p[i];
#pragma unroll
            for (int a = 0; a < MP1; ++a) uv[u][a] = a < MP ? U[size_t(pl.s[a]) * N + i] : T(0);
        }
    };
    fetch(j0);
    Scalars* __restrict__ sc = scs + sg.inst;
    if (tol > 0) {
        // tolerance mode: ||r|| <= tol ||b|| after this iteration's update (FP64, from the
        // partials of (b, b) and (r, r)) stops the instance: no next direction, and every
        // kernel of the instance returns at once for the rest of the frame
        double w[2];
        block_row_sums<2>(part, pstride, sg, P_BB, 2, w);   // rows P_BB, P_RR
        if (sqrt(w[1]) <= tol * sqrt(w[0])) {
            if (sg.local == 0 && threadIdx.x == 0) {
                sc->conv_iter = it + 1;
                done[sg.inst] = 1;
            }
            return;
        }
    }
    __shared__ double sy[MP1];
    __shared__ double sbeta;
    __shared__ bool sbroken;
    double v[NV];
    block_row_sums<NV>(part, pstride, sg, P_RZ1, NV, v);   // (r,z), (Q_a,z) a < MP, (U_a,r) a < MP (entries a >= mp unused)
    __shared__ double y3[MP1];
    if (threadIdx.x < 64) {
        const int k = threadIdx.x;
        if constexpr (MP > 0) {
            if (project_all) {
                // y3 = G+ (U^T r) with G+ from the Gram solve (zero rows and columns for the
                // dropped directions); lane k takes row k
                if (k < mp) {
                    double yk = 0;
#pragma unroll
                    for (int a = 0; a < MP; ++a) {
                        const double g = sc->R[k * mp + (a < mp ? a : 0)];   // loads not behind a condition
                        if (a < mp) yk += g * v[1 + a];
                    }
                    y3[k] = yk;
                }
            } else if (k == 0) {
                const double g = sc->gam[pl.s[0]];
                y3[0] = g > 0 ? v[1] / g : 0.0;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double rzn = v[0];
#pragma unroll
        for (int a = 0; a < MP; ++a)
            if (a < mp) rzn -= y3[a] * v[1 + MP + a];
        const double rz_old = sc->rzb[it & 1];
        double beta = rz_old > 0 ? rzn / rz_old : 0.0;
        bool broken = sc->flags != 0 || !isfinite(beta);
        for (int a = 0; a < mp; ++a) broken = broken || !isfinite(y3[a]);
        if (broken) {
            beta = 0;
            for (int a = 0; a < mp; ++a) y3[a] = 0;
        }
        for (int a = 0; a < mp; ++a) sy[a] = y3[a];
        sbeta = beta;
        sbroken = broken;
        if (sg.local == 0) {
            sc->rzb[(it + 1) & 1] = rzn;
            sc->beta = beta;
            sc->mu = mp ? y3[0] : 0.0;
            if (broken) sc->flags |= kFlagBreakdown;
        }
    }
    __syncthreads();
    const double beta = sbeta;
    if (sbroken) {   // broken frame: the next direction is the zero vector
        for (int64_t j = int64_t(sg.local) * kThreads + threadIdx.x; j < sg.n; j += int64_t(sg.nb) * kThreads)
            pn[sg.off + j] = T(0);
        return;
    }
    double yr[MP1];
#pragma unroll
    for (int a = 0; a < MP; ++a) yr[a] = a < mp ? sy[a] : 0.0;
    for (int64_t jb = j0; jb < sg.n; jb += 4 * stride) {
        T z0[4], p0[4], u0[4][MP1];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            z0[u] = zv[u];
            p0[u] = pv[u];
#pragma unroll
            for (int a = 0; a < MP1; ++a) u0[u][a] = uv[u][a];
        }
        if (jb + 4 * stride < sg.n) fetch(jb + 4 * stride);   // the next step's operands in flight
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (jb + u * stride < sg.n) {
                double vv = double(z0[u]) + beta * double(p0[u]);
#pragma unroll
                for (int a = 0; a < MP; ++a) vv -= yr[a] * double(u0[u][a]);   // yr = 0 beyond mp
                pn[sg.off + jb + u * stride] = T(vv);
            }
        }
    }
}

// Frame statistics (relative residual in FP64) of every instance (one workgroup each) into
// the context's and the caller's info.  Tolerance mode: iters is the instance's first
// iteration that met the tolerance (flag bit 1: not met within the frame).  A frame whose
// right-hand side was not finite reports a NaN relative residual.  A broken-down instance
// writes the frame's number into the host-visible breakdown word.
__device__ __forceinline__ void finish_instance(int b, Scalars* __restrict__ scs, const InstDev* __restrict__ insts,
                                                int pstride, const double* __restrict__ part,
                                                fewha_solve_info* __restrict__ infos,
                                                fewha_solve_info* __restrict__ infos_user, int iters, double tol,
                                                int64_t* __restrict__ brk) {
    const bool tol_mode = tol > 0;
    const InstDev I = insts[b];
    const Seg sg{I.off, int(I.n), 0, I.nvb, b, I.vb0, I.pq0, I.npq};
    Scalars* __restrict__ sc = scs + b;
    fewha_solve_info* info = infos + b;
    fewha_solve_info* info_user = infos_user ? infos_user + b : nullptr;
    double v[2];
    block_row_sums<2>(part, pstride, sg, P_BB, 2, v);   // rows P_BB, P_RR
    if (threadIdx.x == 0) {
        fewha_solve_info in;
        const int32_t fl = sc->flags;
        // the last iteration has no next-direction kernel: its crossing is found here
        if (tol_mode && sc->conv_iter == 0 && !(fl & kFlagBreakdown) && sqrt(v[1]) <= tol * sqrt(v[0]))
            sc->conv_iter = iters;
        in.iters = tol_mode && sc->conv_iter ? sc->conv_iter : iters;
        in.recycle_used = sc->used;
        in.dropped = sc->dropped;
        in.flags = fl | (tol_mode && !sc->conv_iter ? kFlagTolUnmet : 0) | (sc->ws_state == 2 ? kFlagWsRejected : 0);
        in.rel_res = (fl & kFlagBadRhs) ? __builtin_nan("") : (v[0] > 0 ? sqrt(v[1] / v[0]) : 0.0);
        sc->bb = v[0];
        sc->rr = v[1];
        const int64_t fno = sc->frame_no + 1;
        sc->frame_no = fno;
        *info = in;
        if (info_user) *info_user = in;
        if (brk && (fl & kFlagBreakdown)) *reinterpret_cast<volatile int64_t*>(brk) = fno;
    }
}

__global__ void __launch_bounds__(kThreads) k_finish(Scalars* __restrict__ scs, const InstDev* __restrict__ insts,
                                                      int pstride, const double* __restrict__ part,
                                                      fewha_solve_info* __restrict__ infos,
                                                      fewha_solve_info* __restrict__ infos_user, int iters,
                                                      double tol, int64_t* __restrict__ brk) {
    finish_instance(blockIdx.x, scs, insts, pstride, part, infos, infos_user, iters, tol, brk);
}

// End of a tolerance-stopped frame (after the statistics): an instance that stopped after
// `stop` < cap iterations wrote its directions to ring slots head .. head + stop - 1 only, while
// the next frame projects against the k slots before head + cap.  Its last k directions (with
// their (p_j, q_j)) are moved there, read before written since the two windows may overlap.
// `avail` counts the real directions now at the end of the window: GALERKIN keeps a ring over
// frames, PAPER only the frame's own directions.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_ring_forward(int64_t N, const VecBlk* __restrict__ vb, int K, int head,
                                                            int cap, int k, int paper, int first,
                                                            Scalars* __restrict__ scs, T* __restrict__ U,
                                                            T* __restrict__ Q) {
    const Seg sg = seg_of(vb, N, 0);
    Scalars* __restrict__ sc = scs + sg.inst;
    const int stop = sc->conv_iter ? sc->conv_iter : cap;
    if (sg.local == 0 && threadIdx.x == 0) {
        const int prev = first ? 0 : sc->avail;
        const int got = paper ? stop : prev + stop;
        if (stop < cap) {
            double g[kKMax];
            for (int a = 0; a < k; ++a) g[a] = sc->gam[(head + stop - k + a + 2 * K) % K];
            for (int a = 0; a < k; ++a) sc->gam[(head + cap - k + a + 2 * K) % K] = g[a];
        }
        sc->avail = got < k ? got : k;
    }
    if (stop >= cap) return;
    for (int64_t j = int64_t(sg.local) * kThreads + threadIdx.x; j < sg.n; j += int64_t(sg.nb) * kThreads) {
        const int64_t i = sg.off + j;
        T u[kKMax], q[kKMax];
#pragma unroll
        for (int a = 0; a < kKMax; ++a)
            if (a < k) {
                const size_t src = size_t((head + stop - k + a + 2 * K) % K) * N + i;
                u[a] = U[src];
                q[a] = Q[src];
            }
#pragma unroll
        for (int a = 0; a < kKMax; ++a)
            if (a < k) {
                const size_t dst = size_t((head + cap - k + a + 2 * K) % K) * N + i;
                U[dst] = u[a];
                Q[dst] = q[a];
            }
    }
}

// avail of every instance to (to_state) or from a checkpoint: a double at base + stride i.
__global__ void k_state_avail(Scalars* __restrict__ scs, int B, char* __restrict__ base, size_t stride, int to_state) {
    const int i = int(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= B) return;
    double* d = reinterpret_cast<double*>(base + stride * size_t(i));
    if (to_state) *d = double(scs[i].avail);
    else scs[i].avail = int(*d);
}

// ------------------------------------------------------------------ warm start

// z = J^-1 r
template <typename T>
__global__ void __launch_bounds__(kThreads) k_scale(int64_t N, const T* __restrict__ jinv, const T* __restrict__ r,
                                                     T* __restrict__ z) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < N) z[i] = jinv[i] * r[i];
}

__device__ __forceinline__ int layer_of(const LayerDev* __restrict__ lays, int L, int64_t i) {
    int lo = 0, hi = L - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lays[mid].off <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// network input of node i: [W^-1 c / s_c, W^-1 J^-1 r / s_r, h / 20 km, gamma] (FP32)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_ws_pack(int64_t N, const LayerDev* __restrict__ lays, int L,
                                                       const float2* __restrict__ lconst, const T* __restrict__ pc,
                                                       const T* __restrict__ pr, float isc, float isr,
                                                       float* __restrict__ in) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= N) return;
    const float2 k = lconst[layer_of(lays, L, i)];
    reinterpret_cast<float4*>(in)[i] = make_float4(float(pc[i]) * isc, float(pr[i]) * isr, k.x, k.y);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_ws_unpack(int64_t N, const float* __restrict__ out, float so,
                                                         T* __restrict__ d) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < N) d[i] = T(out[i] * so);
}

// z = J^-1 r with r = b - M c (rounded to the element type first, as the residual update does)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_ws_resid(int64_t N, const T* __restrict__ jinv, const T* __restrict__ b,
                                                        const T* __restrict__ mc, T* __restrict__ z) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < N) z[i] = jinv[i] * T(double(b[i]) - double(mc[i]));
}

// correction in coefficients: e = W d with W = delta^2 W^-T (W^-1 = DWT^T / delta, DWT
// orthonormal), from wtd = W^-T d
template <typename T>
__global__ void __launch_bounds__(kThreads) k_ws_delta(int64_t N, const LayerDev* __restrict__ lays, int L,
                                                        const T* __restrict__ wtd, T* __restrict__ e) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= N) return;
    const double id = lays[layer_of(lays, L, i)].inv_delta;
    e[i] = T(double(wtd[i]) / (id * id));
}

// partials of (e, r) and (e, M e) in rows P_PROJ, P_PROJ + 1
template <typename T>
__global__ void __launch_bounds__(kThreads) k_ws_dots(int64_t N, const VecBlk* __restrict__ vb, int pstride,
                                                       const T* __restrict__ e, const T* __restrict__ me,
                                                       const T* __restrict__ r, double* __restrict__ part) {
    const Seg sg = seg_of(vb, N, 0);
    double er = 0, em = 0;
    for (int64_t j = int64_t(sg.local) * kThreads + threadIdx.x; j < sg.n; j += int64_t(sg.nb) * kThreads) {
        const int64_t i = sg.off + j;
        const double ei = double(e[i]);
        er += ei * double(r[i]);
        em += ei * double(me[i]);
    }
    const double vv[2] = {er, em};
    block_partials<2>(vv, part, P_PROJ, pstride, sg.col);
}

// Exact line search of the energy 1/2 c^T M c - b^T c along the correction e, restricted to
// its own direction: tau = max(0, (e, r) / (e, M e)); c += tau e, r -= tau M e.  tau = 0
// (the correction points uphill, or is zero) leaves the frame as it was.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_ws_step(int64_t N, const VecBlk* __restrict__ vb, int pstride,
                                                       const double* __restrict__ part, T* __restrict__ c,
                                                       T* __restrict__ r, const T* __restrict__ e,
                                                       const T* __restrict__ me, Scalars* __restrict__ scs) {
    const Seg sg = seg_of(vb, N, 0);
    double v[2];
    block_row_sums<2>(part, pstride, sg, P_PROJ, 2, v);
    const bool skip = scs[sg.inst].flags != 0;   // broken frame: no correction
    const double tau = !skip && v[1] > 0 && v[0] > 0 && isfinite(v[0] / v[1]) ? v[0] / v[1] : 0.0;
    if (sg.local == 0 && threadIdx.x == 0) scs[sg.inst].ws_state = skip ? 0 : (tau > 0 ? 1 : 2);
    if (!(tau > 0)) return;
    for (int64_t j = int64_t(sg.local) * kThreads + threadIdx.x; j < sg.n; j += int64_t(sg.nb) * kThreads) {
        const int64_t i = sg.off + j;
        c[i] = T(double(c[i]) + tau * double(e[i]));
        r[i] = T(double(r[i]) - tau * double(me[i]));
    }
}

// The frame's outputs to the caller in one launch after the graph: the coefficients
// (c -> c_out, may be null) and, by the first workgroup, the per-instance statistics
// (info -> info_user, may be null).
// End of a graphed fixed-count frame, after the graph: workgroups b < B write instance b's
// frame statistics (as k_finish), every workgroup copies its share of c to c_out (if given).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_frame_out(int64_t N, const T* __restrict__ c, T* __restrict__ c_out,
                                                         int B, Scalars* __restrict__ scs,
                                                         const InstDev* __restrict__ insts, int pstride,
                                                         const double* __restrict__ part,
                                                         fewha_solve_info* __restrict__ infos,
                                                         fewha_solve_info* __restrict__ infos_user, int iters,
                                                         double tol, int64_t* __restrict__ brk) {
    if (int(blockIdx.x) < B) finish_instance(blockIdx.x, scs, insts, pstride, part, infos, infos_user, iters, tol, brk);
    if (c_out)
        for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < N; i += int64_t(gridDim.x) * kThreads)
            c_out[i] = c[i];
}

// Compile-time sizes of the recycle-space loops: exact up to 16, then in steps of 4.
int bucket(int m) {
    if (m <= 16) return m < 0 ? 0 : m;
    return (m + 3) / 4 * 4;
}

// Slot list padded to `mb` entries by repeating the first (the kernels give the padding
// coefficient 0, so every ring load is unconditional).
SlotList padded(const SlotList& sl, int m, int mb) {
    SlotList p = sl;
    for (int a = m; a < mb; ++a) p.s[a] = m > 0 ? sl.s[0] : 0;
    return p;
}

#define FEWHA_MB_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(20) X(24) X(28) X(32)

// Launch geometry shared by the vector kernels of one context.
struct VecLaunch {
    int64_t N;
    const VecBlk* vb;   // workgroup table (NULL for a single instance)
    int grid, pstride;
};

template <typename T, int MB>
void launch_gal(const VecLaunch& vl, int m, const SlotList& sl, const T* U, const T* Q, const Scalars* sc, T* c, T* r,
                T* p, const T* jinv, double* part, hipStream_t s) {
    k_galerkin_apply<T, MB><<<vl.grid, kThreads, 0, s>>>(vl.N, vl.vb, vl.pstride, m, sl, U, Q, sc, c, r, p, jinv, part);
}

// done (tolerance mode, else NULL): the per-instance stop flags.
template <typename T, int MP>
void launch_upd(const VecLaunch& vl, int it, int mp, const SlotList& pl, const T* U, const T* Q, Scalars* sc,
                T* p, T* q, T* c, T* r, T* z, const T* jinv, int last, int npq, const double* pq_part,
                double* part, int pslot, int project_all, T* pn, const Ctx& ctx, hipStream_t s, int32_t* done) {
    {
        ProfScope ps_(ctx, KID_UPDATE1, s);
        k_update1<T, MP><<<vl.grid, kThreads, 0, s>>>(vl.N, vl.vb, vl.pstride, it, mp, pl, U, Q, sc, p, q, c, r, z,
                                                      jinv, last, npq, pq_part, part, pslot, done);
    }
    if (!last) {
        ProfScope ps_(ctx, KID_UPDATE2, s);
        k_update2<T, MP><<<vl.grid, kThreads, 0, s>>>(vl.N, vl.vb, vl.pstride, it, mp, project_all, pl, U, sc, z, p, pn,
                                                      part, done ? ctx.rel_tol : 0.0, done);
    }
}

}  // namespace

// Pointers and recycle sets of one frame (derived from the host-side ring bookkeeping).
template <typename T>
struct Frame {
    int64_t N;
    int K, m, mb, mp, mpb;
    SlotList act, actp, pl;
    T *b, *bp, *r, *z, *cv, *vx, *vy, *U, *Q;
    const T* jinv;
    double *part, *pqp, *gpart;
    Scalars* sc;
    const InstDev* insts;
    fewha_solve_info* info;
    VecLaunch vl;
    const GramBlk* gt;
    int ke;
    int32_t* done;   // tolerance mode: per-instance stop flags (NULL with a fixed count)

    explicit Frame(const Ctx& c) {
        N = c.N;
        K = c.slots;
        b = c.at<T>(c.lay.b);
        bp = c.at<T>(c.lay.b_prev);
        r = c.at<T>(c.lay.r);
        z = c.at<T>(c.lay.z);
        cv = c.at<T>(c.lay.c);
        vx = c.at<T>(c.lay.vx);
        vy = c.at<T>(c.lay.vy);
        U = c.at<T>(c.lay.ring_u);
        Q = c.at<T>(c.lay.ring_q);
        jinv = c.at<T>(c.lay.jinv);
        part = c.at<double>(c.lay.partials);
        pqp = c.at<double>(c.lay.pq_part);
        gpart = c.at<double>(c.lay.gram_part);
        sc = c.at<Scalars>(c.lay.scalars);
        insts = c.at<InstDev>(c.lay.insts);
        info = c.at<fewha_solve_info>(c.lay.info);
        vl = VecLaunch{N, c.B > 1 ? c.at<VecBlk>(c.lay.vecblk) : nullptr, c.VB, c.VB};
        gt = c.B > 1 ? c.at<GramBlk>(c.lay.gramblk) : nullptr;
        ke = std::max(1, 2 * c.k * (c.k + 1));
        done = c.rel_tol > 0 ? c.at<int32_t>(c.lay.done) : nullptr;
        m = 0;
        if (!c.first && c.k > 0)
            m = c.mode == FEWHA_RECYCLE_PAPER ? std::min(c.last_iters, c.k) : std::min(c.count, c.k);
        act = SlotList{};
        for (int j = 0; j < m; ++j) act.s[j] = ((c.head - m + j) % K + K) % K;
        mb = bucket(m);
        actp = padded(act, m, mb);
        // in-loop projection set: all of U (project_all) or the most recent recycled direction
        pl = SlotList{};
        mp = 0;
        if (m > 0) {
            if (c.project_all) {
                pl = act;
                mp = m;
            } else {
                pl.s[0] = ((c.head - 1) % K + K) % K;
                mp = 1;
            }
        }
        mpb = bucket(mp);
        pl = padded(pl, mp, mpb);
    }
};

// a1 + a2: right-hand side and residual update.
template <typename T>
void enqueue_rhs_residual(const Ctx& c, const Frame<T>& f, const T* slopes, hipStream_t s) {
    launch_rhs<T>(c, slopes, f.b, s, f.pqp);   // with the partials of (b, b)
    if (c.first) launch_apply_M<T>(c, f.cv, f.vx, nullptr, s);
    ProfScope ps_(c, KID_RESIDUAL, s);
    k_residual<T><<<f.vl.grid, kThreads, 0, s>>>(f.N, f.vl.vb, f.vl.pstride, f.b, f.bp, f.r,
                                                 c.first ? f.vx : nullptr, f.part, f.sc, f.m, c.npq, f.pqp, f.done);
}

// a3 + a4: Galerkin step and initial direction.
template <typename T>
void enqueue_galerkin_init(const Ctx& c, const Frame<T>& f, hipStream_t s) {
    const int m = f.m;
    T* p0 = f.U + size_t(c.head) * f.N;
    if (m > 0) {
        {
            ProfScope ps_(c, KID_GRAM, s);
            const dim3 grid(c.GB, ((m + 15) / 16) * ((m + 1 + 15) / 16));
            if (m <= 11 && c.mode != FEWHA_RECYCLE_PAPER)
                k_gram<T, true, true><<<grid, kGramThreads, 0, s>>>(f.N, f.gt, m, f.act, f.U, f.Q, f.r, f.jinv, f.gpart);
            else if (m < 16)
                k_gram<T, true><<<grid, kGramThreads, 0, s>>>(f.N, f.gt, m, f.act, f.U, f.Q, f.r, f.jinv, f.gpart);
            else
                k_gram<T, false><<<grid, kGramThreads, 0, s>>>(f.N, f.gt, m, f.act, f.U, f.Q, f.r, f.jinv, f.gpart);
        }
        {
            ProfScope ps_(c, KID_GRAM_SOLVE, s);
#define GS(mb) k_gram_solve<mb><<<c.B, kSolveThreads, 0, s>>>(m, c.mode, f.act, f.sc, f.insts, f.ke, f.gpart, \
                                                             f.done ? 1 : 0)
            if (m <= 4) GS(4);
            else if (m <= 8) GS(8);
            else if (m <= 12) GS(12);
            else if (m <= 16) GS(16);
            else if (m <= 24) GS(24);
            else GS(32);
#undef GS
        }
        ProfScope ps_(c, KID_GALERKIN, s);
        switch (f.mb) {
#define X(v) case v: launch_gal<T, v>(f.vl, m, f.actp, f.U, f.Q, f.sc, f.cv, f.r, p0, f.jinv, f.part, s); break;
            FEWHA_MB_CASES(X)
#undef X
        }
    } else {
        ProfScope ps_(c, KID_INIT_DIR, s);
        k_init_dir<T><<<f.vl.grid, kThreads, 0, s>>>(f.vl.N, f.vl.vb, f.vl.pstride, f.r, f.jinv, p0, f.part, f.sc);
    }
}

// a5 + a6: iteration `it` (the last one skips the next direction).
template <typename T>
void enqueue_iteration(const Ctx& c, const Frame<T>& f, int it, int last, hipStream_t s) {
    const int ps = (c.head + it) % f.K;
    T* p = f.U + size_t(ps) * f.N;
    T* q = f.Q + size_t(ps) * f.N;
    T* pn = f.U + size_t((c.head + it + 1) % f.K) * f.N;
    launch_apply_M<T>(c, p, q, f.pqp, s, nullptr, f.done);
    switch (f.mpb) {
        case 0: launch_upd<T, 0>(f.vl, it, f.mp, f.pl, f.U, f.Q, f.sc, p, q, f.cv, f.r, f.z, f.jinv, last, c.npq,
                                 f.pqp, f.part, ps, c.project_all, pn, c, s, f.done); break;
#define X(v) case v: launch_upd<T, v>(f.vl, it, f.mp, f.pl, f.U, f.Q, f.sc, p, q, f.cv, f.r, f.z, f.jinv, last, \
                                      c.npq, f.pqp, f.part, ps, c.project_all, pn, c, s, f.done); break;
        FEWHA_MB_CASES(X)
#undef X
    }
}

template <typename T>
void enqueue_finish(const Ctx& c, const Frame<T>& f, int iters, fewha_solve_info* info_user, hipStream_t s) {
    ProfScope ps_(c, KID_FINISH, s);
    k_finish<<<c.B, kThreads, 0, s>>>(f.sc, f.insts, f.vl.pstride, f.part, f.info, info_user, iters, c.rel_tol,
                                      c.brk_dev);
}

// Tolerance mode, after the frame's statistics: move the last directions of instances that
// stopped early to the end of the recycle window.
template <typename T>
void enqueue_ring_forward(const Ctx& c, const Frame<T>& f, hipStream_t s) {
    if (!f.done || c.k == 0) return;
    k_ring_forward<T><<<f.vl.grid, kThreads, 0, s>>>(f.N, f.vl.vb, f.K, c.head, c.max_iter, c.k,
                                                     c.mode == FEWHA_RECYCLE_PAPER ? 1 : 0, c.first ? 1 : 0, f.sc,
                                                     f.U, f.Q);
}

// Enqueues one fixed-count frame on stream s (no host-state change, so it can be captured).
template <typename T>
void enqueue_frame(const Ctx& c, const T* slopes, fewha_solve_info* info_user, hipStream_t s, bool finish = true) {
    const Frame<T> f(c);
    enqueue_rhs_residual<T>(c, f, slopes, s);
    enqueue_galerkin_init<T>(c, f, s);
    for (int it = 0; it < c.max_iter; ++it) enqueue_iteration<T>(c, f, it, it == c.max_iter - 1, s);
    if (finish) {
        enqueue_finish<T>(c, f, c.max_iter, info_user, s);
        enqueue_ring_forward<T>(c, f, s);
    }
}

// Frame with direct launches (fixed count or tolerance mode; the device decides each
// instance's stop, so nothing here waits for the device).  `between` runs after the residual
// update (a warm start).
template <typename T, typename Hook>
hipError_t run_frame(Ctx& c, const T* slopes, fewha_solve_info* info_user, hipStream_t s, int* iters, Hook between) {
    const Frame<T> f(c);
    enqueue_rhs_residual<T>(c, f, slopes, s);
    hipError_t e = between(f);
    if (e != hipSuccess) return e;
    enqueue_galerkin_init<T>(c, f, s);
    for (int it = 0; it < c.max_iter; ++it) enqueue_iteration<T>(c, f, it, it == c.max_iter - 1, s);
    enqueue_finish<T>(c, f, c.max_iter, info_user, s);
    enqueue_ring_forward<T>(c, f, s);
    *iters = c.max_iter;
    return hipGetLastError();
}

// Host ring bookkeeping after a frame of `iters` iterations, and the coefficient copy.
template <typename T>
hipError_t end_frame(Ctx& c, T* c_out, int iters, hipError_t e, hipStream_t s) {
    if (e == hipSuccess && c_out)
        e = hipMemcpyAsync(c_out, c.at<T>(c.lay.c), sizeof(T) * c.N, hipMemcpyDeviceToDevice, s);
    const int K = c.slots;
    c.head = (c.head + iters) % K;
    c.count = std::min(c.count + iters, K);
    c.last_iters = iters;
    c.frame_iters = iters;
    c.first = false;
    return e;
}

template <typename T>
hipError_t launch_solve_frame(Ctx& c, const T* slopes, T* c_out, fewha_solve_info* info_user, hipStream_t s) {
    int m = 0;
    if (!c.first && c.k > 0)
        m = c.mode == FEWHA_RECYCLE_PAPER ? std::min(c.last_iters, c.k) : std::min(c.count, c.k);
    hipError_t e = hipSuccess;
    int iters = c.max_iter;
    if (c.use_graphs && !c.prof.on) {
        // the slope adjoint runs before the graph on the caller's slopes (the graph starts from
        // the sensor-node buffer it fills); the frame statistics and the copy of c follow it
        fewha_solve_info* info = c.at<fewha_solve_info>(c.lay.info);
        const auto key = std::make_tuple(c.head, c.first ? 1 : 0, m);
        auto it = c.graphs.find(key);
        if (it == c.graphs.end()) {
            if (!c.cap_stream) e = hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking);
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            if (e == hipSuccess) e = hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                enqueue_frame<T>(c, static_cast<const T*>(nullptr), nullptr, c.cap_stream, false);
                e = hipStreamEndCapture(c.cap_stream, &g);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) return e;
            it = c.graphs.emplace(key, ge).first;
        }
        launch_slopes_adj<T>(c, slopes, c.at<T>(c.lay.psi_nodes), 1, s);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipGraphLaunch(it->second, s);
        if (e == hipSuccess) {   // frame statistics (the graph ends with the last iteration) and c_out
            const Frame<T> f(c);
            const int64_t ncopy = c_out ? std::min<int64_t>((c.N + 4 * kThreads - 1) / (4 * kThreads), 4096) : 0;
            const int64_t nb = std::max<int64_t>(c.B, ncopy);
            k_frame_out<T><<<unsigned(nb), kThreads, 0, s>>>(c.N, c.at<T>(c.lay.c), c_out, c.B, f.sc, f.insts,
                                                             f.vl.pstride, f.part, info, info_user, c.max_iter,
                                                             c.rel_tol, c.brk_dev);
            enqueue_ring_forward<T>(c, f, s);
            e = hipGetLastError();
        }
        return end_frame<T>(c, static_cast<T*>(nullptr), iters, e, s);
    } else {
        enqueue_frame<T>(c, slopes, info_user, s);
    }
    return end_frame<T>(c, c_out, iters, e, s);
}

// Warm-started frame: after the residual update, the network maps [W^-1 c, W^-1 J^-1 r,
// h / 20 km, gamma] of every layer to a nodal correction d; the coefficient correction
// e = W d (W = delta^2 W^-T) enters with the step that minimises the energy the PCG minimises,
// tau = max(0, (e, r) / (e, M e)) (one extra operator apply; the solver sizes the correction
// and takes none of it when it points uphill); then the Galerkin step, the initial direction
// and the iterations as in any frame.
template <typename T>
hipError_t launch_solve_frame_ws(Ctx& c, const WarmStart& w, const T* slopes, T* c_out, fewha_solve_info* info_user,
                                 hipStream_t s) {
    int iters = c.max_iter;
    const LayerDev* lays = c.at<LayerDev>(c.lay.layers);
    float* in = c.at<float>(c.lay.ws_in);
    float* out = c.at<float>(c.lay.ws_out);
    T* nod = c.at<T>(c.lay.nodal);
    T* nod_r = c.at<T>(c.lay.psi_layers);
    auto hook = [&](const Frame<T>& f) -> hipError_t {
        const unsigned gN = unsigned((f.N + kThreads - 1) / kThreads);
        k_scale<T><<<gN, kThreads, 0, s>>>(f.N, f.jinv, f.r, f.z);            // z = J^-1 r
        launch_winv<T>(c, f.cv, nod, s);                                      // W^-1 c
        launch_winv<T>(c, f.z, nod_r, s);                                     // W^-1 J^-1 r
        k_ws_pack<T><<<gN, kThreads, 0, s>>>(f.N, lays, c.L, c.at<float2>(c.lay.lconst), nod, nod_r, 1.f / w.scale_c,
                                            1.f / w.scale_r, in);
        const fewha_status st = fewha_unet_forward(static_cast<fewha_unet*>(w.net), in, out, s);
        if (st != FEWHA_OK) return hipErrorLaunchFailure;
        k_ws_unpack<T><<<gN, kThreads, 0, s>>>(f.N, out, w.scale_out, nod);   // d (nodal)
        launch_winvt<T>(c, nod, f.z, static_cast<const T*>(nullptr), nullptr, s);   // W^-T d
        k_ws_delta<T><<<gN, kThreads, 0, s>>>(f.N, lays, c.L, f.z, f.vy);      // e = delta^2 W^-T d
        launch_apply_M<T>(c, f.vy, f.vx, nullptr, s);                         // M e
        k_ws_dots<T><<<f.vl.grid, kThreads, 0, s>>>(f.N, f.vl.vb, f.vl.pstride, f.vy, f.vx, f.r, f.part);
        k_ws_step<T><<<f.vl.grid, kThreads, 0, s>>>(f.N, f.vl.vb, f.vl.pstride, f.part, f.cv, f.r, f.vy, f.vx, f.sc);
        return hipGetLastError();
    };
    const hipError_t e = run_frame<T>(c, slopes, info_user, s, &iters, hook);
    return end_frame<T>(c, c_out, iters, e, s);
}

// Network input of the warm start of the frame with slopes `slopes` that follows the
// coefficients c_in: r = b - M c_in, then [W^-1 c_in / s_c, W^-1 J^-1 r / s_r, h / 20 km, gamma]
// per node into `in` (FP32, N x 4).  Uses the context's scratch vectors only (the carried state
// is not touched).
template <typename T>
hipError_t launch_ws_input(const Ctx& c, const WarmStart& w, const T* c_in, const T* slopes, float* in,
                           hipStream_t s) {
    const unsigned gN = unsigned((c.N + kThreads - 1) / kThreads);
    T* b = c.at<T>(c.lay.vy);
    T* mc = c.at<T>(c.lay.vx);
    T* z = c.at<T>(c.lay.z);
    T* nod = c.at<T>(c.lay.nodal);
    T* nod_r = c.at<T>(c.lay.psi_layers);
    launch_rhs<T>(c, slopes, b, s);
    launch_apply_M<T>(c, c_in, mc, nullptr, s);
    k_ws_resid<T><<<gN, kThreads, 0, s>>>(c.N, c.at<T>(c.lay.jinv), b, mc, z);
    launch_winv<T>(c, c_in, nod, s);
    launch_winv<T>(c, z, nod_r, s);
    k_ws_pack<T><<<gN, kThreads, 0, s>>>(c.N, c.at<LayerDev>(c.lay.layers), c.L, c.at<float2>(c.lay.lconst), nod,
                                         nod_r, 1.f / w.scale_c, 1.f / w.scale_r, in);
    return hipGetLastError();
}

hipError_t launch_state_avail(const Ctx& c, char* base, size_t stride, bool to_state, hipStream_t s) {
    const int B = c.B;
    k_state_avail<<<(B + kThreads - 1) / kThreads, kThreads, 0, s>>>(c.at<Scalars>(c.lay.scalars), B,
                                                                     base + sizeof(double) * c.slots, stride,
                                                                     to_state ? 1 : 0);
    return hipGetLastError();
}

void release_graphs(Ctx& c) {
    for (auto& kv : c.graphs) (void)hipGraphExecDestroy(kv.second);
    c.graphs.clear();
    if (c.cap_stream) (void)hipStreamDestroy(c.cap_stream);
    c.cap_stream = nullptr;
}

template hipError_t launch_solve_frame<float>(Ctx&, const float*, float*, fewha_solve_info*, hipStream_t);
template hipError_t launch_solve_frame<double>(Ctx&, const double*, double*, fewha_solve_info*, hipStream_t);
template hipError_t launch_solve_frame_ws<float>(Ctx&, const WarmStart&, const float*, float*, fewha_solve_info*,
                                                 hipStream_t);
template hipError_t launch_solve_frame_ws<double>(Ctx&, const WarmStart&, const double*, double*, fewha_solve_info*,
                                                  hipStream_t);
template hipError_t launch_ws_input<float>(const Ctx&, const WarmStart&, const float*, const float*, float*,
                                           hipStream_t);
template hipError_t launch_ws_input<double>(const Ctx&, const WarmStart&, const double*, const double*, float*,
                                            hipStream_t);

}  // namespace fewha
