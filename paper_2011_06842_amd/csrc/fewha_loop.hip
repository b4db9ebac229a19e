// Closed-loop wrapper of the augmented wavelet reconstructor (Sec. 5, Alg. 3; declared in
// include/fewha_loop.h): pseudo-open-loop slopes, fitting of the layers to DM commands and
// gain control, around the frame solve of the loop's context.
//
// Kernels (HIP, gfx950).  Coordinates and bilinear weights are computed in FP64 from per-pair
// affine maps built on the host (u = u0 + column du, v = v0 + row dv); values are summed in the
// context's element type.
//   k_dm_slopes    per slope: the DM surfaces at the sensor's 4 subaperture corners (cone and
//                  shift per DM), the Shack-Hartmann slope, added to the measured slope
//   k_fit_direct   per actuator: layer d's function at the actuator (direct fitting)
//   k_fit_project  per (direction, pupil point): sum over layers or DMs of their bilinear value
//   k_fit_adj      per actuator: the transpose of the DM projection as a gather over the pupil
//                  points whose cell touches the actuator (fixed order, no atomics)
//   k_cg_init/step one workgroup: the CG vectors of the fitting's normal equations (a few
//                  thousand actuators) and its FP64 scalars
//   k_gain         per actuator: the gain control of Alg. 3
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fewha_internal.h"
#include "../../include/fewha_loop.h"

namespace fewha {
namespace {

struct Affine { double u0, du, v0, dv; };   // u = u0 + column du, v = v0 + row dv (grid coordinates)
struct Grid { int32_t n, pad_; int64_t off; };

constexpr int kCgThreads = 1024;

// Bilinear interpolant of an n x n node grid at (u, v), nodes beyond the grid being zero.
template <typename T>
__device__ __forceinline__ T bil_zero(const T* __restrict__ img, int n, double u, double v) {
    const double fb = floor(u), fa = floor(v);
    const int b0 = int(fb), a0 = int(fa);
    const double fx = u - fb, fy = v - fa;
    T acc = 0;
#pragma unroll
    for (int da = 0; da < 2; ++da) {
        const int a = a0 + da;
        const double wa = da ? fy : 1.0 - fy;
#pragma unroll
        for (int db = 0; db < 2; ++db) {
            const int b = b0 + db;
            const double wb = db ? fx : 1.0 - fx;
            if (a >= 0 && a < n && b >= 0 && b < n) acc += T(wa * wb) * img[size_t(a) * n + b];
        }
    }
    return acc;
}

// Weight of node `a` in the bilinear interpolation at coordinate u (as bil_zero forms it).
__device__ __forceinline__ double bil_weight(double u, int a) {
    const double fb = floor(u);
    const int b0 = int(fb);
    const double f = u - fb;
    return b0 == a ? 1.0 - f : (b0 + 1 == a ? f : 0.0);
}

// Shack-Hartmann slope of every measurement plus H a: the DM surfaces (sum over DMs) at the 4
// corners of the subaperture, x-slope ((c01 - c00) + (c11 - c10)) / 2, y-slope
// ((c10 - c00) + (c11 - c01)) / 2; out = in + slope on active subapertures (weight != 0), in on
// the others (in NULL: 0).
template <typename T>
__global__ void __launch_bounds__(256) k_dm_slopes(const int64_t* __restrict__ soff, const int32_t* __restrict__ nsub,
                                                    int G, int64_t S, const Grid* __restrict__ dms, int nd,
                                                    const Affine* __restrict__ aff, const T* __restrict__ a,
                                                    const T* __restrict__ w, const T* __restrict__ in,
                                                    T* __restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= S) return;
    int g = 0;
    while (g + 1 < G && soff[g + 1] <= e) ++g;
    const int ns = nsub[g];
    const int loc = int(e - soff[g]);
    const int comp = loc / (ns * ns), q = loc % (ns * ns), i = q / ns, j = q % ns;
    T c[2][2] = {{0, 0}, {0, 0}};
    for (int d = 0; d < nd; ++d) {
        const Affine A = aff[g * nd + d];
        const T* ad = a + dms[d].off;
        const int n = dms[d].n;
#pragma unroll
        for (int di = 0; di < 2; ++di)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj)
                c[di][dj] += bil_zero(ad, n, A.u0 + double(j + dj) * A.du, A.v0 + double(i + di) * A.dv);
    }
    const T sl = comp == 0 ? T(0.5) * ((c[0][1] - c[0][0]) + (c[1][1] - c[1][0]))
                           : T(0.5) * ((c[1][0] - c[0][0]) + (c[1][1] - c[0][1]));
    const T base = in ? in[e] : T(0);
    out[e] = w[e] != T(0) ? base + sl : base;
}

// Direct fitting: actuator (row, col) of DM d takes layer d's function there.
template <typename T>
__global__ void __launch_bounds__(256) k_fit_direct(const Grid* __restrict__ dms, int nd, const Grid* __restrict__ lays,
                                                     const Affine* __restrict__ aff, const T* __restrict__ phi,
                                                     int64_t n_act, T* __restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n_act) return;
    int d = 0;
    while (d + 1 < nd && dms[d + 1].off <= e) ++d;
    const int n = dms[d].n;
    const int loc = int(e - dms[d].off), row = loc / n, col = loc % n;
    const Affine A = aff[d];
    out[e] = bil_zero(phi + lays[d].off, lays[d].n, A.u0 + col * A.du, A.v0 + row * A.dv);
}

// value[dir][p] = sum over the grids (layers or DMs) of their bilinear value at pupil point p
// seen from direction dir.
template <typename T>
__global__ void __launch_bounds__(256) k_fit_project(const Grid* __restrict__ grids, int ng,
                                                      const Affine* __restrict__ aff, const int2* __restrict__ pts,
                                                      int npts, int ndir, const T* __restrict__ x,
                                                      T* __restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(npts) * ndir) return;
    const int dir = int(e / npts), p = int(e % npts);
    const int2 pc = pts[p];   // (column, row) on the pupil grid
    T v = 0;
    for (int k = 0; k < ng; ++k) {
        const Affine A = aff[dir * ng + k];
        v += bil_zero(x + grids[k].off, grids[k].n, A.u0 + pc.x * A.du, A.v0 + pc.y * A.dv);
    }
    out[e] = v;
}

// Transpose of the DM projection: actuator (row, col) of DM d gathers, for every direction,
// the pupil points whose bilinear cell touches it (|u - col| < 1 and |v - row| < 1), with the
// weights the projection gives it; directions, then rows, then columns in increasing order.
template <typename T>
__global__ void __launch_bounds__(256) k_fit_adj(const Grid* __restrict__ dms, int nd, const Affine* __restrict__ aff,
                                                  const int32_t* __restrict__ pmap, int n_pts, int npts, int ndir,
                                                  int64_t n_act, const T* __restrict__ val, T* __restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n_act) return;
    int d = 0;
    while (d + 1 < nd && dms[d + 1].off <= e) ++d;
    const int n = dms[d].n;
    const int loc = int(e - dms[d].off), row = loc / n, col = loc % n;
    T acc = 0;
    for (int dir = 0; dir < ndir; ++dir) {
        const Affine A = aff[dir * nd + d];
        const int c0 = max(0, int(ceil((col - 1 - A.u0) / A.du)) - 1);
        const int c1 = min(n_pts - 1, int(floor((col + 1 - A.u0) / A.du)) + 1);
        const int r0 = max(0, int(ceil((row - 1 - A.v0) / A.dv)) - 1);
        const int r1 = min(n_pts - 1, int(floor((row + 1 - A.v0) / A.dv)) + 1);
        for (int r = r0; r <= r1; ++r) {
            const double wy = bil_weight(A.v0 + r * A.dv, row);
            if (wy == 0.0) continue;
            for (int cc = c0; cc <= c1; ++cc) {
                const int p = pmap[r * n_pts + cc];
                if (p < 0) continue;
                const double wx = bil_weight(A.u0 + cc * A.du, col);
                if (wx != 0.0) acc += T(wy * wx) * val[int64_t(dir) * npts + p];
            }
        }
    }
    out[e] = acc;
}

// Fixed-order FP64 sum of one value per thread over the workgroup (every thread gets it).
__device__ __forceinline__ double cg_block_sum(double v) {
    __shared__ double sh[kCgThreads];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = kCgThreads / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// r = b - A x, p = r, rr = (r, r).
template <typename T>
__global__ void __launch_bounds__(kCgThreads) k_cg_init(int64_t n, const T* __restrict__ b, const T* __restrict__ ax,
                                                         T* __restrict__ r, T* __restrict__ p, double* __restrict__ scal) {
    double rr = 0;
    for (int64_t i = threadIdx.x; i < n; i += kCgThreads) {
        const T ri = b[i] - ax[i];
        r[i] = ri;
        p[i] = ri;
        rr += double(ri) * double(ri);
    }
    rr = cg_block_sum(rr);
    if (threadIdx.x == 0) scal[0] = rr;
}

// One CG step with q = A p: alpha = rr / (p, q), x += alpha p, r -= alpha q, beta = rr' / rr,
// p = r + beta p.
template <typename T>
__global__ void __launch_bounds__(kCgThreads) k_cg_step(int64_t n, T* __restrict__ x, T* __restrict__ r,
                                                         T* __restrict__ p, const T* __restrict__ q,
                                                         double* __restrict__ scal) {
    double pq = 0;
    for (int64_t i = threadIdx.x; i < n; i += kCgThreads) pq += double(p[i]) * double(q[i]);
    pq = cg_block_sum(pq);
    const double rr = scal[0];
    const double alpha = pq > 0 ? rr / pq : 0.0;
    double rn = 0;
    for (int64_t i = threadIdx.x; i < n; i += kCgThreads) {
        x[i] = T(double(x[i]) + alpha * double(p[i]));
        const T ri = T(double(r[i]) - alpha * double(q[i]));
        r[i] = ri;
        rn += double(ri) * double(ri);
    }
    rn = cg_block_sum(rn);
    const double beta = rr > 0 ? rn / rr : 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kCgThreads) p[i] = T(double(r[i]) + beta * double(p[i]));
    __syncthreads();
    if (threadIdx.x == 0) scal[0] = rn;
}

// Gain control of Alg. 3.
template <typename T>
__global__ void __launch_bounds__(256) k_gain(int64_t n, const T* __restrict__ prev, const T* __restrict__ cur,
                                               const T* __restrict__ fit, T* __restrict__ next, double gain,
                                               int closed) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double pv = double(prev[i]), cv = double(cur[i]), fv = double(fit[i]);
    next[i] = T(closed ? cv + gain * (fv - pv) : (1.0 - gain) * cv + gain * fv);
}

unsigned cdiv64(int64_t a, int b) { return unsigned((a + b - 1) / b); }

}  // namespace
}  // namespace fewha

struct fewha_loop {
    fewha_ctx* ctx = nullptr;
    int nd = 0, G = 0, L = 0, ndir = 0, n_pts = 0, npts = 0, fit_iter = 0, closed = 1;
    double gain = 0.4;
    int64_t n_act = 0, N = 0, S = 0;
    size_t esz = 8;
    char* ws = nullptr;
    // workspace offsets
    size_t o_soff, o_nsub, o_dms, o_lays, o_sd_aff, o_dir_aff, o_fd_aff, o_fl_aff, o_pts, o_pmap;
    size_t o_cmd[4], o_r, o_p, o_q, o_b, o_pup, o_nodal, o_spol, o_scal, total;
    int prev = 0, cur = 1, fit = 2, spare = 3;   // which command buffer holds a^(i-1), a^(i), a~
    std::string err;
    template <typename P> P* at(size_t o) const { return reinterpret_cast<P*>(ws + o); }
};

namespace {

using fewha::Affine;
using fewha::Grid;

fewha_status loop_fail(fewha_loop* lp, fewha_status st, const std::string& m) {
    if (lp) lp->err = m;
    return st;
}

thread_local std::string g_loop_err;

// Host-side description shared by sizing and setup.
struct LoopPlan {
    std::vector<int64_t> soff;
    std::vector<int32_t> nsub;
    std::vector<Grid> dms, lays;
    std::vector<Affine> sd_aff, dir_aff, fd_aff, fl_aff;
    std::vector<int2> pts;
    std::vector<int32_t> pmap;
    int64_t n_act = 0;
};

fewha_status plan_loop(const fewha_ctx* ctx, const fewha_loop_config* cfg, LoopPlan& pl, std::string& err) {
    if (!ctx || !cfg) { err = "NULL argument"; return FEWHA_E_INVAL; }
    const fewha::Ctx& c = ctx->c;
    if (cfg->abi_version != FEWHA_ABI_VERSION) { err = "abi_version mismatch"; return FEWHA_E_INVAL; }
    if (c.B != 1) { err = "the closed loop needs a single-instance context"; return FEWHA_E_INVAL; }
    if (cfg->n_dm < 1 || cfg->n_dm > FEWHA_LOOP_MAX_DM || !cfg->dms) { err = "n_dm out of range"; return FEWHA_E_INVAL; }
    if (!(cfg->gain > 0) || !(cfg->gain <= 1)) { err = "gain must be in (0, 1]"; return FEWHA_E_INVAL; }
    if (cfg->fit_iter < 0 || cfg->fit_iter > 64) { err = "fit_iter out of range [0, 64]"; return FEWHA_E_INVAL; }
    for (int d = 0; d < cfg->n_dm; ++d) {
        const fewha_dm& D = cfg->dms[d];
        if (D.n < 2 || D.n > 1024) { err = "DM actuators per side out of range [2, 1024]"; return FEWHA_E_INVAL; }
        if (!(D.spacing > 0) || !std::isfinite(D.spacing) || !std::isfinite(D.height) || D.height < 0 ||
            !std::isfinite(D.origin_x) || !std::isfinite(D.origin_y)) {
            err = "bad DM geometry";
            return FEWHA_E_INVAL;
        }
    }
    pl = LoopPlan{};
    int64_t off = 0;
    for (int d = 0; d < cfg->n_dm; ++d) {
        pl.dms.push_back(Grid{cfg->dms[d].n, 0, off});
        off += int64_t(cfg->dms[d].n) * cfg->dms[d].n;
    }
    pl.n_act = off;
    int64_t lo = 0;
    for (const fewha_layer& Ly : c.layers) {
        pl.lays.push_back(Grid{Ly.n, 0, lo});
        lo += int64_t(Ly.n) * Ly.n;
    }
    // sensors and the (sensor, DM) maps of node (i, j) -> DM grid coordinates
    int64_t so = 0;
    for (const fewha_wfs& W : c.wfs) {
        pl.soff.push_back(so);
        pl.nsub.push_back(W.n_sub);
        so += 2 * int64_t(W.n_sub) * W.n_sub;
        for (int d = 0; d < cfg->n_dm; ++d) {
            const fewha_dm& D = cfg->dms[d];
            const double sc = W.lgs_height > 0 ? 1.0 - D.height / W.lgs_height : 1.0;
            const double x0 = -0.5 * W.n_sub * W.subap;
            Affine A;
            A.du = sc * W.subap / D.spacing;
            A.u0 = (sc * x0 + W.theta_x * D.height - D.origin_x) / D.spacing + 0.5 * (D.n - 1);
            A.dv = A.du;
            A.v0 = (sc * x0 + W.theta_y * D.height - D.origin_y) / D.spacing + 0.5 * (D.n - 1);
            pl.sd_aff.push_back(A);
        }
    }
    pl.soff.push_back(so);
    if (cfg->fit_iter == 0) {
        if (cfg->n_dm != int(c.layers.size())) { err = "direct fitting needs one DM per layer"; return FEWHA_E_INVAL; }
        for (int d = 0; d < cfg->n_dm; ++d) {
            const fewha_dm& D = cfg->dms[d];
            const fewha_layer& Ly = c.layers[d];
            if (std::fabs(D.height - Ly.height) > 1e-9 * std::max(1.0, Ly.height)) {
                err = "direct fitting needs DM " + std::to_string(d) + " at the altitude of layer " + std::to_string(d);
                return FEWHA_E_INVAL;
            }
            Affine A;   // actuator column -> layer grid coordinate
            A.du = D.spacing / Ly.spacing;
            A.u0 = (D.origin_x - 0.5 * (D.n - 1) * D.spacing - Ly.origin_x) / Ly.spacing + 0.5 * (Ly.n - 1);
            A.dv = A.du;
            A.v0 = (D.origin_y - 0.5 * (D.n - 1) * D.spacing - Ly.origin_y) / Ly.spacing + 0.5 * (Ly.n - 1);
            pl.dir_aff.push_back(A);
        }
    } else {
        if (cfg->n_dirs < 1 || cfg->n_dirs > FEWHA_LOOP_MAX_DIRS || !cfg->dirs) { err = "n_dirs out of range"; return FEWHA_E_INVAL; }
        if (cfg->n_pts < 2 || cfg->n_pts > 512) { err = "n_pts out of range [2, 512]"; return FEWHA_E_INVAL; }
        if (!(cfg->pupil_d > 0) || !(cfg->obstruction >= 0) || !(cfg->obstruction < 1)) { err = "bad fitting pupil"; return FEWHA_E_INVAL; }
        const int np = cfg->n_pts;
        const double dp = cfg->pupil_d / (np - 1);
        pl.pmap.assign(size_t(np) * np, -1);
        for (int r = 0; r < np; ++r)
            for (int cc = 0; cc < np; ++cc) {
                const double x = (cc - 0.5 * (np - 1)) * dp, y = (r - 0.5 * (np - 1)) * dp;
                const double rad = std::hypot(x, y);
                if (rad <= 0.5 * cfg->pupil_d && rad >= 0.5 * cfg->obstruction * cfg->pupil_d) {
                    pl.pmap[size_t(r) * np + cc] = int32_t(pl.pts.size());
                    pl.pts.push_back(make_int2(cc, r));
                }
            }
        if (pl.pts.empty()) { err = "the fitting pupil has no points"; return FEWHA_E_INVAL; }
        const double x0 = -0.5 * (np - 1) * dp;
        for (int k = 0; k < cfg->n_dirs; ++k) {
            const double tx = cfg->dirs[2 * k], ty = cfg->dirs[2 * k + 1];
            if (!std::isfinite(tx) || !std::isfinite(ty)) { err = "bad fitting direction"; return FEWHA_E_INVAL; }
            for (int d = 0; d < cfg->n_dm; ++d) {
                const fewha_dm& D = cfg->dms[d];
                pl.fd_aff.push_back(Affine{(x0 + tx * D.height - D.origin_x) / D.spacing + 0.5 * (D.n - 1), dp / D.spacing,
                                           (x0 + ty * D.height - D.origin_y) / D.spacing + 0.5 * (D.n - 1), dp / D.spacing});
            }
            for (const fewha_layer& Ly : c.layers)
                pl.fl_aff.push_back(Affine{(x0 + tx * Ly.height - Ly.origin_x) / Ly.spacing + 0.5 * (Ly.n - 1), dp / Ly.spacing,
                                           (x0 + ty * Ly.height - Ly.origin_y) / Ly.spacing + 0.5 * (Ly.n - 1), dp / Ly.spacing});
        }
    }
    return FEWHA_OK;
}

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

// Workspace layout of a plan (offsets into the loop's workspace).
void layout(fewha_loop& lp, const LoopPlan& pl, const fewha::Ctx& c, int ndir) {
    size_t o = 0;
    auto take = [&](size_t b) { const size_t r = o; o += a256(std::max<size_t>(b, 1)); return r; };
    lp.o_soff = take(sizeof(int64_t) * pl.soff.size());
    lp.o_nsub = take(sizeof(int32_t) * pl.nsub.size());
    lp.o_dms = take(sizeof(Grid) * pl.dms.size());
    lp.o_lays = take(sizeof(Grid) * pl.lays.size());
    lp.o_sd_aff = take(sizeof(Affine) * pl.sd_aff.size());
    lp.o_dir_aff = take(sizeof(Affine) * pl.dir_aff.size());
    lp.o_fd_aff = take(sizeof(Affine) * pl.fd_aff.size());
    lp.o_fl_aff = take(sizeof(Affine) * pl.fl_aff.size());
    lp.o_pts = take(sizeof(int2) * pl.pts.size());
    lp.o_pmap = take(sizeof(int32_t) * pl.pmap.size());
    const size_t e = c.esz;
    for (int k = 0; k < 4; ++k) lp.o_cmd[k] = take(e * pl.n_act);
    lp.o_r = take(e * pl.n_act);
    lp.o_p = take(e * pl.n_act);
    lp.o_q = take(e * pl.n_act);
    lp.o_b = take(e * pl.n_act);
    lp.o_pup = take(e * pl.pts.size() * std::max(ndir, 1));
    lp.o_nodal = take(e * size_t(c.N));
    lp.o_spol = take(e * size_t(c.S));
    lp.o_scal = take(sizeof(double) * 8);
    lp.total = o;
}

template <typename T>
hipError_t enqueue_fit(const fewha_loop& lp, const T* phi, T* x, hipStream_t s) {
    const int nd = lp.nd;
    const Grid* dms = lp.at<Grid>(lp.o_dms);
    if (lp.fit_iter == 0) {
        fewha::k_fit_direct<T><<<fewha::cdiv64(lp.n_act, 256), 256, 0, s>>>(dms, nd, lp.at<Grid>(lp.o_lays),
                                                                          lp.at<Affine>(lp.o_dir_aff), phi, lp.n_act, x);
        return hipGetLastError();
    }
    const int2* pts = lp.at<int2>(lp.o_pts);
    const int64_t npp = int64_t(lp.npts) * lp.ndir;
    T* pup = lp.at<T>(lp.o_pup);
    T *r = lp.at<T>(lp.o_r), *p = lp.at<T>(lp.o_p), *q = lp.at<T>(lp.o_q), *b = lp.at<T>(lp.o_b);
    double* scal = lp.at<double>(lp.o_scal);
    auto adj = [&](T* out) {
        fewha::k_fit_adj<T><<<fewha::cdiv64(lp.n_act, 256), 256, 0, s>>>(dms, nd, lp.at<Affine>(lp.o_fd_aff),
                                                                        lp.at<int32_t>(lp.o_pmap), lp.n_pts, lp.npts,
                                                                        lp.ndir, lp.n_act, pup, out);
    };
    auto dm_proj = [&](const T* v) {
        fewha::k_fit_project<T><<<fewha::cdiv64(npp, 256), 256, 0, s>>>(dms, nd, lp.at<Affine>(lp.o_fd_aff), pts,
                                                                       lp.npts, lp.ndir, v, pup);
    };
    // right-hand side sum_theta P_theta^T (layers seen along theta), then r = b - A x
    fewha::k_fit_project<T><<<fewha::cdiv64(npp, 256), 256, 0, s>>>(lp.at<Grid>(lp.o_lays), lp.L,
                                                                   lp.at<Affine>(lp.o_fl_aff), pts, lp.npts, lp.ndir,
                                                                   phi, pup);
    adj(b);
    dm_proj(x);
    adj(q);
    fewha::k_cg_init<T><<<1, fewha::kCgThreads, 0, s>>>(lp.n_act, b, q, r, p, scal);
    for (int it = 0; it < lp.fit_iter; ++it) {
        dm_proj(p);
        adj(q);
        fewha::k_cg_step<T><<<1, fewha::kCgThreads, 0, s>>>(lp.n_act, x, r, p, q, scal);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t enqueue_dm_slopes(const fewha_loop& lp, const T* a, const T* in, T* out, hipStream_t s) {
    const fewha::Ctx& c = lp.ctx->c;
    fewha::k_dm_slopes<T><<<fewha::cdiv64(lp.S, 256), 256, 0, s>>>(
        lp.at<int64_t>(lp.o_soff), lp.at<int32_t>(lp.o_nsub), lp.G, lp.S, lp.at<Grid>(lp.o_dms), lp.nd,
        lp.at<Affine>(lp.o_sd_aff), a, c.at<T>(c.lay.weight), in, out);
    return hipGetLastError();
}

template <typename T>
fewha_status loop_step(fewha_loop* lp, const void* d_s, void* d_a, void* d_info, hipStream_t s) {
    const fewha::Ctx& c = lp->ctx->c;
    const T* slopes = static_cast<const T*>(d_s);
    if (lp->closed) {
        if (enqueue_dm_slopes<T>(*lp, lp->at<T>(lp->o_cmd[lp->prev]), slopes, lp->at<T>(lp->o_spol), s) != hipSuccess)
            return loop_fail(lp, FEWHA_E_HIP, "launch of the pseudo-open-loop slopes failed");
        slopes = lp->at<T>(lp->o_spol);
    }
    const fewha_status st = fewha_solve_aug(lp->ctx, slopes, nullptr, d_info, s);
    if (st != FEWHA_OK && st != FEWHA_E_BREAKDOWN) return loop_fail(lp, st, fewha_last_error(lp->ctx));
    T* phi = lp->at<T>(lp->o_nodal);
    fewha::launch_winv<T>(c, c.at<T>(c.lay.c), phi, s);
    if (enqueue_fit<T>(*lp, phi, lp->at<T>(lp->o_cmd[lp->fit]), s) != hipSuccess)
        return loop_fail(lp, FEWHA_E_HIP, "launch of the fitting failed");
    fewha::k_gain<T><<<fewha::cdiv64(lp->n_act, 256), 256, 0, s>>>(
        lp->n_act, lp->at<T>(lp->o_cmd[lp->prev]), lp->at<T>(lp->o_cmd[lp->cur]), lp->at<T>(lp->o_cmd[lp->fit]),
        lp->at<T>(lp->o_cmd[lp->spare]), lp->gain, lp->closed);
    if (hipGetLastError() != hipSuccess) return loop_fail(lp, FEWHA_E_HIP, "launch of the gain control failed");
    // a^(i-1) <- a^(i), a^(i) <- the new commands
    const int old_prev = lp->prev;
    lp->prev = lp->cur;
    lp->cur = lp->spare;
    lp->spare = old_prev;
    if (d_a && hipMemcpyAsync(d_a, lp->at<T>(lp->o_cmd[lp->cur]), sizeof(T) * lp->n_act, hipMemcpyDeviceToDevice, s) !=
                   hipSuccess)
        return loop_fail(lp, FEWHA_E_HIP, "copy of the commands failed");
    return st;
}

}  // namespace

extern "C" {

fewha_status fewha_loop_workspace_size(const fewha_ctx* ctx, const fewha_loop_config* cfg, size_t* bytes) {
    LoopPlan pl;
    std::string err;
    const fewha_status st = plan_loop(ctx, cfg, pl, err);
    if (st != FEWHA_OK) {
        g_loop_err = err;
        return st;
    }
    if (!bytes) return FEWHA_E_INVAL;
    fewha_loop tmp;
    layout(tmp, pl, ctx->c, cfg->fit_iter ? cfg->n_dirs : 0);
    *bytes = tmp.total;
    return FEWHA_OK;
}

fewha_status fewha_loop_setup(fewha_ctx* ctx, const fewha_loop_config* cfg, void* d_workspace, size_t bytes,
                              void* stream, fewha_loop** out) {
    if (!out) return FEWHA_E_INVAL;
    *out = nullptr;
    LoopPlan pl;
    std::string err;
    fewha_status st = plan_loop(ctx, cfg, pl, err);
    if (st != FEWHA_OK) {
        g_loop_err = err;
        return st;
    }
    fewha_loop* lp = new (std::nothrow) fewha_loop();
    if (!lp) return FEWHA_E_NOMEM;
    const fewha::Ctx& c = ctx->c;
    lp->ctx = ctx;
    lp->nd = cfg->n_dm;
    lp->G = c.G;
    lp->L = c.L;
    lp->fit_iter = cfg->fit_iter;
    lp->ndir = cfg->fit_iter ? cfg->n_dirs : 0;
    lp->n_pts = cfg->fit_iter ? cfg->n_pts : 0;
    lp->npts = int(pl.pts.size());
    lp->closed = cfg->closed ? 1 : 0;
    lp->gain = cfg->gain;
    lp->n_act = pl.n_act;
    lp->N = c.N;
    lp->S = c.S;
    lp->esz = c.esz;
    layout(*lp, pl, c, lp->ndir);
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255) || bytes < lp->total) {
        g_loop_err = "the loop workspace must be 256-byte aligned and at least " + std::to_string(lp->total) + " bytes";
        delete lp;
        return bytes < lp->total ? FEWHA_E_NOMEM : FEWHA_E_INVAL;
    }
    lp->ws = static_cast<char*>(d_workspace);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    auto up = [&](size_t dst, const void* src, size_t b) {
        return b == 0 || hipMemcpyAsync(lp->ws + dst, src, b, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    bool ok = hipMemsetAsync(lp->ws, 0, lp->total, s) == hipSuccess &&
              up(lp->o_soff, pl.soff.data(), sizeof(int64_t) * pl.soff.size()) &&
              up(lp->o_nsub, pl.nsub.data(), sizeof(int32_t) * pl.nsub.size()) &&
              up(lp->o_dms, pl.dms.data(), sizeof(Grid) * pl.dms.size()) &&
              up(lp->o_lays, pl.lays.data(), sizeof(Grid) * pl.lays.size()) &&
              up(lp->o_sd_aff, pl.sd_aff.data(), sizeof(Affine) * pl.sd_aff.size()) &&
              up(lp->o_dir_aff, pl.dir_aff.data(), sizeof(Affine) * pl.dir_aff.size()) &&
              up(lp->o_fd_aff, pl.fd_aff.data(), sizeof(Affine) * pl.fd_aff.size()) &&
              up(lp->o_fl_aff, pl.fl_aff.data(), sizeof(Affine) * pl.fl_aff.size()) &&
              up(lp->o_pts, pl.pts.data(), sizeof(int2) * pl.pts.size()) &&
              up(lp->o_pmap, pl.pmap.data(), sizeof(int32_t) * pl.pmap.size());
    if (ok) ok = hipStreamSynchronize(s) == hipSuccess;   // the host tables die at return
    if (!ok) {
        g_loop_err = "upload of the loop tables failed";
        delete lp;
        return FEWHA_E_HIP;
    }
    *out = lp;
    return FEWHA_OK;
}

fewha_status fewha_loop_num_actuators(const fewha_loop* loop, int64_t* n) {
    if (!loop || !n) return FEWHA_E_INVAL;
    *n = loop->n_act;
    return FEWHA_OK;
}

fewha_status fewha_loop_step(fewha_loop* loop, const void* d_s, void* d_a, void* d_info, void* stream) {
    if (!loop || !d_s) return loop_fail(loop, FEWHA_E_INVAL, "NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return loop->esz == 8 ? loop_step<double>(loop, d_s, d_a, d_info, s) : loop_step<float>(loop, d_s, d_a, d_info, s);
}

fewha_status fewha_loop_piece(fewha_loop* loop, int32_t piece, const void* d_in, void* d_out, void* stream) {
    if (!loop || !d_in || !d_out) return loop_fail(loop, FEWHA_E_INVAL, "NULL argument");
    if (d_in == d_out) return loop_fail(loop, FEWHA_E_INVAL, "d_out must not alias d_in");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const fewha::Ctx& c = loop->ctx->c;
    auto run = [&](auto tag) -> hipError_t {
        using T = decltype(tag);
        if (piece == FEWHA_LOOP_DM_SLOPES)
            return enqueue_dm_slopes<T>(*loop, static_cast<const T*>(d_in), static_cast<const T*>(nullptr),
                                        static_cast<T*>(d_out), s);
        T* phi = loop->at<T>(loop->o_nodal);
        fewha::launch_winv<T>(c, static_cast<const T*>(d_in), phi, s);
        hipError_t e = hipMemcpyAsync(d_out, loop->at<T>(loop->o_cmd[loop->fit]), sizeof(T) * loop->n_act,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        return enqueue_fit<T>(*loop, phi, static_cast<T*>(d_out), s);
    };
    if (piece != FEWHA_LOOP_DM_SLOPES && piece != FEWHA_LOOP_FIT) return loop_fail(loop, FEWHA_E_INVAL, "unknown piece");
    const hipError_t e = loop->esz == 8 ? run(double{}) : run(float{});
    return e == hipSuccess ? FEWHA_OK : loop_fail(loop, FEWHA_E_HIP, std::string("launch failed: ") + hipGetErrorString(e));
}

fewha_status fewha_loop_get_commands(fewha_loop* loop, int32_t which, void* d_out, void* stream) {
    if (!loop || !d_out || which < 0 || which > 2) return loop_fail(loop, FEWHA_E_INVAL, "bad argument");
    const int idx = which == 0 ? loop->prev : (which == 1 ? loop->cur : loop->fit);
    return hipMemcpyAsync(d_out, loop->ws + loop->o_cmd[idx], loop->esz * loop->n_act, hipMemcpyDeviceToDevice,
                          reinterpret_cast<hipStream_t>(stream)) == hipSuccess
               ? FEWHA_OK
               : loop_fail(loop, FEWHA_E_HIP, "copy failed");
}

fewha_status fewha_loop_set_commands(fewha_loop* loop, const void* d_prev, const void* d_cur, const void* d_fit,
                                     void* stream) {
    if (!loop) return FEWHA_E_INVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const void* src[3] = {d_prev, d_cur, d_fit};
    const int idx[3] = {loop->prev, loop->cur, loop->fit};
    for (int k = 0; k < 3; ++k)
        if (src[k] && hipMemcpyAsync(loop->ws + loop->o_cmd[idx[k]], src[k], loop->esz * loop->n_act,
                                     hipMemcpyDeviceToDevice, s) != hipSuccess)
            return loop_fail(loop, FEWHA_E_HIP, "copy failed");
    return FEWHA_OK;
}

fewha_status fewha_loop_destroy(fewha_loop* loop) {
    delete loop;
    return FEWHA_OK;
}

const char* fewha_loop_last_error(const fewha_loop* loop) {
    return loop ? loop->err.c_str() : g_loop_err.c_str();
}

}  // extern "C"
