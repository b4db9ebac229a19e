// Host-side setup of the augmented-FEWHA library: configuration checks, workspace layout,
// geometry tables of the bilinear propagation (Sec. 2), the von Karman prior D (Sec. 3) and
// the exact Jacobi preconditioner J^-1 = 1 / diag(M) (Sec. 4).  Runs once per context;
// nothing here is on the per-frame path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fewha_internal.h"

namespace fewha {

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

// Daubechies' closed form of the orthonormal 6-tap scaling filter (sum sqrt 2) and the
// wavelet filter g_m = (-1)^m h_{5-m}.
void db3(double h[6], double g[6]) {
    const double s10 = std::sqrt(10.0), r = std::sqrt(5.0 + 2.0 * s10), k = std::sqrt(2.0) / 32.0;
    const double v[6] = {1 + s10 + r, 5 + s10 + 3 * r, 10 - 2 * s10 + 2 * r,
                         10 - 2 * s10 - 2 * r, 5 + s10 - 3 * r, 1 + s10 - r};
    for (int m = 0; m < 6; ++m) h[m] = k * v[m];
    for (int m = 0; m < 6; ++m) g[m] = ((m & 1) ? -1.0 : 1.0) * h[5 - m];
}

// In-place multi-level periodic 1-D synthesis of x[0..n) (transpose of the analysis
// a_k = sum_t h_t x_{(2k+t) mod n}, d_k = sum_t g_t x_{(2k+t) mod n}, output [a | d]).
void synth1d(std::vector<double>& x, int n, int levels, const double h[6], const double g[6]) {
    std::vector<double> out(n);
    for (int lev = levels; lev >= 1; --lev) {
        const int nb = n >> (lev - 1), m = nb / 2;
        std::fill(out.begin(), out.begin() + nb, 0.0);
        for (int k = 0; k < m; ++k)
            for (int t = 0; t < 6; ++t) out[(2 * k + t) % nb] += h[t] * x[k] + g[t] * x[m + k];
        std::copy(out.begin(), out.begin() + nb, x.begin());
    }
}

// Level (1 = finest) of coefficient (row, col) of an n x n Mallat pyramid with `levels`
// levels; the approximation block reports the coarsest level.
int coef_level(int row, int col, int n, int levels) {
    const int mx = std::max(row, col);
    for (int l = 1; l <= levels; ++l) {
        const int m = n >> l;
        if (mx >= m && mx < 2 * m) return l;
    }
    return levels;
}

struct Cells {
    std::vector<int32_t> idx;   // rows then columns
    std::vector<double> frac;
};

}  // namespace

std::vector<WaveStep> wavelet_steps(const fewha_config* cfg) {
    // block sizes (> the coarse block) of the tiled wavelet levels, ascending, with their layers
    const int cb = coarse_block(cfg->precision);
    std::vector<WaveStep> st;
    for (int nb = 2 * cb; nb <= 1024; nb *= 2) {
        WaveStep w;
        w.nb = nb;
        for (int l = 0; l < cfg->n_layers; ++l) {
            const fewha_layer& L = cfg->layers[l];
            if (L.n >= nb && ilog2(L.n / nb) + 1 <= L.levels) w.layers.push_back(l);
        }
        if (!w.layers.empty()) st.push_back(w);
    }
    return st;
}

int pq_partials(const fewha_config* cfg) {
    int n = cfg->n_layers;   // coarse analysis: one workgroup per layer
    for (const WaveStep& w : wavelet_steps(cfg)) n += (w.nb / 2 / kAT) * (w.nb / 2 / kAT) * int(w.layers.size());
    return n;
}

fewha_status validate_config(const fewha_config* cfg, std::string& err) {
    if (!cfg) { err = "config is NULL"; return FEWHA_E_INVAL; }
    if (cfg->abi_version != FEWHA_ABI_VERSION) { err = "abi_version mismatch"; return FEWHA_E_INVAL; }
    if (cfg->n_layers < 1 || cfg->n_layers > FEWHA_MAX_LAYERS || !cfg->layers) { err = "n_layers out of range"; return FEWHA_E_INVAL; }
    if (cfg->n_wfs < 1 || cfg->n_wfs > FEWHA_MAX_WFS || !cfg->wfs) { err = "n_wfs out of range"; return FEWHA_E_INVAL; }
    for (int l = 0; l < cfg->n_layers; ++l) {
        const fewha_layer& L = cfg->layers[l];
        if (!is_pow2(L.n) || L.n < 8 || L.n > 1024) { err = "layer n must be a power of two in [8, 1024]"; return FEWHA_E_INVAL; }
        if (L.levels < 1 || L.levels > ilog2(L.n)) { err = "layer levels out of range"; return FEWHA_E_INVAL; }
        if (!(L.spacing > 0) || !std::isfinite(L.spacing)) { err = "layer spacing must be positive"; return FEWHA_E_INVAL; }
        if (!cfg->prior_diag && !(L.weight > 0)) { err = "layer weight must be positive for the default prior"; return FEWHA_E_INVAL; }
        if (!std::isfinite(L.height) || L.height < 0) { err = "layer height must be finite and >= 0"; return FEWHA_E_INVAL; }
    }
    for (int g = 0; g < cfg->n_wfs; ++g) {
        const fewha_wfs& W = cfg->wfs[g];
        if (W.n_sub < 1 || W.n_sub > 1024) { err = "n_sub out of range"; return FEWHA_E_INVAL; }
        if (!(W.subap > 0)) { err = "subap must be positive"; return FEWHA_E_INVAL; }
        if (!(W.lgs_height >= 0)) { err = "lgs_height must be >= 0"; return FEWHA_E_INVAL; }
        if (!W.slope_weight) { err = "slope_weight is NULL"; return FEWHA_E_INVAL; }
        for (int i = 0; i < 2 * W.n_sub * W.n_sub; ++i)
            if (!(W.slope_weight[i] >= 0) || !std::isfinite(W.slope_weight[i])) { err = "slope weights must be finite and >= 0"; return FEWHA_E_INVAL; }
        for (int l = 0; l < cfg->n_layers; ++l)
            if (W.lgs_height > 0 && cfg->layers[l].height >= W.lgs_height) { err = "a layer lies at or above a laser guide star"; return FEWHA_E_INVAL; }
    }
    if (!(cfg->alpha >= 0) || !std::isfinite(cfg->alpha)) { err = "alpha must be finite and >= 0"; return FEWHA_E_INVAL; }
    if (!cfg->prior_diag && (!(cfg->r0 > 0) || !(cfg->L0 > 0))) { err = "r0 and L0 must be positive"; return FEWHA_E_INVAL; }
    if (cfg->max_iter < 1 || cfg->max_iter > 256) { err = "max_iter out of range [1, 256]"; return FEWHA_E_INVAL; }
    if (cfg->recycle_k < 0 || cfg->recycle_k > FEWHA_MAX_RECYCLE) { err = "recycle_k out of range"; return FEWHA_E_INVAL; }
    if (cfg->recycle_mode != FEWHA_RECYCLE_PAPER && cfg->recycle_mode != FEWHA_RECYCLE_GALERKIN) { err = "bad recycle_mode"; return FEWHA_E_INVAL; }
    if (cfg->rel_tol != 0.0) { err = "rel_tol is reserved and must be 0"; return FEWHA_E_INVAL; }
    if (cfg->precision != FEWHA_FP64 && cfg->precision != FEWHA_FP32_OP_FP64_RED) { err = "bad precision"; return FEWHA_E_INVAL; }
    if (cfg->project_all && cfg->recycle_mode != FEWHA_RECYCLE_GALERKIN) { err = "project_all needs GALERKIN mode"; return FEWHA_E_INVAL; }
    // every projected sensor node must fall inside every layer grid (no padding, no wrap)
    for (int g = 0; g < cfg->n_wfs; ++g) {
        const fewha_wfs& W = cfg->wfs[g];
        for (int l = 0; l < cfg->n_layers; ++l) {
            const fewha_layer& Ly = cfg->layers[l];
            const double scale = W.lgs_height > 0 ? 1.0 - Ly.height / W.lgs_height : 1.0;
            for (int axis = 0; axis < 2; ++axis) {
                const double th = axis == 0 ? W.theta_y : W.theta_x;
                const double org = axis == 0 ? Ly.origin_y : Ly.origin_x;
                for (int j = 0; j <= W.n_sub; j += W.n_sub) {
                    const double u = (scale * (j - 0.5 * W.n_sub) * W.subap + th * Ly.height - org) / Ly.spacing + 0.5 * (Ly.n - 1);
                    if (!(u >= 0.0) || !(u <= Ly.n - 1)) {
                        err = "guide-star footprint of sensor " + std::to_string(g) + " leaves the grid of layer " + std::to_string(l);
                        return FEWHA_E_INVAL;
                    }
                }
            }
        }
    }
    return FEWHA_OK;
}

Layout compute_layout(const fewha_config* cfg) {
    Layout lo{};
    const size_t e = cfg->precision == FEWHA_FP64 ? 8 : 4;
    int64_t N = 0, S = 0, V = 0, cells = 0, ranges = 0;
    for (int l = 0; l < cfg->n_layers; ++l) N += int64_t(cfg->layers[l].n) * cfg->layers[l].n;
    for (int g = 0; g < cfg->n_wfs; ++g) {
        const int ns = cfg->wfs[g].n_sub;
        S += 2 * int64_t(ns) * ns;
        V += int64_t(ns + 1) * (ns + 1);
        for (int l = 0; l < cfg->n_layers; ++l) {
            cells += 2 * (ns + 1);
            ranges += 2 * cfg->layers[l].n;
        }
    }
    const int slots = cfg->recycle_k + cfg->max_iter;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + bytes); return r; };
    lo.layers = take(sizeof(LayerDev) * cfg->n_layers);
    lo.wfs = take(sizeof(WfsDev) * cfg->n_wfs);
    lo.pairs = take(sizeof(PairDev) * cfg->n_layers * cfg->n_wfs);
    lo.cellidx = take(sizeof(int32_t) * cells);
    lo.frac = take(e * cells);
    lo.ranges = take(2 * sizeof(int32_t) * ranges);
    lo.weight = take(e * S);
    lo.prior_a = take(e * N);
    lo.jinv = take(e * N);
    lo.nodal = take(e * N);
    lo.tmp0 = take(e * N);
    lo.tmp1 = take(e * N);
    lo.psi_nodes = take(e * V);
    lo.psi_layers = take(e * N);
    lo.vx = take(e * N);
    lo.vy = take(e * N);
    lo.c = take(e * N);
    lo.r = take(e * N);
    lo.z = take(e * N);
    lo.b = take(e * N);
    lo.b_prev = take(e * N);
    lo.s_in = take(e * S);
    lo.ring_u = take(e * N * slots);
    lo.ring_q = take(e * N * slots);
    lo.partials = take(sizeof(double) * kVecBlocks * (2 * kKMax + 8));
    lo.pq_part = take(sizeof(double) * size_t(pq_partials(cfg)));
    lo.gram_part = take(sizeof(double) * kGramBlocks * (kKMax * kKMax + kKMax));
    lo.scalars = take(sizeof(Scalars));
    lo.info = take(sizeof(fewha_solve_info));
    lo.total = o;
    lo.state_bytes = 256 + sizeof(double) * slots + e * N * (3 + 2 * size_t(slots));
    return lo;
}

fewha_status build_tables(Ctx& ctx, const fewha_config* cfg, hipStream_t stream) {
    const int L = cfg->n_layers, G = cfg->n_wfs;
    const bool f32 = cfg->precision == FEWHA_FP32_OP_FP64_RED;
    double h[6], g6[6];
    db3(h, g6);

    // ---- descriptors
    std::vector<LayerDev> ld(L);
    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
        ld[l].n = cfg->layers[l].n;
        ld[l].levels = cfg->layers[l].levels;
        ld[l].coarse_lev = coarse_first_level(ld[l].n, coarse_block(cfg->precision));
        ld[l].pad_ = 0;
        ld[l].off = off;
        ld[l].inv_delta = 1.0 / cfg->layers[l].spacing;
        off += int64_t(ld[l].n) * ld[l].n;
    }
    std::vector<WfsDev> wd(G);
    int64_t soff = 0, noff = 0;
    int toff = 0;
    for (int g = 0; g < G; ++g) {
        const int ns = cfg->wfs[g].n_sub;
        wd[g].ns = ns;
        wd[g].tiles_x = (ns + 1 + kTile - 1) / kTile;
        wd[g].tile_off = toff;
        wd[g].pad_ = 0;
        wd[g].soff = soff;
        wd[g].noff = noff;
        toff += wd[g].tiles_x * wd[g].tiles_x;
        soff += 2 * int64_t(ns) * ns;
        noff += int64_t(ns + 1) * (ns + 1);
    }
    ctx.fwd_tiles = toff;

    // ---- bilinear cells of every (sensor, layer) pair, Sec. 2: the layer point seen from
    // node x is (1 - h/H) x + theta h (H = infinity for a natural guide star)
    std::vector<PairDev> pd(size_t(G) * L);
    std::vector<int32_t> cidx;
    std::vector<double> cfrac;
    std::vector<int32_t> rng;
    for (int g = 0; g < G; ++g) {
        const fewha_wfs& W = cfg->wfs[g];
        const int ns = W.n_sub;
        for (int l = 0; l < L; ++l) {
            const fewha_layer& Ly = cfg->layers[l];
            const double scale = W.lgs_height > 0 ? 1.0 - Ly.height / W.lgs_height : 1.0;
            PairDev& p = pd[size_t(g) * L + l];
            p.fwd_off = int64_t(cidx.size());
            p.rng_off = int64_t(rng.size() / 2);
            for (int axis = 0; axis < 2; ++axis) {            // 0: rows (y), 1: columns (x)
                const double th = axis == 0 ? W.theta_y : W.theta_x;
                const double org = axis == 0 ? Ly.origin_y : Ly.origin_x;
                std::vector<int32_t> c0(ns + 1);
                for (int j = 0; j <= ns; ++j) {
                    const double x = (j - 0.5 * ns) * W.subap;
                    const double u = (scale * x + th * Ly.height - org) / Ly.spacing + 0.5 * (Ly.n - 1);
                    if (!(u >= 0.0) || !(u <= Ly.n - 1)) {
                        ctx.err = "guide-star footprint of sensor " + std::to_string(g) + " leaves the grid of layer " + std::to_string(l);
                        return FEWHA_E_INVAL;
                    }
                    int i0 = int(std::floor(u));
                    if (i0 > Ly.n - 2) i0 = Ly.n - 2;
                    c0[j] = i0;
                    cidx.push_back(i0);
                    cfrac.push_back(u - i0);
                }
                // gather ranges of the adjoint: nodes j with cell c0[j] in {a-1, a}
                for (int a = 0; a < Ly.n; ++a) {
                    int first = -1, last = -2;
                    for (int j = 0; j <= ns; ++j)
                        if (c0[j] == a || c0[j] == a - 1) {
                            if (first < 0) first = j;
                            last = j;
                        }
                    rng.push_back(first < 0 ? 0 : first);
                    rng.push_back(first < 0 ? 0 : last - first + 1);
                }
            }
        }
    }
    ctx.n_cells = int64_t(cidx.size());
    ctx.max_rng = 0;
    for (size_t i = 1; i < rng.size(); i += 2) ctx.max_rng = std::max(ctx.max_rng, int(rng[i]));
    ctx.steps = wavelet_steps(cfg);
    ctx.npq = pq_partials(cfg);
    ctx.n_ranges = int64_t(rng.size() / 2);

    // ---- prior D (Sec. 3): inverse von Karman spectrum at the band frequency
    const int64_t N = ctx.N;
    std::vector<double> D(N);
    if (cfg->prior_diag) {
        std::memcpy(D.data(), cfg->prior_diag, sizeof(double) * N);
    } else {
        for (int l = 0; l < L; ++l) {
            const fewha_layer& Ly = cfg->layers[l];
            const int n = Ly.n, J = ilog2(n);
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    const int lev = coef_level(a, b, n, Ly.levels);
                    const double f = std::ldexp(1.0, J - lev) / (n * Ly.spacing);
                    D[ld[l].off + int64_t(a) * n + b] =
                        std::pow(f * f + 1.0 / (cfg->L0 * cfg->L0), 11.0 / 6.0) *
                        std::pow(cfg->r0, 5.0 / 3.0) / (0.023 * Ly.weight);
                }
        }
    }

    // ---- Jacobi preconditioner: diag(M)_i = alpha D_i + ||C^-1/2 A W^-1 e_i||^2.  The
    // wavelet basis function of coefficient (a, b) at level lev is the outer product of two
    // 1-D level-lev functions; bilinear propagation and both slope components keep that
    // product form, so every diagonal block is a pair of small matrix products.
    std::vector<double> Jinv(N);
    if (cfg->precond_inv) {
        std::memcpy(Jinv.data(), cfg->precond_inv, sizeof(double) * N);
    } else {
        std::vector<double> diag(N, 0.0);
        for (int l = 0; l < L; ++l) {
            const fewha_layer& Ly = cfg->layers[l];
            const int n = Ly.n;
            for (int lev = 1; lev <= Ly.levels; ++lev) {
                const int m2 = n >> (lev - 1);
                // basis functions B[p][y], p < m2
                std::vector<double> B(size_t(m2) * n);
                std::vector<double> tmp(n);
                for (int p = 0; p < m2; ++p) {
                    std::fill(tmp.begin(), tmp.end(), 0.0);
                    tmp[p] = 1.0;
                    synth1d(tmp, n, lev, h, g6);
                    std::copy(tmp.begin(), tmp.end(), B.begin() + size_t(p) * n);
                }
                std::vector<double> blk(size_t(m2) * m2, 0.0);
                for (int g = 0; g < G; ++g) {
                    const fewha_wfs& W = cfg->wfs[g];
                    const int ns = W.n_sub;
                    const PairDev& p = pd[size_t(g) * L + l];
                    // interpolated 1-D functions at the sensor nodes, rows (y) and columns (x)
                    std::vector<double> Yh(size_t(ns + 1) * m2), Xh(size_t(ns + 1) * m2);
                    for (int axis = 0; axis < 2; ++axis) {
                        std::vector<double>& H = axis == 0 ? Yh : Xh;
                        for (int i = 0; i <= ns; ++i) {
                            const int c0 = cidx[p.fwd_off + axis * (ns + 1) + i];
                            const double f = cfrac[p.fwd_off + axis * (ns + 1) + i];
                            for (int q = 0; q < m2; ++q)
                                H[size_t(i) * m2 + q] = (1 - f) * B[size_t(q) * n + c0] + f * B[size_t(q) * n + c0 + 1];
                        }
                    }
                    // s^x_ij = avg_y(i) * diff_x(j), s^y_ij = diff_y(i) * avg_x(j)
                    std::vector<double> Sy2(size_t(ns) * m2), Dy2(size_t(ns) * m2), Sx2(size_t(ns) * m2), Dx2(size_t(ns) * m2);
                    for (int i = 0; i < ns; ++i)
                        for (int q = 0; q < m2; ++q) {
                            const double y0 = Yh[size_t(i) * m2 + q], y1 = Yh[size_t(i + 1) * m2 + q];
                            const double x0 = Xh[size_t(i) * m2 + q], x1 = Xh[size_t(i + 1) * m2 + q];
                            Sy2[size_t(i) * m2 + q] = 0.25 * (y0 + y1) * (y0 + y1);
                            Dy2[size_t(i) * m2 + q] = (y1 - y0) * (y1 - y0);
                            Sx2[size_t(i) * m2 + q] = 0.25 * (x0 + x1) * (x0 + x1);
                            Dx2[size_t(i) * m2 + q] = (x1 - x0) * (x1 - x0);
                        }
                    const double* wx = W.slope_weight;
                    const double* wy = W.slope_weight + size_t(ns) * ns;
                    std::vector<double> T1(size_t(ns) * m2), T2(size_t(ns) * m2);
                    for (int i = 0; i < ns; ++i)
                        for (int q = 0; q < m2; ++q) {
                            double s1 = 0, s2 = 0;
                            for (int j = 0; j < ns; ++j) {
                                s1 += wx[size_t(i) * ns + j] * Dx2[size_t(j) * m2 + q];
                                s2 += wy[size_t(i) * ns + j] * Sx2[size_t(j) * m2 + q];
                            }
                            T1[size_t(i) * m2 + q] = s1;
                            T2[size_t(i) * m2 + q] = s2;
                        }
                    for (int a = 0; a < m2; ++a)
                        for (int b = 0; b < m2; ++b) {
                            if (coef_level(a, b, n, Ly.levels) != lev) continue;
                            double s = 0;
                            for (int i = 0; i < ns; ++i)
                                s += Sy2[size_t(i) * m2 + a] * T1[size_t(i) * m2 + b] + Dy2[size_t(i) * m2 + a] * T2[size_t(i) * m2 + b];
                            blk[size_t(a) * m2 + b] += s;
                        }
                }
                const double id2 = 1.0 / (Ly.spacing * Ly.spacing);
                for (int a = 0; a < m2; ++a)
                    for (int b = 0; b < m2; ++b)
                        if (coef_level(a, b, n, Ly.levels) == lev)
                            diag[ld[l].off + int64_t(a) * n + b] = blk[size_t(a) * m2 + b] * id2;
            }
        }
        for (int64_t i = 0; i < N; ++i) {
            const double d = diag[i] + cfg->alpha * D[i];
            if (!(d > 0) || !std::isfinite(d)) {
                ctx.err = "diag(M) is not positive at index " + std::to_string(i);
                return FEWHA_E_NOT_SPD;
            }
            Jinv[i] = 1.0 / d;
        }
    }

    // ---- upload (typed copies of the floating tables)
    const Layout& lo = ctx.lay;
    auto up = [&](size_t dst, const void* src, size_t bytes) -> bool {
        return hipMemcpyAsync(ctx.ws + dst, src, bytes, hipMemcpyHostToDevice, stream) == hipSuccess;
    };
    auto typed = [&](const std::vector<double>& v, double scale) {
        std::vector<char> out(v.size() * ctx.esz);
        if (f32) {
            float* o = reinterpret_cast<float*>(out.data());
            for (size_t i = 0; i < v.size(); ++i) o[i] = float(v[i] * scale);
        } else {
            double* o = reinterpret_cast<double*>(out.data());
            for (size_t i = 0; i < v.size(); ++i) o[i] = v[i] * scale;
        }
        return out;
    };
    std::vector<double> wts;
    for (int g = 0; g < G; ++g) {
        const int ns = cfg->wfs[g].n_sub;
        wts.insert(wts.end(), cfg->wfs[g].slope_weight, cfg->wfs[g].slope_weight + 2 * ns * ns);
    }
    const auto frac_t = typed(cfrac, 1.0);
    const auto w_t = typed(wts, 1.0);
    const auto pa_t = typed(D, cfg->alpha);
    const auto j_t = typed(Jinv, 1.0);
    bool ok = up(lo.layers, ld.data(), sizeof(LayerDev) * L) && up(lo.wfs, wd.data(), sizeof(WfsDev) * G) &&
              up(lo.pairs, pd.data(), sizeof(PairDev) * pd.size()) &&
              up(lo.cellidx, cidx.data(), sizeof(int32_t) * cidx.size()) && up(lo.frac, frac_t.data(), frac_t.size()) &&
              up(lo.ranges, rng.data(), sizeof(int32_t) * rng.size()) && up(lo.weight, w_t.data(), w_t.size()) &&
              up(lo.prior_a, pa_t.data(), pa_t.size()) && up(lo.jinv, j_t.data(), j_t.size());
    if (ok) ok = hipStreamSynchronize(stream) == hipSuccess;   // host vectors die at return
    if (!ok) { ctx.err = "hipMemcpyAsync of the setup tables failed"; return FEWHA_E_HIP; }
    return FEWHA_OK;
}

}  // namespace fewha
