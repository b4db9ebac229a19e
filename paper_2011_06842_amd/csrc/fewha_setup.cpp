// Host-side setup of the augmented-FEWHA library: configuration checks, workspace layout,
// geometry tables of the bilinear propagation (Sec. 2), the von Karman prior D (Sec. 3) and
// the exact Jacobi preconditioner J^-1 = 1 / diag(M) (Sec. 4).  Runs once per context;
// nothing here is on the per-frame path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "fewha_internal.h"

namespace fewha {

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Workgroup table that gives die x (workgroups x, x + kXcds, ...) the x-th contiguous share of
// `items`, so that neighbouring tiles share one die's L2; padding entries are (-1, 0).
template <typename Item>
std::vector<Item> die_order(const std::vector<Item>& items) {
    const int T = int(items.size()), grid = round_up(std::max(T, 1), kXcds), per = grid / kXcds;
    Item pad{};
    pad.x = -1;   // padding: the kernels return at once
    std::vector<Item> out(grid, pad);
    for (int b = 0; b < grid; ++b) {
        const int e = (b % kXcds) * per + b / kXcds;
        if (e < T) out[b] = items[e];
    }
    return out;
}

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

}  // namespace

namespace {

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
        {
            const int n2 = W.n_sub * W.n_sub;
            double gx = 0, gy = 0, gc = 0;
            for (int i = 0; i < n2; ++i) {
                const double wx = W.slope_weight[i], wy = W.slope_weight[n2 + i], wc = W.cross_weight ? W.cross_weight[i] : 0.0;
                if (!std::isfinite(wc)) { err = "cross weights must be finite"; return FEWHA_E_INVAL; }
                if (wx == 0 && wy == 0 && wc != 0) { err = "cross weight on an inactive subaperture"; return FEWHA_E_INVAL; }
                if (wx * wy - wc * wc < -1e-12 * wx * wy) {
                    err = "the 2x2 noise block of subaperture " + std::to_string(i) + " is not positive semi-definite";
                    return FEWHA_E_INVAL;
                }
                gx += wx;
                gy += wy;
                gc += wc;
            }
            if (W.tt_filter != 0 && W.tt_filter != 1) { err = "tt_filter must be 0 or 1"; return FEWHA_E_INVAL; }
            if (W.tt_filter && !(gx > 0 && gy > 0 && gx * gy - gc * gc > 1e-12 * gx * gy)) {
                err = "tip/tilt filter: T^T B T is singular";
                return FEWHA_E_INVAL;
            }
        }
        for (int l = 0; l < cfg->n_layers; ++l)
            if (W.lgs_height > 0 && cfg->layers[l].height >= W.lgs_height) { err = "a layer lies at or above a laser guide star"; return FEWHA_E_INVAL; }
    }
    if (!(cfg->alpha >= 0) || !std::isfinite(cfg->alpha)) { err = "alpha must be finite and >= 0"; return FEWHA_E_INVAL; }
    if (!cfg->prior_diag && (!(cfg->r0 > 0) || !(cfg->L0 > 0))) { err = "r0 and L0 must be positive"; return FEWHA_E_INVAL; }
    if (cfg->max_iter < 1 || cfg->max_iter > 256) { err = "max_iter out of range [1, 256]"; return FEWHA_E_INVAL; }
    if (cfg->recycle_k < 0 || cfg->recycle_k > FEWHA_MAX_RECYCLE) { err = "recycle_k out of range"; return FEWHA_E_INVAL; }
    if (cfg->recycle_mode != FEWHA_RECYCLE_PAPER && cfg->recycle_mode != FEWHA_RECYCLE_GALERKIN) { err = "bad recycle_mode"; return FEWHA_E_INVAL; }
    if (!(cfg->rel_tol >= 0.0) || !(cfg->rel_tol < 1.0)) { err = "rel_tol must be in [0, 1)"; return FEWHA_E_INVAL; }
    if (cfg->precision != FEWHA_FP64 && cfg->precision != FEWHA_FP32_OP_FP64_RED) { err = "bad precision"; return FEWHA_E_INVAL; }
    if (cfg->project_all && cfg->recycle_mode != FEWHA_RECYCLE_GALERKIN) { err = "project_all needs GALERKIN mode"; return FEWHA_E_INVAL; }
    if (cfg->block_elems != 0 && (cfg->block_elems < 64 || cfg->block_elems > (1 << 22))) { err = "block_elems must be 0 or in [64, 2^22]"; return FEWHA_E_INVAL; }
    // a caller-given prior or preconditioner must keep M (and J) symmetric positive definite
    {
        int64_t n_coef = 0;
        for (int l = 0; l < cfg->n_layers; ++l) n_coef += int64_t(cfg->layers[l].n) * cfg->layers[l].n;
        for (int64_t i = 0; cfg->prior_diag && i < n_coef; ++i)
            if (!(cfg->prior_diag[i] > 0) || !std::isfinite(cfg->prior_diag[i])) {
                err = "prior_diag must be finite and > 0 (entry " + std::to_string(i) + ")";
                return FEWHA_E_INVAL;
            }
        if (cfg->level_weight && !cfg->precond_inv) {
            int lmax = 0;
            for (int l = 0; l < cfg->n_layers; ++l) lmax = std::max(lmax, cfg->layers[l].levels);
            for (int j = 0; j <= lmax; ++j)
                if (!(cfg->level_weight[j] > 0) || !std::isfinite(cfg->level_weight[j])) {
                    err = "level_weight must be finite and > 0 (entry " + std::to_string(j) + ")";
                    return FEWHA_E_INVAL;
                }
        }
        for (int64_t i = 0; cfg->precond_inv && i < n_coef; ++i)
            if (!(cfg->precond_inv[i] > 0) || !std::isfinite(cfg->precond_inv[i])) {
                err = "precond_inv must be finite and > 0 (entry " + std::to_string(i) + ")";
                return FEWHA_E_INVAL;
            }
    }
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

// Derived sizes of one instance and of the batch (identical for validation, layout and setup).
struct Sizes {
    int B = 0, L = 0, G = 0, slots = 0, esz = 8, KE = 1;
    int64_t N = 0, S = 0, V = 0, cells = 0, ranges = 0, pairs = 0;   // pairs: also the record bases
    int VB = 0, GB = 0, NPQ = 0, data_tiles = 0, gather_tiles1 = 0, gather_tiles4 = 0, gather_rows = 1;
    int syn_small = 0, syn_large = 0, syn_huge = 0, ana_items = 0, ana_groups = 0;
    int64_t gwin = 0;   // gather windows: (layer tile, sensor of its instance) pairs
    std::vector<StepInfo> steps;
};

int gather_tiles_of(int n, int rows) {
    const int tr = kGRowStep * rows;
    return ((n + tr - 1) / tr) * ((n + kGT - 1) / kGT);
}

int block_elems(const fewha_config* c) { return c->block_elems ? c->block_elems : kDefaultBlockElems; }

int vec_blocks(int64_t n, int be) { return int(std::min<int64_t>(kVecBlocksMax, std::max<int64_t>(1, (n + be - 1) / be))); }

// Gram workgroups of an instance: a function of its size alone, so that an instance of a batch
// sums its Gram partials exactly as the same instance alone does.
int gram_blocks(int64_t n) { return int(std::min<int64_t>(kGramBlocks, std::max<int64_t>(1, (n + kGramElems - 1) / kGramElems))); }

// Tiled analysis levels of one layer: for every group of block sizes above the coarse block
// (groups of kmax consecutive sizes counted from the coarse end, one launch each) the layer has
// levels in, its first level there and their count; finest first.
struct AnaSeg {
    int g, l1, k;
};
std::vector<AnaSeg> ana_segments(int n, int levels, int cb, int kmax) {
    std::vector<AnaSeg> out;
    const int last = std::min(levels, coarse_first_level(n, cb) - 1);
    for (int lev = 1; lev <= last; ++lev) {
        const int g = (ilog2(n >> (lev - 1)) - ilog2(cb) - 1) / kmax;
        if (out.empty() || out.back().g != g) out.push_back(AnaSeg{g, lev, 1});
        else ++out.back().k;
    }
    return out;
}

// workgroups (tiles of the segment's last level) of one segment
int seg_tiles(int n, const AnaSeg& s) {
    const int m = (n >> (s.l1 - 1)) >> s.k, t = ana_tile(s.k);
    return (m / t) * (m / t);
}

// (p, q) partials of one layer: one per tiled analysis workgroup (launches in order), then the
// coarse one
int layer_pq(int n, int levels, int cb, int kmax) {
    int t = 0;
    for (const AnaSeg& sg : ana_segments(n, levels, cb, kmax)) t += seg_tiles(n, sg);
    return t + 1;
}

// Synthesis tiles of one layer with tile side st (n when the layer is smaller).
int syn_tiles(int n, int st) {
    const int ts = std::min(st, n);
    return (n / ts) * (n / ts);
}

Sizes batch_sizes(const fewha_config* cfgs, int nb) {
    Sizes z;
    z.B = nb;
    z.esz = cfgs[0].precision == FEWHA_FP64 ? 8 : 4;
    z.slots = cfgs[0].recycle_k + cfgs[0].max_iter;
    z.KE = std::max(1, 2 * cfgs[0].recycle_k * (cfgs[0].recycle_k + 1));   // X and Y of the Gram pass
    const int cb = coarse_block(cfgs[0].precision), kmax = ana_levels_per_launch(cfgs[0].precision);
    for (int i = 0; i < nb; ++i) {
        const fewha_config* c = &cfgs[i];
        int64_t Ni = 0;
        for (int l = 0; l < c->n_layers; ++l) {
            const int n = c->layers[l].n;
            Ni += int64_t(n) * n;
            z.NPQ += layer_pq(n, c->layers[l].levels, cb, kmax);
            z.syn_small += syn_tiles(n, kSynTile / 2);
            z.syn_large += syn_tiles(n, kSynTile);
            z.syn_huge += syn_tiles(n, 2 * kSynTile);
            for (const AnaSeg& sg : ana_segments(n, c->layers[l].levels, cb, kmax))
                z.ana_groups = std::max(z.ana_groups, sg.g + 1);
        }
        for (int g = 0; g < c->n_wfs; ++g) {
            const int ns = c->wfs[g].n_sub;
            z.S += 2 * int64_t(ns) * ns;
            z.V += int64_t(ns + 1) * (ns + 1);
            const int tx = (ns + 1 + kTile - 1) / kTile;
            z.data_tiles += tx * tx;
            for (int l = 0; l < c->n_layers; ++l) {
                z.cells += 2 * (ns + 1);
                z.ranges += 2 * c->layers[l].n;
            }
        }
        z.pairs += int64_t(c->n_layers) * c->n_wfs;
        z.L += c->n_layers;
        z.G += c->n_wfs;
        z.N += Ni;
        z.VB += vec_blocks(Ni, block_elems(c));
        z.GB += gram_blocks(Ni);
    }
    // adjoint-gather tiles: 8 x kGT nodes for small systems (more workgroups), 32 x kGT beyond
    // (both tile shapes are built; the context starts with this one, see fewha_set_tuning)
    z.gather_rows = z.N >= kGatherWide ? 4 : 1;
    for (int i = 0; i < nb; ++i)
        for (int l = 0; l < cfgs[i].n_layers; ++l) {
            z.gather_tiles1 += gather_tiles_of(cfgs[i].layers[l].n, 1);
            const int gt = gather_tiles_of(cfgs[i].layers[l].n, 4);
            z.gather_tiles4 += gt;
            z.gwin += int64_t(gt) * cfgs[i].n_wfs;
        }
    z.syn_small = round_up(z.syn_small, kXcds);
    z.syn_large = round_up(z.syn_large, kXcds);
    z.syn_huge = round_up(z.syn_huge, kXcds);
    // tiled analysis launches: one per group of block sizes that has workgroups, finest first
    for (int g = z.ana_groups - 1; g >= 0; --g) {
        StepInfo st;
        st.loff = z.ana_items;
        int items = 0;
        for (int i = 0; i < nb; ++i)
            for (int l = 0; l < cfgs[i].n_layers; ++l) {
                const fewha_layer& Ly = cfgs[i].layers[l];
                for (const AnaSeg& sg : ana_segments(Ly.n, Ly.levels, cb, kmax))
                    if (sg.g == g) {
                        items += seg_tiles(Ly.n, sg);
                        ++st.nl;
                        st.nb = std::max(st.nb, Ly.n >> (sg.l1 - 1));
                    }
            }
        if (items) {
            st.ni = round_up(items, kXcds);
            z.ana_items += st.ni;
            z.steps.push_back(st);
        }
    }
    return z;
}

}  // namespace

fewha_status validate_batch(const fewha_config* cfgs, int n, std::string& err) {
    if (!cfgs) { err = "config is NULL"; return FEWHA_E_INVAL; }
    if (n < 1 || n > FEWHA_MAX_INSTANCES) { err = "instance count out of range"; return FEWHA_E_INVAL; }
    for (int i = 0; i < n; ++i) {
        const fewha_status st = validate_config(&cfgs[i], err);
        if (st != FEWHA_OK) {
            if (n > 1) err = "instance " + std::to_string(i) + ": " + err;
            return st;
        }
        const fewha_config& a = cfgs[0];
        const fewha_config& b = cfgs[i];
        if (a.precision != b.precision || a.max_iter != b.max_iter || a.recycle_k != b.recycle_k ||
            a.recycle_mode != b.recycle_mode || a.project_all != b.project_all || a.rel_tol != b.rel_tol ||
            block_elems(&a) != block_elems(&b)) {
            err = "instance " + std::to_string(i) +
                  ": precision, iterations, recycling and block_elems must be the same for every instance";
            return FEWHA_E_INVAL;
        }
    }
    return FEWHA_OK;
}

Layout compute_layout(const fewha_config* cfgs, int nb) {
    const Sizes z = batch_sizes(cfgs, nb);
    Layout lo{};
    const size_t e = size_t(z.esz);
    const int64_t N = z.N, S = z.S, V = z.V;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + bytes); return r; };
    lo.layers = take(sizeof(LayerDev) * z.L);
    lo.wfs = take(sizeof(WfsDev) * z.G);
    lo.pairs = take(sizeof(PairDev) * z.pairs);
    lo.cellidx = take(sizeof(int32_t) * z.cells);
    lo.frac = take(e * z.cells);
    lo.ranges = take(2 * sizeof(int32_t) * z.ranges);
    lo.insts = take(sizeof(InstDev) * z.B);
    lo.vecblk = take(sizeof(VecBlk) * z.VB);
    lo.gramblk = take(sizeof(GramBlk) * z.GB);
    lo.syn_items = take(sizeof(int2) * (z.syn_small + z.syn_large + z.syn_huge));
    lo.ana_items = take(sizeof(int4) * std::max(1, z.ana_items));
    lo.data_tiles = take(sizeof(int2) * round_up(z.data_tiles, kXcds));
    lo.gather_tiles = take(sizeof(int2) * (round_up(z.gather_tiles1, kXcds) + round_up(z.gather_tiles4, kXcds)));
    lo.grecs = take((z.esz == 8 ? sizeof(GatherRec<double>) : sizeof(GatherRec<float>)) * z.ranges);
    lo.recbase = take(sizeof(int64_t) * std::max<int64_t>(1, z.pairs));
    lo.gwin = take(sizeof(int4) * std::max<int64_t>(1, z.gwin));
    lo.node_sensor = take(sizeof(int32_t) * std::max<int64_t>(1, (V + kThreads - 1) / kThreads));
    lo.weight = take(e * S);
    lo.xweight = take(e * (S / 2));
    lo.ttv = take(e * 2 * V);
    lo.prior_a = take(e * N);
    lo.jinv = take(e * N);
    lo.nodal = take(e * N);
    lo.tmp0 = take(e * N);
    lo.tmp1 = take(e * N);
    lo.psi_nodes = take(e * V);
    lo.psi_layers = take(e * N);
    lo.wslopes = take(e * S);
    lo.vx = take(e * N);
    lo.vy = take(e * N);
    lo.c = take(e * N);
    lo.r = take(e * N);
    lo.z = take(e * N);
    lo.b = take(e * N);
    lo.b_prev = take(e * N);
    lo.ring_u = take(e * N * z.slots);
    lo.ring_q = take(e * N * z.slots);
    lo.partials = take(sizeof(double) * size_t(z.VB) * (2 * kKMax + 8));
    lo.pq_part = take(sizeof(double) * size_t(z.NPQ));
    lo.gram_part = take(sizeof(double) * size_t(z.GB) * z.KE);
    lo.scalars = take(sizeof(Scalars) * z.B);
    lo.info = take(sizeof(fewha_solve_info) * z.B);
    lo.done = take(sizeof(int32_t) * z.B);
    lo.ws_in = take(sizeof(float) * 4 * N);
    lo.ws_out = take(sizeof(float) * N);
    lo.lconst = take(sizeof(float) * 2 * z.L);
    lo.total = o;
    lo.state_bytes = 256 + sizeof(double) * size_t(z.B) * (z.slots + 1) + e * N * (3 + 2 * size_t(z.slots));
    return lo;
}

namespace {

// Host tables of all instances, concatenated in instance order.
struct Tables {
    std::vector<LayerDev> ld;
    std::vector<WfsDev> wd;
    std::vector<PairDev> pd;
    std::vector<int32_t> cidx, rng;
    std::vector<double> cfrac, D, Jinv, wts;
    std::vector<double> xw;         // cross weights, n_sub^2 per sensor (slope offset / 2)
    std::vector<double> ttv;        // tip/tilt filter node vectors Gamma^T B T e_x, then e_y (V each)
    std::vector<double> ttvy;
};

// Prior D (Sec. 3): inverse von Karman spectrum at the band frequency of every coefficient.
void prior_of(const fewha_config* cfg, const LayerDev* ld, double* D) {
    for (int l = 0; l < cfg->n_layers; ++l) {
        const fewha_layer& Ly = cfg->layers[l];
        const int n = Ly.n, J = ilog2(n);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                const int lev = coef_level(a, b, n, Ly.levels);
                const double f = std::ldexp(1.0, J - lev) / (n * Ly.spacing);
                D[(ld[l].off - ld[0].off) + int64_t(a) * n + b] =
                    std::pow(f * f + 1.0 / (cfg->L0 * cfg->L0), 11.0 / 6.0) * std::pow(cfg->r0, 5.0 / 3.0) /
                    (0.023 * Ly.weight);
            }
    }
}

// diag(M) - alpha D of one instance: the wavelet basis function of coefficient (a, b) at level
// lev is the outer product of two 1-D level-lev functions; bilinear propagation and both slope
// components keep that product form, so every diagonal block is a pair of small matrix
// products.  `pair(g, l)` gives the instance-local pair's table entry.
template <typename PairOf>
void data_diag_of(const fewha_config* cfg, const LayerDev* ld, PairOf pair, const std::vector<int32_t>& cidx,
                  const std::vector<double>& cfrac, double* diag) {
    double h[6], g6[6];
    db3(h, g6);
    const int G = cfg->n_wfs;
    for (int l = 0; l < cfg->n_layers; ++l) {
        const fewha_layer& Ly = cfg->layers[l];
        const int n = Ly.n;
        for (int lev = 1; lev <= Ly.levels; ++lev) {
            const int m2 = n >> (lev - 1);
            std::vector<double> B(size_t(m2) * n);   // basis functions B[p][y], p < m2
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
                const PairDev& p = pair(g, l);
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
                const double* wc = W.cross_weight;
                // cross term 2 w_c s^x s^y: avg_y diff_y (i) times diff_x avg_x (j)
                std::vector<double> SDy(wc ? size_t(ns) * m2 : 0), DSx(wc ? size_t(ns) * m2 : 0);
                if (wc)
                    for (int i = 0; i < ns; ++i)
                        for (int q = 0; q < m2; ++q) {
                            const double y0 = Yh[size_t(i) * m2 + q], y1 = Yh[size_t(i + 1) * m2 + q];
                            const double x0 = Xh[size_t(i) * m2 + q], x1 = Xh[size_t(i + 1) * m2 + q];
                            SDy[size_t(i) * m2 + q] = 0.5 * (y0 + y1) * (y1 - y0);
                            DSx[size_t(i) * m2 + q] = (x1 - x0) * 0.5 * (x0 + x1);
                        }
                std::vector<double> T1(size_t(ns) * m2), T2(size_t(ns) * m2), T3(wc ? size_t(ns) * m2 : 0);
                for (int i = 0; i < ns; ++i)
                    for (int q = 0; q < m2; ++q) {
                        double s1 = 0, s2 = 0, s3 = 0;
                        for (int j = 0; j < ns; ++j) {
                            s1 += wx[size_t(i) * ns + j] * Dx2[size_t(j) * m2 + q];
                            s2 += wy[size_t(i) * ns + j] * Sx2[size_t(j) * m2 + q];
                            if (wc) s3 += wc[size_t(i) * ns + j] * DSx[size_t(j) * m2 + q];
                        }
                        T1[size_t(i) * m2 + q] = s1;
                        T2[size_t(i) * m2 + q] = s2;
                        if (wc) T3[size_t(i) * m2 + q] = s3;
                    }
                for (int a = 0; a < m2; ++a)
                    for (int b = 0; b < m2; ++b) {
                        if (coef_level(a, b, n, Ly.levels) != lev) continue;
                        double s = 0;
                        for (int i = 0; i < ns; ++i)
                            s += Sy2[size_t(i) * m2 + a] * T1[size_t(i) * m2 + b] + Dy2[size_t(i) * m2 + a] * T2[size_t(i) * m2 + b];
                        if (wc)
                            for (int i = 0; i < ns; ++i) s += 2.0 * SDy[size_t(i) * m2 + a] * T3[size_t(i) * m2 + b];
                        blk[size_t(a) * m2 + b] += s;
                    }
            }
            const double id2 = 1.0 / (Ly.spacing * Ly.spacing);
            for (int a = 0; a < m2; ++a)
                for (int b = 0; b < m2; ++b)
                    if (coef_level(a, b, n, Ly.levels) == lev)
                        diag[(ld[l].off - ld[0].off) + int64_t(a) * n + b] = blk[size_t(a) * m2 + b] * id2;
        }
    }
}

// Appends instance `inst` (configuration cfg) to the concatenated tables.
fewha_status add_instance(Tables& t, const fewha_config* cfg, int inst, int cb, int64_t& off, int64_t& soff,
                          int64_t& noff, int& toff, int& pqoff, std::string& err) {
    const int L = cfg->n_layers, G = cfg->n_wfs;
    const int l0 = int(t.ld.size()), g0 = int(t.wd.size());
    const int64_t off0 = off;
    for (int l = 0; l < L; ++l) {
        LayerDev d{};
        d.n = cfg->layers[l].n;
        d.levels = cfg->layers[l].levels;
        d.coarse_lev = coarse_first_level(d.n, cb);
        d.inst = inst;
        d.off = off;
        d.inv_delta = 1.0 / cfg->layers[l].spacing;
        d.l0 = l0;
        d.g0 = g0;
        d.ng = G;
        d.pq0 = pqoff;
        d.pq_coarse = layer_pq(d.n, d.levels, cb, ana_levels_per_launch(cfg->precision)) - 1;
        d.rb0 = 0;                                   // set once every pair exists (build_tables)
        pqoff += d.pq_coarse + 1;
        off += int64_t(d.n) * d.n;
        t.ld.push_back(d);
    }
    // bilinear cells of every (sensor, layer) pair, Sec. 2: the layer point seen from node x
    // is (1 - h/H) x + theta h (H = infinity for a natural guide star)
    for (int g = 0; g < G; ++g) {
        const fewha_wfs& W = cfg->wfs[g];
        const int ns = W.n_sub;
        WfsDev w{};
        w.ns = ns;
        w.tiles_x = (ns + 1 + kTile - 1) / kTile;
        w.tile_off = toff;
        w.inst = inst;
        w.soff = soff;
        w.noff = noff;
        w.l0 = l0;
        w.nl = L;
        w.pair0 = int(t.pd.size());
        w.fwd0 = int64_t(t.cidx.size());
        toff += w.tiles_x * w.tiles_x;
        soff += 2 * int64_t(ns) * ns;
        noff += int64_t(ns + 1) * (ns + 1);
        // noise blocks: cross weights, and for a tip/tilt-filtered sensor (T^T B T)^-1 and the
        // node vectors v_k = Gamma^T B T e_k (the slope adjoint of the device, on the host)
        {
            const int n2 = ns * ns, np = ns + 1;
            const double* wx = W.slope_weight;
            const double* wy = W.slope_weight + n2;
            std::vector<double> wc(n2, 0.0);
            if (W.cross_weight) std::copy(W.cross_weight, W.cross_weight + n2, wc.begin());
            t.xw.insert(t.xw.end(), wc.begin(), wc.end());
            w.tt = W.tt_filter;
            double gx = 0, gy = 0, gc = 0;
            for (int i = 0; i < n2; ++i) {
                gx += wx[i];
                gy += wy[i];
                gc += wc[i];
            }
            const double det = gx * gy - gc * gc;
            w.tg[0] = w.tt ? gy / det : 0.0;
            w.tg[1] = w.tt ? -gc / det : 0.0;
            w.tg[2] = w.tt ? gx / det : 0.0;
            for (int k = 0; k < 2; ++k) {
                // slope field B T e_k: (w_x, w_c) for tip, (w_c, w_y) for tilt
                auto tf = [&](int comp, int si, int sj) -> double {
                    if (!w.tt || si < 0 || si >= ns || sj < 0 || sj >= ns) return 0.0;
                    const int o = si * ns + sj;
                    return comp == 0 ? (k == 0 ? wx[o] : wc[o]) : (k == 0 ? wc[o] : wy[o]);
                };
                std::vector<double>& dst = k == 0 ? t.ttv : t.ttvy;
                for (int i = 0; i < np; ++i)
                    for (int j = 0; j < np; ++j)
                        dst.push_back(0.5 * ((tf(0, i, j - 1) - tf(0, i, j)) + (tf(0, i - 1, j - 1) - tf(0, i - 1, j))) +
                                      0.5 * ((tf(1, i - 1, j) - tf(1, i, j)) + (tf(1, i - 1, j - 1) - tf(1, i, j - 1))));
            }
        }
        t.wd.push_back(w);
        t.wts.insert(t.wts.end(), W.slope_weight, W.slope_weight + 2 * ns * ns);
        for (int l = 0; l < L; ++l) {
            const fewha_layer& Ly = cfg->layers[l];
            const double scale = W.lgs_height > 0 ? 1.0 - Ly.height / W.lgs_height : 1.0;
            PairDev p;
            p.fwd_off = int64_t(t.cidx.size());
            p.rng_off = int64_t(t.rng.size() / 2);
            for (int axis = 0; axis < 2; ++axis) {            // 0: rows (y), 1: columns (x)
                const double th = axis == 0 ? W.theta_y : W.theta_x;
                const double org = axis == 0 ? Ly.origin_y : Ly.origin_x;
                std::vector<int32_t> c0(ns + 1);
                for (int j = 0; j <= ns; ++j) {
                    const double x = (j - 0.5 * ns) * W.subap;
                    const double u = (scale * x + th * Ly.height - org) / Ly.spacing + 0.5 * (Ly.n - 1);
                    if (!(u >= 0.0) || !(u <= Ly.n - 1)) {
                        err = "guide-star footprint of sensor " + std::to_string(g) + " leaves the grid of layer " +
                              std::to_string(l);
                        return FEWHA_E_INVAL;
                    }
                    int i0 = int(std::floor(u));
                    if (i0 > Ly.n - 2) i0 = Ly.n - 2;
                    c0[j] = i0;
                    t.cidx.push_back(i0);
                    t.cfrac.push_back(u - i0);
                }
                // gather ranges of the adjoint: nodes j with cell c0[j] in {a-1, a}
                for (int a = 0; a < Ly.n; ++a) {
                    int first = -1, last = -2;
                    for (int j = 0; j <= ns; ++j)
                        if (c0[j] == a || c0[j] == a - 1) {
                            if (first < 0) first = j;
                            last = j;
                        }
                    t.rng.push_back(first < 0 ? 0 : first);
                    t.rng.push_back(first < 0 ? 0 : last - first + 1);
                }
            }
            t.pd.push_back(p);
        }
    }
    // prior (Sec. 3); the preconditioner follows for all instances at once (jacobi_of)
    const int64_t Ni = off - off0;
    const size_t base = t.D.size();
    t.D.resize(base + Ni);
    t.Jinv.resize(base + Ni);
    double* D = t.D.data() + base;
    if (cfg->prior_diag)
        std::memcpy(D, cfg->prior_diag, sizeof(double) * Ni);
    else
        prior_of(cfg, &t.ld[l0], D);
    if (cfg->precond_inv) std::memcpy(t.Jinv.data() + base, cfg->precond_inv, sizeof(double) * Ni);
    return FEWHA_OK;
}

// Exact Jacobi preconditioner J^-1 = 1 / diag(M) (Sec. 4) of instance i, whose coefficients
// start at `base` of the concatenation and whose first layer / sensor are l0 / g0.
fewha_status jacobi_of(Tables& t, const fewha_config* cfg, size_t base, int l0, int g0, std::string& err) {
    const int64_t Ni = [&] {
        int64_t n = 0;
        for (int l = 0; l < cfg->n_layers; ++l) n += int64_t(cfg->layers[l].n) * cfg->layers[l].n;
        return n;
    }();
    std::vector<double> diag(Ni, 0.0);
    data_diag_of(cfg, &t.ld[l0], [&](int g, int l) -> const PairDev& { return t.pd[t.wd[g0 + g].pair0 + l]; },
                 t.cidx, t.cfrac, diag.data());
    const double* D = t.D.data() + base;
    for (int64_t i = 0; i < Ni; ++i) {
        const double d = diag[i] + cfg->alpha * D[i];
        if (!(d > 0) || !std::isfinite(d)) {
            err = "diag(M) is not positive at index " + std::to_string(i);
            return FEWHA_E_NOT_SPD;
        }
        t.Jinv[base + i] = 1.0 / d;
    }
    if (cfg->level_weight) {   // modified Jacobi: a weight per wavelet level (scaling block: index levels)
        int64_t off = 0;
        for (int l = 0; l < cfg->n_layers; ++l) {
            const int n = cfg->layers[l].n, lv = cfg->layers[l].levels, nc = n >> lv;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    const int j = (a < nc && b < nc) ? lv : coef_level(a, b, n, lv) - 1;
                    t.Jinv[base + off + int64_t(a) * n + b] /= cfg->level_weight[j];
                }
            off += int64_t(n) * n;
        }
    }
    return FEWHA_OK;
}

}  // namespace

fewha_status build_tables(Ctx& ctx, const fewha_config* cfgs, int nb, hipStream_t stream) {
    const Sizes z = batch_sizes(cfgs, nb);
    const int cb = coarse_block(cfgs[0].precision);
    const bool f32 = cfgs[0].precision == FEWHA_FP32_OP_FP64_RED;
    ctx.B = nb;
    ctx.L = z.L;
    ctx.G = z.G;
    ctx.N = z.N;
    ctx.S = z.S;
    ctx.V = z.V;
    ctx.VB = z.VB;
    ctx.GB = z.GB;
    ctx.npq = z.NPQ;
    ctx.slots = z.slots;
    ctx.data_grid = round_up(std::max(z.data_tiles, 1), kXcds);
    ctx.gather_grid1 = round_up(std::max(z.gather_tiles1, 1), kXcds);
    ctx.gather_grid4 = round_up(std::max(z.gather_tiles4, 1), kXcds);
    ctx.gather_rows = z.gather_rows;
    ctx.steps = z.steps;
    ctx.block_elems = block_elems(&cfgs[0]);

    Tables t;
    int64_t off = 0, soff = 0, noff = 0;
    int toff = 0, pqoff = 0;
    ctx.insts.assign(nb, InstDev{});
    ctx.s_offs.assign(nb + 1, 0);
    std::vector<VecBlk> vb;
    std::vector<GramBlk> gb;
    std::vector<int> l0s(nb), g0s(nb);
    for (int i = 0; i < nb; ++i) {
        const int64_t off0 = off;
        const int pq0 = pqoff;
        l0s[i] = int(t.ld.size());
        g0s[i] = int(t.wd.size());
        const fewha_status st = add_instance(t, &cfgs[i], i, cb, off, soff, noff, toff, pqoff, ctx.err);
        if (st != FEWHA_OK) {
            if (nb > 1) ctx.err = "instance " + std::to_string(i) + ": " + ctx.err;
            return st;
        }
        InstDev& I = ctx.insts[i];
        I.off = off0;
        I.n = off - off0;
        I.nvb = vec_blocks(I.n, ctx.block_elems);
        I.vb0 = int(vb.size());
        I.ngb = gram_blocks(I.n);
        I.gb0 = int(gb.size());
        I.pq0 = pq0;
        I.npq = pqoff - pq0;
        for (int k = 0; k < I.nvb; ++k)
            vb.push_back(VecBlk{I.off, int32_t(I.n), k, I.nvb, i, I.vb0 + k, I.pq0, I.npq, 0});
        for (int k = 0; k < I.ngb; ++k)
            gb.push_back(GramBlk{I.off, int32_t(I.n), k, I.ngb, i, I.gb0 * z.KE, 0});
        ctx.s_offs[i + 1] = soff;
    }
    {   // exact Jacobi preconditioners, instances in parallel (a bounded pool of host threads)
        std::vector<int> todo;
        for (int i = 0; i < nb; ++i)
            if (!cfgs[i].precond_inv) todo.push_back(i);
        const int nthreads = int(std::min<size_t>(todo.size(), std::max(1u, std::min(16u, std::thread::hardware_concurrency()))));
        std::vector<fewha_status> sts(nb, FEWHA_OK);
        std::vector<std::string> errs(nb);
        std::atomic<size_t> next{0};
        auto work = [&] {
            for (size_t k = next++; k < todo.size(); k = next++) {
                const int i = todo[k];
                sts[i] = jacobi_of(t, &cfgs[i], size_t(ctx.insts[i].off), l0s[i], g0s[i], errs[i]);
            }
        };
        std::vector<std::thread> pool;
        for (int k = 1; k < nthreads; ++k) pool.emplace_back(work);
        work();
        for (auto& th : pool) th.join();
        for (int i = 0; i < nb; ++i)
            if (sts[i] != FEWHA_OK) {
                ctx.err = (nb > 1 ? "instance " + std::to_string(i) + ": " : std::string()) + errs[i];
                return sts[i];
            }
        for (int i = 0; i < nb; ++i)   // the device keeps alpha D
            for (int64_t j = 0; j < ctx.insts[i].n; ++j) t.D[ctx.insts[i].off + j] *= cfgs[i].alpha;
    }
    // host copies of the layer and sensor descriptors of all instances, in order (the slope
    // weights are read during setup only: their pointer is not kept)
    ctx.layers.clear();
    ctx.wfs.clear();
    for (int i = 0; i < nb; ++i) {
        ctx.layers.insert(ctx.layers.end(), cfgs[i].layers, cfgs[i].layers + cfgs[i].n_layers);
        for (int g = 0; g < cfgs[i].n_wfs; ++g) {
            fewha_wfs w = cfgs[i].wfs[g];
            w.slope_weight = nullptr;
            ctx.wfs.push_back(w);
        }
    }
    ctx.layers_n.clear();
    for (const LayerDev& d : t.ld) {
        ctx.layers_n.push_back(d.n);
        ctx.max_levels = std::max(ctx.max_levels, int(d.levels));
        ctx.max_n = std::max(ctx.max_n, int(d.n));
    }
    ctx.n_cells = int64_t(t.cidx.size());
    ctx.n_ranges = int64_t(t.rng.size() / 2);
    ctx.max_rng = 0;
    for (size_t i = 1; i < t.rng.size(); i += 2) ctx.max_rng = std::max(ctx.max_rng, int(t.rng[i]));
    // layers of every tiled wavelet level, and the block -> sensor / layer tables
    // synthesis tiles (half-size tiles, then full-size), die-ordered per launch
    std::vector<int2> s16, s32, s64;
    for (int l = 0; l < z.L; ++l) {
        for (int k = 0; k < syn_tiles(t.ld[l].n, kSynTile / 2); ++k) s16.push_back(make_int2(l, k));
        for (int k = 0; k < syn_tiles(t.ld[l].n, kSynTile); ++k) s32.push_back(make_int2(l, k));
        for (int k = 0; k < syn_tiles(t.ld[l].n, 2 * kSynTile); ++k) s64.push_back(make_int2(l, k));
    }
    std::vector<int2> syn = die_order(s16);
    ctx.syn_small = int(syn.size());
    {
        const std::vector<int2> o32 = die_order(s32), o64 = die_order(s64);
        ctx.syn_large = int(o32.size());
        ctx.syn_huge = int(o64.size());
        syn.insert(syn.end(), o32.begin(), o32.end());
        syn.insert(syn.end(), o64.begin(), o64.end());
    }
    // tiled analysis items (layer, tile, l1 | k << 8 | tile side << 16, partial slot) of every
    // launch, the partial slots of a layer numbered in launch and tile order
    std::vector<int4> ana;
    {
        const int kmax = ana_levels_per_launch(cfgs[0].precision);
        std::vector<int> slot(z.L, 0);
        for (int g = z.ana_groups - 1; g >= 0; --g) {
            std::vector<int4> items;
            for (int l = 0; l < z.L; ++l)
                for (const AnaSeg& sg : ana_segments(t.ld[l].n, t.ld[l].levels, cb, kmax))
                    if (sg.g == g)
                        for (int k = 0; k < seg_tiles(t.ld[l].n, sg); ++k)
                            items.push_back(make_int4(l, k, sg.l1 | (sg.k << 8) | (ana_tile(sg.k) << 16), slot[l]++));
            if (!items.empty()) {
                const std::vector<int4> o = die_order(items);
                ana.insert(ana.end(), o.begin(), o.end());
            }
        }
        for (int l = 0; l < z.L; ++l)
            if (slot[l] != t.ld[l].pq_coarse) { ctx.err = "internal: analysis partial count mismatch"; return FEWHA_E_INVAL; }
        if (int(ana.size()) != z.ana_items || int(syn.size()) != z.syn_small + z.syn_large + z.syn_huge) {
            ctx.err = "internal: wavelet item count mismatch";
            return FEWHA_E_INVAL;
        }
        if (ana.empty()) ana.push_back(make_int4(-1, 0, 0, 0));
    }
    std::vector<int2> dt_items, gt_items;
    for (int g = 0; g < z.G; ++g)
        for (int k = 0; k < t.wd[g].tiles_x * t.wd[g].tiles_x; ++k) dt_items.push_back(make_int2(g, k));
    std::vector<int2> gt_items4;
    for (int l = 0; l < z.L; ++l) {
        for (int k = 0; k < gather_tiles_of(t.ld[l].n, 1); ++k) gt_items.push_back(make_int2(l, k));
        for (int k = 0; k < gather_tiles_of(t.ld[l].n, 4); ++k) gt_items4.push_back(make_int2(l, k));
    }
    const std::vector<int2> dtiles = die_order(dt_items);
    std::vector<int2> gtiles = die_order(gt_items);   // 8 x kGT node tiles, then 32 x kGT
    {
        const std::vector<int2> g4 = die_order(gt_items4);
        gtiles.insert(gtiles.end(), g4.begin(), g4.end());
    }
    // record bases of every (layer, sensor of its instance) pair
    std::vector<int64_t> recbase;
    for (int l = 0; l < z.L; ++l) {
        LayerDev& d = t.ld[l];
        d.rb0 = int32_t(recbase.size());
        for (int j = 0; j < d.ng; ++j) recbase.push_back(t.pd[t.wd[d.g0 + j].pair0 + (l - d.l0)].rng_off);
    }
    // gather windows of the 32 x kGT tiles: per (layer tile, sensor of the layer's instance)
    // the rectangle of sensor nodes that the tile's records reach, {first row, rows, first
    // column, columns}; a tile the sensor does not see gets the 1 x 1 window {0, 1, 0, 1} (all
    // its weights are zero)
    std::vector<int4> gwin;
    ctx.max_gwin_side = 1;
    {
        const int tr = kGRowStep * 4;
        for (int l = 0; l < z.L; ++l) {
            LayerDev& d = t.ld[l];
            d.wb0 = int32_t(gwin.size());
            const int n = d.n, tx = (n + kGT - 1) / kGT, nt = gather_tiles_of(n, 4);
            for (int k = 0; k < nt; ++k) {
                const int a0 = (k / tx) * tr, b0 = (k % tx) * kGT;
                for (int j = 0; j < d.ng; ++j) {
                    const PairDev& p = t.pd[t.wd[d.g0 + j].pair0 + (l - d.l0)];
                    int lo[2] = {INT32_MAX, INT32_MAX}, hi[2] = {INT32_MIN, INT32_MIN};
                    for (int axis = 0; axis < 2; ++axis) {
                        const int first = axis == 0 ? a0 : b0, cnt = axis == 0 ? tr : kGT;
                        for (int a = first; a < std::min(n, first + cnt); ++a) {
                            const size_t ri = size_t(p.rng_off) + size_t(axis) * n + a;
                            const int st = t.rng[2 * ri], c = t.rng[2 * ri + 1];
                            if (c > 0) {
                                lo[axis] = std::min(lo[axis], st);
                                hi[axis] = std::max(hi[axis], st + c);
                            }
                        }
                    }
                    int4 w = make_int4(0, 1, 0, 1);
                    if (lo[0] < hi[0] && lo[1] < hi[1]) w = make_int4(lo[0], hi[0] - lo[0], lo[1], hi[1] - lo[1]);
                    ctx.max_gwin_side = std::max(ctx.max_gwin_side, std::max(w.y, w.w));
                    gwin.push_back(w);
                }
            }
        }
    }
    // gather records: per pair, layer rows then columns, parallel to the ranges
    std::vector<char> recs;
    auto build_recs = [&](auto tag) {
        using R = GatherRec<decltype(tag)>;
        std::vector<R> out(t.rng.size() / 2);
        for (int g = 0; g < z.G; ++g) {
            const WfsDev& w = t.wd[g];
            const int np = w.ns + 1;
            for (int j = 0; j < w.nl; ++j) {
                const PairDev& p = t.pd[w.pair0 + j];
                const int n = t.ld[w.l0 + j].n;
                for (int axis = 0; axis < 2; ++axis)
                    for (int a = 0; a < n; ++a) {
                        const size_t ri = size_t(p.rng_off) + size_t(axis) * n + a;
                        R r{};
                        r.start = t.rng[2 * ri];
                        r.count = t.rng[2 * ri + 1];
                        for (int q = 0; q < std::min(r.count, kRMax); ++q) {
                            const size_t ci = size_t(p.fwd_off) + size_t(axis) * np + r.start + q;
                            const double f = t.cfrac[ci];
                            r.w[q] = decltype(tag)(t.cidx[ci] == a ? 1.0 - f : f);
                        }
                        out[ri] = r;
                    }
            }
        }
        recs.resize(out.size() * sizeof(R));
        std::memcpy(recs.data(), out.data(), recs.size());
    };
    if (f32)
        build_recs(float{});
    else
        build_recs(double{});

    // warm-start layer constants: height / 20 km and turbulence weight of every layer
    std::vector<float> lconst;
    for (int i = 0; i < nb; ++i)
        for (int l = 0; l < cfgs[i].n_layers; ++l) {
            lconst.push_back(float(cfgs[i].layers[l].height / 20000.0));
            lconst.push_back(float(cfgs[i].layers[l].weight));
        }

    // ---- upload (typed copies of the floating tables)
    const Layout& lo = ctx.lay;
    auto up = [&](size_t dst, const void* src, size_t bytes) -> bool {
        return bytes == 0 || hipMemcpyAsync(ctx.ws + dst, src, bytes, hipMemcpyHostToDevice, stream) == hipSuccess;
    };
    auto typed = [&](const std::vector<double>& v) {
        std::vector<char> out(v.size() * ctx.esz);
        if (f32) {
            float* o = reinterpret_cast<float*>(out.data());
            for (size_t i = 0; i < v.size(); ++i) o[i] = float(v[i]);
        } else {
            std::memcpy(out.data(), v.data(), v.size() * sizeof(double));
        }
        return out;
    };
    const auto frac_t = typed(t.cfrac);
    const auto w_t = typed(t.wts);
    const auto xw_t = typed(t.xw);
    std::vector<double> ttv_all(t.ttv);
    ttv_all.insert(ttv_all.end(), t.ttvy.begin(), t.ttvy.end());
    const auto ttv_t = typed(ttv_all);
    ctx.any_cross = false;
    ctx.any_tt = false;
    for (double v : t.xw) ctx.any_cross = ctx.any_cross || v != 0.0;
    for (const WfsDev& w : t.wd) ctx.any_tt = ctx.any_tt || w.tt;
    const auto pa_t = typed(t.D);
    const auto j_t = typed(t.Jinv);
    // sensor of the first node of every kThreads-node block of the sensor-node vector (the slope
    // adjoint starts its search there)
    std::vector<int32_t> node_sensor(size_t(std::max<int64_t>(1, (ctx.V + kThreads - 1) / kThreads)), 0);
    for (size_t b = 0, g = 0; b < node_sensor.size(); ++b) {
        const int64_t e0 = int64_t(b) * kThreads;
        while (g + 1 < t.wd.size() && t.wd[g + 1].noff <= e0) ++g;
        node_sensor[b] = int32_t(g);
    }
    bool ok = up(lo.layers, t.ld.data(), sizeof(LayerDev) * t.ld.size()) &&
              up(lo.node_sensor, node_sensor.data(), sizeof(int32_t) * node_sensor.size()) &&
              up(lo.wfs, t.wd.data(), sizeof(WfsDev) * t.wd.size()) &&
              up(lo.pairs, t.pd.data(), sizeof(PairDev) * t.pd.size()) &&
              up(lo.cellidx, t.cidx.data(), sizeof(int32_t) * t.cidx.size()) &&
              up(lo.frac, frac_t.data(), frac_t.size()) &&
              up(lo.ranges, t.rng.data(), sizeof(int32_t) * t.rng.size()) &&
              up(lo.insts, ctx.insts.data(), sizeof(InstDev) * ctx.insts.size()) &&
              up(lo.vecblk, vb.data(), sizeof(VecBlk) * vb.size()) &&
              up(lo.gramblk, gb.data(), sizeof(GramBlk) * gb.size()) &&
              up(lo.syn_items, syn.data(), sizeof(int2) * syn.size()) &&
              up(lo.ana_items, ana.data(), sizeof(int4) * ana.size()) &&
              up(lo.data_tiles, dtiles.data(), sizeof(int2) * dtiles.size()) &&
              up(lo.gather_tiles, gtiles.data(), sizeof(int2) * gtiles.size()) &&
              up(lo.grecs, recs.data(), recs.size()) &&
              up(lo.recbase, recbase.data(), sizeof(int64_t) * recbase.size()) &&
              up(lo.gwin, gwin.data(), sizeof(int4) * gwin.size()) &&
              up(lo.lconst, lconst.data(), sizeof(float) * lconst.size()) &&
              up(lo.weight, w_t.data(), w_t.size()) && up(lo.xweight, xw_t.data(), xw_t.size()) &&
              up(lo.ttv, ttv_t.data(), ttv_t.size()) && up(lo.prior_a, pa_t.data(), pa_t.size()) &&
              up(lo.jinv, j_t.data(), j_t.size());
    if (ok) ok = hipStreamSynchronize(stream) == hipSuccess;   // host vectors die at return
    if (!ok) { ctx.err = "hipMemcpyAsync of the setup tables failed"; return FEWHA_E_HIP; }
    return FEWHA_OK;
}

}  // namespace fewha
