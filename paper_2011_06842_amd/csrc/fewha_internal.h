// Internal declarations of the MI355X augmented-FEWHA library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fewha.h"

namespace fewha {

constexpr int kThreads = 256;       // threads of every 1-D kernel (4 wavefronts of 64)
constexpr int kVecBlocks = 512;     // fixed grid of the vector/reduction kernels (determinism)
constexpr int kKMax = FEWHA_MAX_RECYCLE;
constexpr int kSlotsMax = kKMax + 256;
constexpr int kTile = 16;           // wavefront-node tile side of the fused data-term kernel

// Device descriptors (plain data, copied into the workspace at setup).
struct LayerDev {
    int32_t n, levels;
    int64_t off;          // offset of the layer in coefficient / nodal vectors
    double inv_delta;     // 1 / delta_l
};

struct WfsDev {
    int32_t ns;           // subapertures per side
    int32_t tiles_x;      // node tiles per side (ceil((ns+1)/kTile))
    int32_t tile_off;     // first tile of this sensor in the fused kernel's grid
    int32_t pad_;
    int64_t soff;         // slope offset
    int64_t noff;         // wavefront-node offset
};

struct PairDev {          // one (sensor g, layer l) pair, index g * L + l
    int64_t fwd_off;      // rows then columns: 2 (ns+1) entries of cell index / fraction
    int64_t rng_off;      // rows then columns: 2 n entries of (first node, count)
};

template <typename T>
struct Filt { T h[6], g[6]; };

// Scalars of a solve, in device memory (never copied to the host inside a frame).
struct Scalars {
    double rz, rz_new, pq, alpha, beta, mu, rr, bb, zq_last, ru_last;
    double y[kKMax];      // Galerkin coefficients
    double y2[kKMax];     // initial-direction coefficients
    double gam[kSlotsMax];// (p_j, q_j) of every ring slot
    double R[kKMax * kKMax];
    int32_t keep[kKMax];
    int32_t flags, dropped, used, iters;
};

// Byte layout of the workspace (offsets from its base).
struct Layout {
    size_t layers, wfs, pairs, cellidx, frac, ranges, weight, prior_a, jinv;
    size_t nodal, tmp0, tmp1, psi_nodes, psi_layers, vx, vy;
    size_t c, r, z, b, b_prev, s_in;
    size_t ring_u, ring_q;
    size_t partials, scalars, info;
    size_t total;
    size_t state_bytes;
};

struct Ctx {
    // configuration
    int L = 0, G = 0;
    int64_t N = 0, S = 0, V = 0;
    int prec = 0;              // fewha_precision
    size_t esz = 8;            // element size
    double alpha = 0;
    int max_iter = 0, k = 0, mode = 1, project_all = 0;
    int max_levels = 0, max_n = 0;
    int slots = 0;             // ring capacity k + max_iter
    int fwd_tiles = 0;         // total tiles of the fused data-term kernel
    int64_t n_cells = 0, n_ranges = 0;
    std::vector<fewha_layer> layers;
    std::vector<fewha_wfs> wfs;
    // host-side ring bookkeeping (fixed iteration count: the device never decides)
    int head = 0, count = 0, last_iters = 0;
    bool first = true;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout lay{};
    std::string err;
    template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
};

// Host setup (fewha_setup.cpp)
fewha_status validate_config(const fewha_config* cfg, std::string& err);
Layout compute_layout(const fewha_config* cfg);
fewha_status build_tables(Ctx& ctx, const fewha_config* cfg, hipStream_t stream);

// Launchers (fewha_kernels.hip)
template <typename T> void launch_winv(const Ctx& c, const T* x, T* phi, hipStream_t s);
template <typename T> void launch_winvt(const Ctx& c, const T* phi, T* y, const T* xprior, hipStream_t s);
template <typename T> void launch_data_term(const Ctx& c, const T* phi, T* psi_nodes, hipStream_t s);
template <typename T> void launch_slopes_adj(const Ctx& c, const T* slopes, T* psi_nodes, int weighted, hipStream_t s);
template <typename T> void launch_adj_gather(const Ctx& c, const T* psi_nodes, T* psi_layers, hipStream_t s);
template <typename T> void launch_fwd_slopes(const Ctx& c, const T* phi, T* slopes, hipStream_t s);
template <typename T> void launch_apply_M(const Ctx& c, const T* x, T* y, hipStream_t s);
template <typename T> void launch_rhs(const Ctx& c, const T* slopes, T* b, hipStream_t s);
template <typename T> void launch_solve_frame(Ctx& c, const T* slopes, T* c_out, fewha_solve_info* info, hipStream_t s);

}  // namespace fewha
