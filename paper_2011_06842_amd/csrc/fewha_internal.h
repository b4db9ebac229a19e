// Internal declarations of the MI355X augmented-FEWHA library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fewha.h"

namespace fewha {

constexpr int kThreads = 256;       // threads of every 1-D kernel (4 wavefronts of 64)
constexpr int kVecBlocks = 512;     // fixed grid of the vector/reduction kernels (determinism)
constexpr int kKMax = FEWHA_MAX_RECYCLE;
constexpr int kSlotsMax = kKMax + 256;
constexpr int kTile = 16;           // wavefront-node tile side of the fused data-term kernel
constexpr int kCoarseThreads = 1024;  // threads of the one-workgroup-per-layer coarse wavelet kernels
// Wavelet blocks up to CB x CB are transformed inside one workgroup's LDS; larger levels are
// tiled over many workgroups (one CU's LDS bandwidth is the limit of the in-LDS passes).
template <typename T> struct CoarseBlock { static constexpr int value = 64; };
inline int coarse_block(int /*precision*/) { return 64; }
constexpr int kST = 32;             // output tile side of a tiled synthesis step
constexpr int kAT = 16;             // coefficient tile side (per band) of a tiled analysis step
constexpr int kGT = 16;             // layer-node tile side of the adjoint gather
constexpr int kRMax = 6;            // contributions per layer row/column kept in LDS by the gather
constexpr int kGramBlocks = 256;    // grid of the Gram pass
constexpr int kDataThreads = 1024;  // threads of the fused data-term kernel
constexpr int kSolveThreads = 1024; // threads of the single-block Gram reduction and solve
constexpr int kLayerGroups = 3;     // threads sharing one wavefront node's layer sum
constexpr int kGatherGroup = 8;     // sensors whose gather lists are built together
constexpr int kGatherRegion = 16384; // LDS bytes for the gather's sensor-node rectangles

// Device descriptors (plain data, copied into the workspace at setup).
struct LayerDev {
    int32_t n, levels;
    int32_t coarse_lev;   // finest level whose block fits the coarse block (levels >= coarse_lev run in LDS)
    int32_t pad_;
    int64_t off;          // offset of the layer in coefficient / nodal vectors
    double inv_delta;     // 1 / delta_l
};

inline int coarse_first_level(int n, int cb) {
    int l = 1;
    while ((n >> (l - 1)) > cb) ++l;
    return l;
}

// One tiled wavelet level of block size nb and the layers that have it.
struct WaveStep {
    int nb = 0;
    std::vector<int> layers;
};
struct StepLayers { int32_t count; int32_t l[FEWHA_MAX_LAYERS]; };

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
    double rzb[2];        // (r, z) of the current iteration, double-buffered by iteration parity
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
    size_t partials, pq_part, gram_part, scalars, info;
    size_t total;
    size_t state_bytes;
};

// Kernels, for the optional event profiler and the per-kernel timer.
enum KernelId : int {
    KID_IDWT_COARSE = 0, KID_IDWT_STEP, KID_DATA_TERM, KID_ADJ_GATHER, KID_DWT_STEP, KID_DWT_COARSE,
    KID_SLOPES_ADJ, KID_RESIDUAL, KID_GRAM, KID_GRAM_SOLVE, KID_GALERKIN, KID_INIT_DIR, KID_UPDATE1,
    KID_UPDATE2, KID_FINISH, KID_FWD_SLOPES, KID_COUNT
};
extern const char* const kKernelNames[KID_COUNT];

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;          // begin/end pairs
    std::vector<int> pending;              // kernel id of every recorded pair
    double ms[KID_COUNT] = {};
    int64_t launches[KID_COUNT] = {};
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
    int max_rng = 0;           // largest gather contribution count of a layer row/column
    std::vector<WaveStep> steps;  // tiled wavelet levels (ascending block size)
    int npq = 0;               // (p, q) partial entries written by one analysis
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
    mutable Profiler prof;
    // captured frame graphs, keyed by (ring head, first frame, recycled directions)
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;
    template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
};

// Records HIP events around one kernel launch on `s` when profiling is enabled.
struct ProfScope {
    const Ctx& c;
    hipStream_t s;
    ProfScope(const Ctx& ctx, int kid, hipStream_t stream);
    ~ProfScope();
};
hipError_t profiler_collect(const Ctx& c, hipStream_t s);

// Host setup (fewha_setup.cpp)
fewha_status validate_config(const fewha_config* cfg, std::string& err);
Layout compute_layout(const fewha_config* cfg);
std::vector<WaveStep> wavelet_steps(const fewha_config* cfg);
int pq_partials(const fewha_config* cfg);
fewha_status build_tables(Ctx& ctx, const fewha_config* cfg, hipStream_t stream);

// Launchers (fewha_kernels.hip)
template <typename T> void launch_winv(const Ctx& c, const T* x, T* phi, hipStream_t s);
template <typename T> void launch_winvt(const Ctx& c, const T* img, T* y, const T* xprior, const T* xdot,
                                        double* pq_part, hipStream_t s);
template <typename T> void launch_data_term(const Ctx& c, const T* phi, T* psi_nodes, hipStream_t s);
template <typename T> void launch_slopes_adj(const Ctx& c, const T* slopes, T* psi_nodes, int weighted, hipStream_t s);
template <typename T> void launch_adj_gather(const Ctx& c, const T* psi_nodes, T* psi_layers, hipStream_t s);
template <typename T> void launch_fwd_slopes(const Ctx& c, const T* phi, T* slopes, hipStream_t s);
template <typename T> void launch_apply_M(const Ctx& c, const T* x, T* y, double* pq_part, hipStream_t s);
template <typename T> void launch_rhs(const Ctx& c, const T* slopes, T* b, hipStream_t s);
template <typename T> hipError_t launch_solve_frame(Ctx& c, const T* slopes, T* c_out, fewha_solve_info* info,
                                                   hipStream_t s);
void release_graphs(Ctx& c);
template <typename T> hipError_t time_operator_kernel(Ctx& c, int kid, int step, int reps, hipStream_t s, float* ms);

}  // namespace fewha
