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
constexpr int kAnaWide = 512;       // tiled analysis of a small context: eight wavefronts per workgroup
constexpr int kAnaWideItems = 512;  // ... up to this many tiles per launch
constexpr int kVecBlocksMax = 1024; // vector-kernel workgroups of one instance (grid-stride beyond)
constexpr int kDefaultBlockElems = 384;  // default elements per vector workgroup
constexpr int kGramElems = 1536;    // elements per Gram workgroup (one instance: <= kGramBlocks)
constexpr int kKMax = FEWHA_MAX_RECYCLE;
constexpr int kSlotsMax = kKMax + 256;
constexpr int kTile = 14;           // wavefront-node tile side of the fused data-term kernel (16 with the halo)
constexpr int kCoarseThreads = 256;  // threads of the one-workgroup-per-layer coarse analysis kernel
// Analysis levels whose block fits CB x CB run inside one workgroup's LDS; larger levels are
// tiled over many workgroups, up to kAnaLevels<T> of them per launch.
template <typename T> struct CoarseBlock { static constexpr int value = 32; };
inline int coarse_block(int /*precision*/) { return 32; }
inline int ana_levels_per_launch(int precision) { return precision == FEWHA_FP64 ? 2 : 3; }
// output tile side (per band) of the last level of a tiled analysis launch of k levels: the
// first level's outputs are then 16 x 16 per band
inline int ana_tile(int k) { return 16 >> (k - 1); }
constexpr int kSynTile = 32;        // image tile side of the synthesis
constexpr int kSmallTileBelow = 256; // synthesis tiles of kSynTile / 2 when there are fewer kSynTile tiles
constexpr int kGT = 32;             // layer-node tile columns of the adjoint gather
constexpr int kGRowStep = kThreads / kGT;        // tile rows per gather thread row (8)
constexpr int64_t kGatherWide = int64_t(1) << 21;  // from this many coefficients on, 4 rows per gather thread
constexpr int kRMax = 6;            // contributions per layer row/column held by a gather record
constexpr int kXcds = 8;            // accelerator complex dies; workgroup i runs on die i mod kXcds
constexpr int kGramBlocks = 128;    // Gram workgroups of one instance at most (partials per entry)
constexpr int kGramThreads = 1024;  // threads of a Gram workgroup (16 wavefronts)
constexpr int kDataThreads = 256;   // threads of the fused data-term kernel (one halo-tile node each)
constexpr int kSolveThreads = 1024; // threads of the single-block Gram reduction and solve
constexpr int kGatherGroup = 8;     // sensors whose gather lists are staged together

// Device descriptors (plain data, copied into the workspace at setup).  The layers and
// sensors of all instances of a batch are listed one after the other; a sensor only sees the
// layers of its own instance.
struct LayerDev {
    int32_t n, levels;
    int32_t coarse_lev;   // finest level whose block fits the coarse block (levels >= coarse_lev run in LDS)
    int32_t inst;         // instance of the layer
    int64_t off;          // offset of the layer in coefficient / nodal vectors
    double inv_delta;     // 1 / delta_l
    int32_t l0;           // first layer of the instance
    int32_t g0, ng;       // sensors of the instance
    int32_t pq0;          // first (p, q) partial of the layer: tiled analysis tiles by level, then coarse
    int32_t pq_coarse;    // index of the coarse analysis partial (relative to pq0)
    int32_t rb0;          // the gather records of (sensor d.g0 + j, this layer) start at recbase[rb0 + j]
    int32_t wb0;          // gather windows of (tile k of this layer, sensor d.g0 + j) at gwin[wb0 + k ng + j]
};

inline int coarse_first_level(int n, int cb) {
    int l = 1;
    while ((n >> (l - 1)) > cb) ++l;
    return l;
}

struct WfsDev {
    int32_t ns;           // subapertures per side
    int32_t tiles_x;      // node tiles per side (ceil((ns+1)/kTile))
    int32_t tile_off;     // first tile of this sensor in the fused kernel's grid
    int32_t inst;         // instance of the sensor
    int64_t soff;         // slope offset
    int64_t noff;         // wavefront-node offset
    int32_t l0, nl;       // layers of the instance
    int32_t pair0;        // pair (this sensor, layer l0 + j) is pair0 + j
    int32_t pad_;
    int64_t fwd0;         // bilinear cells of pair (this sensor, layer l0 + j) at fwd0 + j * 2 (ns + 1)
    int32_t tt;           // tip/tilt filter of C_eta^-1
    int32_t pad2_;
    double tg[3];         // (T^T B T)^-1: [0] [1]; [1] [2]
};

// Transpose of the bilinear propagation along one axis, for one layer row (column) a of one
// pair: sensor rows (columns) start .. start + count - 1 contribute with weights w.
template <typename T>
struct GatherRec {
    int32_t start, count;
    T w[kRMax];
};

struct PairDev {          // one (sensor, layer) pair of the same instance
    int64_t fwd_off;      // rows then columns: 2 (ns+1) entries of cell index / fraction
    int64_t rng_off;      // rows then columns: 2 n entries of (first node, count)
};

// One independent instance of a batch (a single system is a batch of one).
struct InstDev {
    int64_t off, n;       // coefficient range
    int32_t vb0, nvb;     // vector workgroups [vb0, vb0 + nvb): partial columns of the instance
    int32_t gb0, ngb;     // Gram workgroups
    int32_t pq0, npq;     // (p, q) partials of its analysis tiles
};

// What a vector-kernel workgroup works on: elements local * kThreads + t, stepping by
// nb * kThreads, of its instance's range; partial column `col` (the instance's columns are
// col - local .. col - local + nb - 1); the instance's (p, q) partials [pq0, pq0 + npq).
struct VecBlk {
    int64_t off;
    int32_t n, local, nb, inst, col, pq0, npq, pad_;
};
struct GramBlk {
    int64_t off;
    int32_t n, local, nb, inst, gbase, pad_;   // partial of entry e: gbase + e * nb + local
};

template <typename T>
struct Filt { T h[6], g[6]; };

// Bits of fewha_solve_info.flags (and of Scalars::flags during a frame).
constexpr int32_t kFlagBreakdown = 1;   // a non-finite value or non-positive curvature; c, r kept
constexpr int32_t kFlagTolUnmet = 2;    // tolerance mode: not met within the frame
constexpr int32_t kFlagWsRejected = 4;  // warm start: the correction was not taken
constexpr int32_t kFlagBadRhs = 8;      // (b, b) not finite: the frame was not solved

// Scalars of one instance's solve, in device memory (never copied to the host inside a frame).
struct Scalars {
    double rzb[2];        // (r, z) of the current iteration, double-buffered by iteration parity
    double rz, rz_new, pq, alpha, beta, mu, rr, bb, zq_last, ru_last;
    double y[kKMax];      // Galerkin coefficients
    double y2[kKMax];     // initial-direction coefficients
    double gam[kSlotsMax];// (p_j, q_j) of every ring slot
    double R[kKMax * kKMax];   // GALERKIN: G+ of the recycled Gram matrix (m x m, row-major); PAPER: rows of X
    int32_t keep[kKMax];
    int32_t flags, dropped, used, iters;
    int32_t conv_iter;    // tolerance mode: first iteration whose residual met the tolerance (0: not yet)
    int32_t ws_state;     // warm start of this frame: 0 none, 1 accepted, 2 rejected
    int64_t frame_no;     // frames finished since setup (the breakdown report names a frame by it)
    int32_t avail;        // tolerance mode: real directions at the end of the recycle window (the rest of
                          // the window is hidden from the projections)
    int32_t pad_;
};

// Byte layout of the workspace (offsets from its base).
struct Layout {
    size_t layers, wfs, pairs, cellidx, frac, ranges, weight, xweight, ttv, wslopes, prior_a, jinv;
    size_t insts, vecblk, gramblk, syn_items, ana_items, data_tiles, gather_tiles, grecs, recbase, gwin, node_sensor;
    size_t nodal, tmp0, tmp1, psi_nodes, psi_layers, vx, vy;
    size_t c, r, z, b, b_prev;
    size_t ring_u, ring_q;
    size_t partials, pq_part, gram_part, scalars, info, done;
    size_t ws_in, ws_out, lconst;   // warm start: network input (N x 4 FP32), output (N FP32), layer constants
    size_t total;
    size_t state_bytes;
};

// Kernels, for the optional event profiler and the per-kernel timer.
enum KernelId : int {
    KID_IDWT = 0, KID_DATA_TERM, KID_ADJ_GATHER, KID_DWT_TILES, KID_DWT_COARSE, KID_SLOPES_ADJ, KID_RESIDUAL, KID_GRAM, KID_GRAM_SOLVE, KID_GALERKIN, KID_INIT_DIR, KID_UPDATE1,
    KID_UPDATE2, KID_FINISH, KID_FWD_SLOPES, KID_TT_CORRECT, KID_COUNT
};
extern const char* const kKernelNames[KID_COUNT];
constexpr int KID_APPLY = -1;   // the per-kernel timer's id of a whole application of M

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;          // begin/end pairs
    std::vector<int> pending;              // kernel id of every recorded pair
    double ms[KID_COUNT] = {};
    int64_t launches[KID_COUNT] = {};
};

// One tiled analysis launch: ni workgroup items at loff of the device item list, from nl
// layers; nb is the largest block it transforms.
struct StepInfo {
    int nb = 0, nl = 0, loff = 0, ni = 0;
};

struct Ctx {
    // configuration
    int B = 1;                 // instances
    int L = 0, G = 0;          // layers and sensors of all instances
    int64_t N = 0, S = 0, V = 0;
    int VB = 0, GB = 0;        // vector and Gram workgroups of all instances
    int block_elems = kDefaultBlockElems;
    int data_grid = 0;         // workgroups of the fused data term (tiles, padded to kXcds)
    int gather_grid1 = 0, gather_grid4 = 0;   // gather workgroups (layer tiles, padded to kXcds) of 1 and 4 rows
    int gather_rows = 1;       // layer rows per gather thread (tile of 8 gather_rows x kGT nodes), 1 or 4
    int syn_tile = 0;          // synthesis image tile: 16, 32, 64 (FP32), or 0 (by the number of tiles)
    std::vector<InstDev> insts;
    std::vector<int> layers_n;     // grid size of every layer (host)
    std::vector<int64_t> s_offs;   // slope offsets of the instances (B + 1)
    int prec = 0;              // fewha_precision
    size_t esz = 8;            // element size
    double alpha = 0;
    int max_iter = 0, k = 0, mode = 1, project_all = 0;
    double rel_tol = 0;        // > 0: iterate until every instance meets it (or max_iter)
    int frame_iters = 0;       // iterations of the last frame
    int max_levels = 0, max_n = 0;
    int slots = 0;             // ring capacity k + max_iter
    int max_rng = 0;           // largest gather contribution count of a layer row/column
    int max_gwin_side = 0;     // largest side of the sensor-node rectangle of a gather tile
    std::vector<StepInfo> steps;  // tiled analysis launches (finest levels first)
    int syn_small = 0, syn_large = 0, syn_huge = 0;   // synthesis tiles of kSynTile / 2, kSynTile, 2 kSynTile
    bool any_cross = false, any_tt = false;   // LGS noise model: 2x2 noise blocks / tip/tilt filters
    int npq = 0;               // (p, q) partial entries written by one analysis
    int64_t n_cells = 0, n_ranges = 0;
    std::vector<fewha_layer> layers;
    std::vector<fewha_wfs> wfs;
    // host-side ring bookkeeping (fixed iteration count: the device never decides)
    int head = 0, count = 0, last_iters = 0;
    bool first = true;
    // breakdown report: pinned, device-mapped host word into which the end of a frame writes
    // its frame number when an instance broke down; the host reports each new value once
    int64_t* brk_host = nullptr;
    int64_t* brk_dev = nullptr;
    int64_t brk_reported = 0;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout lay{};
    std::string err;
    const char* err_lit = nullptr;   // static message of the last error, when set (preferred over err)
    mutable Profiler prof;
    // captured frame graphs, keyed by (ring head, first frame, recycled directions)
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;
    template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
};

// Intermediates of one operator application: the nodal image, the two wavelet ping-pong
// buffers (N elements each), the sensor-node field (V) and the layer adjoint field (N).  The
// context's own live in its workspace; fewha_apply_A_noalloc brings its own.
struct OpBufs {
    char *nodal, *tmp0, *tmp1, *psi_nodes, *psi_layers, *wslopes;
};
inline OpBufs ctx_bufs(const Ctx& c) {
    return OpBufs{c.ws + c.lay.nodal, c.ws + c.lay.tmp0, c.ws + c.lay.tmp1, c.ws + c.lay.psi_nodes,
                  c.ws + c.lay.psi_layers, c.ws + c.lay.wslopes};
}

// Records HIP events around one kernel launch on `s` when profiling is enabled.
struct ProfScope {
    const Ctx& c;
    hipStream_t s;
    ProfScope(const Ctx& ctx, int kid, hipStream_t stream);
    ~ProfScope();
};
hipError_t profiler_collect(const Ctx& c, hipStream_t s);

// Host setup (fewha_setup.cpp): a batch is an array of n configurations
fewha_status validate_batch(const fewha_config* cfgs, int n, std::string& err);
Layout compute_layout(const fewha_config* cfgs, int n);
fewha_status build_tables(Ctx& ctx, const fewha_config* cfgs, int n, hipStream_t stream);

// Launchers (fewha_kernels.hip)
// skip (may be NULL): per-instance flags; the workgroups of an instance whose flag is set return
// at once (tolerance mode: the instance has converged within the frame).
template <typename T> void launch_winv(const Ctx& c, const T* x, T* phi, hipStream_t s, const OpBufs* ob = nullptr,
                                       const int32_t* skip = nullptr);
template <typename T> void launch_winvt(const Ctx& c, const T* img, T* y, const T* xprior, double* pq_part,
                                        hipStream_t s, const OpBufs* ob = nullptr, const int32_t* skip = nullptr);
template <typename T> void launch_data_term(const Ctx& c, const T* phi, T* psi_nodes, hipStream_t s,
                                            const int32_t* skip = nullptr, T* wsl = nullptr);
template <typename T> void launch_slopes_adj(const Ctx& c, const T* slopes, T* psi_nodes, int weighted, hipStream_t s);
template <typename T> void launch_adj_gather(const Ctx& c, const T* psi_nodes, T* psi_layers, hipStream_t s,
                                             const int32_t* skip = nullptr);
template <typename T> void launch_fwd_slopes(const Ctx& c, const T* phi, T* slopes, hipStream_t s);
template <typename T> void launch_apply_M(const Ctx& c, const T* x, T* y, double* pq_part, hipStream_t s,
                                          const OpBufs* ob = nullptr, const int32_t* skip = nullptr);

template <typename T> void launch_rhs(const Ctx& c, const T* slopes, T* b, hipStream_t s,
                                      double* bb_part = nullptr);
template <typename T> hipError_t launch_solve_frame(Ctx& c, const T* slopes, T* c_out, fewha_solve_info* info,
                                                   hipStream_t s);
// Warm start of a frame by the U-Net (include/fewha_unet.h): input/output scales.
struct WarmStart {
    void* net;                 // fewha_unet*
    float scale_c, scale_r, scale_out;
};
template <typename T> hipError_t launch_solve_frame_ws(Ctx& c, const WarmStart& w, const T* slopes, T* c_out,
                                                      fewha_solve_info* info, hipStream_t s);
template <typename T> hipError_t launch_ws_input(const Ctx& c, const WarmStart& w, const T* c_in, const T* slopes,
                                                 float* in, hipStream_t s);
void release_graphs(Ctx& c);
// Copies every instance's count of real recycled directions to (to_state) or from a checkpoint:
// the double at base + stride i + 8 slots.
hipError_t launch_state_avail(const Ctx& c, char* base, size_t stride, bool to_state, hipStream_t s);
// Address of fewha_apply_A_noalloc's static scratch array on the current device, taken once per
// device (fewha_setup calls it).
fewha_status scratch_init(const char** err);
template <typename T> hipError_t time_operator_kernel(Ctx& c, int kid, int step, int reps, hipStream_t s, float* ms);

}  // namespace fewha

// The opaque context of the C ABI.
struct fewha_ctx {
    fewha::Ctx c;
    uint64_t state_header[32];   // host copy of the checkpoint header (kept alive for async H2D)
};
