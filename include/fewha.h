/*
 * fewha.h -- C ABI of the MI355X augmented wavelet reconstructor (augmented FEWHA).
 *
 * The library solves, frame after frame, the wavelet-domain MAP system of atmospheric
 * tomography (Sec. 3, equation for M and the right-hand side b)
 *
 *     M c = b,   M = W^-T A^T C_eta^-1 A W^-1 + alpha D,   b = W^-T A^T C_eta^-1 s,
 *
 * with augmented preconditioned conjugate gradients (Sec. 4.1, Alg. 2) inside the frame
 * update of the augmented wavelet reconstructor (Sec. 5, Alg. 3: right-hand side,
 * residual update, augmented PCG).  A is the tomography operator (Sec. 2): bilinear
 * propagation from every layer to every guide-star direction (natural: shift; laser:
 * cone-scaled shift) followed by the Shack-Hartmann operator.  W is the periodic
 * Daubechies-3 wavelet transform of every layer scaled by its constant delta_l (Sec. 3).
 *
 * Conventions shared by every entry point
 *  - Element type: device vectors (coefficients, slopes) are double in FEWHA_FP64 and
 *    float in FEWHA_FP32_OP_FP64_RED.  Inner products, the recycle Gram matrix, its
 *    factorisation and all scalars are double in both modes.
 *  - Layouts: a coefficient vector is the concatenation over layers of an n_l x n_l
 *    row-major 2-D Mallat pyramid (approximation block top-left; at each level the block
 *    right of it holds the x-detail, below it the y-detail, diagonal the xy-detail).  A
 *    nodal layer vector uses the same offsets with row-major node values (row = y).
 *    A slope vector is the concatenation over sensors of [s^x (n_sub^2 row-major);
 *    s^y (n_sub^2)].
 *  - Ownership: all device buffers are allocated by the caller.  The workspace passed to
 *    fewha_setup belongs to the context until fewha_destroy; the library allocates no
 *    device memory of its own.  Host arrays inside fewha_config are read during
 *    fewha_setup only.
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream).  Compute calls are
 *    stream-ordered and asynchronous; argument errors are returned synchronously.  A
 *    context must be used from one stream at a time and is not thread-safe.
 *  - Errors: every call returns a fewha_status; fewha_last_error() gives a message.
 *  - Breakdown (the paper runs a fixed iteration count and is silent on it): a projection
 *    coefficient, step length or beta that is not finite, or a curvature (p, M p) <= 0 while
 *    (r, J^-1 r) != 0, stops the frame's progress.  The carried coefficients and residual keep
 *    their last finite values (they stay each other's residual pair), the directions the frame
 *    stores from then on are zero vectors (given no weight by later projections), and info
 *    flag bit 0 is set; the next frame continues from that state, with no reset needed.  A
 *    frame whose right-hand side has a non-finite squared norm (non-finite or overflowing
 *    slopes) is not solved at all (flag bits 0 and 3, relative residual NaN).  A later
 *    fewha_solve_aug / fewha_solve_aug_ws call that finds such a frame finished returns
 *    FEWHA_E_BREAKDOWN once for it (after enqueueing its own frame as usual).
 *  - Validation: alpha >= 0; slope weights >= 0; a given prior_diag or precond_inv must be
 *    finite and > 0 everywhere (FEWHA_E_INVAL otherwise).
 */
#ifndef FEWHA_H
#define FEWHA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FEWHA_ABI_VERSION 3
#define FEWHA_MAX_LAYERS 32
#define FEWHA_MAX_LEVELS 10   /* wavelet levels of a layer (n <= 1024) */
#define FEWHA_MAX_WFS 32
#define FEWHA_MAX_RECYCLE 32
#define FEWHA_MAX_INSTANCES 4096

typedef struct fewha_ctx fewha_ctx;

typedef enum {
    FEWHA_OK = 0,
    FEWHA_E_INVAL = 1,      /* bad argument or geometry (e.g. a footprint leaves a layer grid) */
    FEWHA_E_NOMEM = 2,      /* workspace too small */
    FEWHA_E_HIP = 3,        /* a HIP runtime call failed */
    FEWHA_E_NOT_SPD = 4,    /* a diagonal entry of M is not positive */
    FEWHA_E_BREAKDOWN = 5,  /* an earlier frame broke down (see fewha_solve_aug); this call's work was done */
    FEWHA_E_STATE = 6       /* state buffer does not belong to this configuration */
} fewha_status;

typedef enum { FEWHA_FP64 = 0, FEWHA_FP32_OP_FP64_RED = 1 } fewha_precision;

/* Recycling variants of Alg. 2 (Sec. 4.1).  PAPER: sequential single-vector Galerkin and
 * initial-direction projections against the previous frame's directions, as printed.
 * GALERKIN: the same projections solved jointly with the k x k Gram matrix U^T Q (FP64,
 * eliminated in order with the pivots of its Cholesky factorisation; a direction whose pivot is
 * at most 1e-14 of the largest diagonal entry is dropped) over a ring of the k most recent
 * directions. */
typedef enum { FEWHA_RECYCLE_PAPER = 0, FEWHA_RECYCLE_GALERKIN = 1 } fewha_recycle_mode;

/* One turbulence layer (Sec. 2 layered atmosphere; Sec. 3 layer grid of 2^(2 J_l) nodes). */
typedef struct {
    double height;      /* h_l [m] */
    double weight;      /* gamma_l, fraction of turbulence strength (enters the prior) */
    double spacing;     /* d_l [m], node spacing; also the wavelet scaling delta_l */
    double origin_x;    /* grid centre [m]; node (a,b) is at origin + ((b-(n-1)/2) d, (a-(n-1)/2) d) */
    double origin_y;
    int32_t n;          /* nodes per side, a power of two, 8 <= n <= 1024 */
    int32_t levels;     /* wavelet levels, 1 <= levels <= log2(n) */
} fewha_layer;

/* One Shack-Hartmann sensor and its guide star (Sec. 2). */
typedef struct {
    int32_t n_sub;               /* subapertures per side; nodes (n_sub+1)^2 at ((j-n_sub/2) d_s, (i-n_sub/2) d_s) */
    int32_t pad_;
    double subap;                /* d_s [m] */
    double theta_x, theta_y;     /* guide-star direction [rad] */
    double lgs_height;           /* H [m] of a laser guide star; 0 for a natural guide star */
    const double* slope_weight;  /* host, 2 n_sub^2: diagonal of C_eta^-1 (0 = inactive subaperture) */
    /* Laser-guide-star noise model (the paper counts its cost but does not state it; this is the
     * library's reading).  C_eta^-1 of the sensor is B, a symmetric 2x2 block per subaperture
     * [[w_x, w_c], [w_c, w_y]] (w_x, w_y from slope_weight), each positive semi-definite and
     * zero on inactive subapertures; with tt_filter it is B - B T (T^T B T)^-1 T^T B, T the
     * sensor's global tip and tilt slope patterns (all x slopes 1, all y slopes 1 on active
     * subapertures), so that the reconstruction ignores the sensor's tip/tilt.  The Jacobi
     * preconditioner uses the diagonal of the operator with B. */
    const double* cross_weight;  /* host, n_sub^2 (row-major subapertures) w_c entries, or NULL (all 0) */
    int32_t tt_filter;           /* 1: filter the sensor's tip/tilt (T^T B T must be positive definite) */
    int32_t pad2_;
} fewha_wfs;

typedef struct {
    int32_t abi_version;         /* FEWHA_ABI_VERSION */
    int32_t n_layers;            /* 1..FEWHA_MAX_LAYERS */
    const fewha_layer* layers;   /* host */
    int32_t n_wfs;               /* 1..FEWHA_MAX_WFS */
    int32_t pad_;
    const fewha_wfs* wfs;        /* host */
    double alpha;                /* regularisation weight (Sec. 3) */
    double r0, L0;               /* Fried parameter and outer scale [m] for the default prior */
    const double* prior_diag;    /* host, N entries of D, or NULL for the default von Karman prior */
    const double* precond_inv;   /* host, N entries of J^-1, or NULL for 1/diag(M) computed exactly */
    int32_t max_iter;            /* PCG iterations per frame (operator applications), 1..256 */
    int32_t recycle_k;           /* recycled directions, 0..FEWHA_MAX_RECYCLE (0 = plain PCG) */
    int32_t recycle_mode;        /* fewha_recycle_mode */
    int32_t project_all;         /* GALERKIN only: project every new direction against all of U */
    double rel_tol;              /* 0: exactly max_iter iterations per frame.  > 0 (< 1): every instance
                                    stops at its first iteration with ||r|| <= rel_tol ||b|| (FP64; decided
                                    on the device after every iteration), or at max_iter.  A stopped
                                    instance's kernels return at once for the rest of the frame, its c and r
                                    stay those of its stop, and at the end of the frame its last recycle_k
                                    directions move to the end of the shared recycle window.  The frame
                                    never synchronises with the host: all max_iter iterations are enqueued
                                    (and captured into a graph like fixed-count frames), those after every
                                    instance has stopped costing only their launches */
    int32_t precision;           /* fewha_precision */
    int32_t block_elems;         /* elements per workgroup of the vector kernels (0 = 384); fixes the
                                    reduction order, so results are reproducible for a given value */
    int32_t pad2_;
    const double* level_weight;  /* host, FEWHA_MAX_LEVELS + 1 entries, or NULL: the frequency-weighted
                                    ("modified") Jacobi preconditioner J = diag(w) diag(M) of Sec. 4, with
                                    w = level_weight[l - 1] on the detail coefficients of level l (1 =
                                    finest) and w = level_weight[levels] on the scaling coefficients of a
                                    layer with `levels` levels; entries used must be finite and > 0.
                                    Ignored when precond_inv is given. */
} fewha_config;

/* Written by the device at the end of every fewha_solve_aug. */
typedef struct {
    int32_t iters;          /* operator applications in the frame; with rel_tol > 0, the first
                               iteration whose residual met the tolerance */
    int32_t recycle_used;   /* recycled directions used for the projections */
    int32_t dropped;        /* Gram columns dropped as numerically dependent */
    int32_t flags;          /* bit 0: breakdown (non-finite value, or (p,q) <= 0 with (r, J^-1 r) != 0);
                               bit 1: rel_tol not met within the frame;
                               bit 2: warm start not taken (fewha_solve_aug_ws);
                               bit 3: right-hand side not finite, the frame was not solved */
    double rel_res;         /* ||r|| / ||b|| at the end of the frame (FP64); NaN with flag bit 3 */
} fewha_solve_info;

/* Device bytes the workspace of `cfg` needs. */
fewha_status fewha_workspace_size(const fewha_config* cfg, size_t* bytes);

/* Validate `cfg`, build the geometry tables, the prior D and the Jacobi preconditioner
 * J^-1 = 1/diag(M) (Sec. 4, computed exactly on the host from the separable structure
 * of the wavelet basis), copy them into `d_workspace` (device, >= fewha_workspace_size
 * bytes, 256-byte aligned) and return a context.  The recycle store is empty and the
 * carried state (c, r, b_prev) is zero.  Synchronises `stream` before returning. */
fewha_status fewha_setup(const fewha_config* cfg, void* d_workspace, size_t bytes, void* stream,
                         fewha_ctx** out);

/* Batch of independent instances solved together (throughput form of Alg. 3: every instance
 * is its own system of Sec. 3 with its own geometry, prior, preconditioner, carried state and
 * recycle store; each frame advances all of them).  cfgs: host array of n configurations
 * (1 <= n <= FEWHA_MAX_INSTANCES) that agree on precision, max_iter, recycle_k, recycle_mode,
 * project_all, rel_tol and block_elems.  The context's vectors are the concatenations over
 * instances in order (coefficients, slopes; see fewha_instances); every other entry point
 * works on the batch as on a single system, and d_info of fewha_solve_aug receives n
 * records.  An instance gets bit-identical results alone or in a batch (same block_elems).
 * fewha_setup / fewha_workspace_size are the n = 1 case. */
fewha_status fewha_workspace_size_batch(const fewha_config* cfgs, int32_t n, size_t* bytes);
fewha_status fewha_setup_batch(const fewha_config* cfgs, int32_t n, void* d_workspace, size_t bytes, void* stream,
                               fewha_ctx** out);

/* Instance offsets: coeff_offsets[i] / slope_offsets[i] for i <= n_inst (the last entry is the
 * total), host arrays of n entries (filled up to n); *n_out receives the instance count. */
fewha_status fewha_instances(const fewha_ctx* ctx, int64_t* coeff_offsets, int64_t* slope_offsets, int32_t n,
                             int32_t* n_out);

/* Number of coefficients N = sum_l n_l^2 and of slopes S = sum_g 2 n_sub,g^2 (totals over the
 * instances of a batch). */
fewha_status fewha_sizes(const fewha_ctx* ctx, int64_t* n_coeff, int64_t* n_slopes);

/* y = M x (equation for M, Sec. 3).  d_x, d_y: device, N elements; d_y must not alias d_x. */
fewha_status fewha_apply_A(fewha_ctx* ctx, const void* d_x, void* d_y, void* stream);

/* y = M x, as fewha_apply_A, for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid allocation): the operator's
 * intermediates (nodal image, two wavelet buffers, sensor nodes, layer adjoint field, weighted
 * slopes: 4 N + V + S elements, each block 256-byte aligned) live in a 16 MiB device array of
 * the library,
 * one per GPU, held until the process ends; its address is taken by fewha_setup on each
 * device.  Calls nothing that allocates (also no message strings).  FEWHA_E_NOMEM (nothing
 * launched) when the intermediates exceed 16 MiB; FEWHA_E_STATE when no context was set up on
 * the current device.  Every call on a GPU shares that GPU's array and overwrites all of it
 * that it uses, so calls that overlap on one GPU (other streams, other threads) race; the
 * results equal fewha_apply_A's bit for bit. */
fewha_status fewha_apply_A_noalloc(fewha_ctx* ctx, const void* d_x, void* d_y, void* stream);

/* b = W^-T A^T C_eta^-1 s (right-hand side, Sec. 3).  d_s: device, S; d_b: device, N. */
fewha_status fewha_rhs(fewha_ctx* ctx, const void* d_s, void* d_b, void* stream);

/* One frame of Alg. 3 (right-hand side, residual update, augmented PCG of Alg. 2) for the
 * slopes d_s (device, S): the carried coefficients c^(i), residual r^(i), previous
 * right-hand side b^(i) and recycled directions are updated in the context and the new
 * coefficients are written to d_c (device, N).  The first frame after setup or
 * fewha_reset runs Alg. 1 from r = b - M c.  d_info (device, may be NULL) receives a
 * fewha_solve_info. */
fewha_status fewha_solve_aug(fewha_ctx* ctx, const void* d_s, void* d_c, void* d_info, void* stream);

/* Iterations enqueued by the last fewha_solve_aug (max_iter; with rel_tol > 0 each instance's own
 * count is the iters of its fewha_solve_info). */
fewha_status fewha_frame_iterations(const fewha_ctx* ctx, int32_t* iters);

/* Drop the recycle store: the next solve runs Alg. 1 from r = b - M c with the carried c. */
fewha_status fewha_reset(fewha_ctx* ctx);

/* Operator pieces, for testing (in/out device, 16-byte aligned, element type of the context):
 *   FEWHA_PIECE_WINV  : coefficients (N) -> nodal layers (N), W^-1 = DWT^T / delta_l
 *   FEWHA_PIECE_WINVT : nodal layers (N) -> coefficients (N), W^-T = DWT / delta_l
 *   FEWHA_PIECE_A     : nodal layers (N) -> slopes (S), Gamma_g P_g summed over layers,
 *                       zero on inactive subapertures
 *   FEWHA_PIECE_AT    : slopes (S) -> nodal layers (N), sum_g P_g^T Gamma_g^T (inactive ignored) */
typedef enum { FEWHA_PIECE_WINV = 0, FEWHA_PIECE_WINVT = 1, FEWHA_PIECE_A = 2, FEWHA_PIECE_AT = 3 } fewha_piece;
fewha_status fewha_apply_piece(fewha_ctx* ctx, int32_t piece, const void* d_in, void* d_out, void* stream);

/* Copy the scaled prior alpha D (N) or the preconditioner J^-1 (N) in use to d_out (device,
 * element type of the context).  which: 0 = alpha D, 1 = J^-1. */
fewha_status fewha_get_vector(fewha_ctx* ctx, int32_t which, void* d_out, void* stream);

/* Checkpoint of the carried state (c, r, b_prev, recycle store and its bookkeeping).
 * fewha_state_size gives the bytes; get/set copy to/from a device buffer of that size.
 * Layout: 256-byte header of uint64 (magic, N, slots, element size, ring head, stored count,
 * previous iterations, first-frame flag, instances), then per instance `slots` doubles
 * (p_j, q_j) and one double (the number of real recycled directions at the end of the window,
 * used by tolerance-stopped frames), then c, r, b_prev (N each) and the ring U, Q (slots x N
 * each, slot-major). */
fewha_status fewha_state_size(const fewha_ctx* ctx, size_t* bytes);
fewha_status fewha_get_state(fewha_ctx* ctx, void* d_dst, void* stream);
fewha_status fewha_set_state(fewha_ctx* ctx, const void* d_src, void* stream);

/* Frame execution mode.  Enabled (the default): the first frame of every recycle-ring phase is
 * captured once into a HIP graph on a private stream and later frames replay it on `stream`.
 * The graph reads and writes only context memory: the weighted slope adjoint (the first
 * kernel of a frame) is launched before the graph on the caller's slopes, and one kernel after
 * it writes the frame statistics and copies c to the caller, so the caller's pointers may
 * change between frames.  Tolerance-stopped frames (rel_tol > 0) always launch directly.
 * Disabled: every kernel is launched individually.  Both modes give bit-identical results. */
fewha_status fewha_use_graphs(fewha_ctx* ctx, int32_t enable);

/* Diagnostic kernel profiler.  While enabled, every kernel launch of the compute calls is
 * bracketed by HIP events recorded on the call's stream and the call synchronises that
 * stream before returning (so a profiled run is not a latency measurement).
 * fewha_profile_read fills per-kernel totals (milliseconds and launch counts, host
 * arrays of n entries) accumulated since enabling and returns the number of kernels in
 * *n_out; fewha_kernel_name(i) names kernel i (NULL when out of range). */
fewha_status fewha_profile(fewha_ctx* ctx, int32_t enable);
fewha_status fewha_profile_read(const fewha_ctx* ctx, double* ms, int64_t* launches, int32_t n, int32_t* n_out);
const char* fewha_kernel_name(int32_t i);

/* Diagnostic timer of one operator kernel (profiler index 0-4: synthesis, fused data term,
 * propagation adjoint, tiled analysis, coarse analysis; `step` selects the tiled analysis
 * launch, see fewha_wavelet_steps; -1 times a whole application of M).  The kernel is launched `reps` times with
 * the arguments it has inside M x (input: the carried coefficients), captured into one graph and
 * replayed between two events recorded on `stream`; *avg_ms receives the mean duration.
 * Overwrites the context's scratch vectors (not the carried state).  Synchronises `stream`. */
fewha_status fewha_time_kernel(fewha_ctx* ctx, int32_t kernel, int32_t step, int32_t reps, void* stream,
                               float* avg_ms);

/* Tile shapes of the operator kernels that change no result bit: the synthesis image tile
 * (16, 32 or, FP32 only, 64; 0 = 16 when 32 would give fewer than 256 workgroups, else 32, the
 * default) and the layer
 * rows per thread of the propagation adjoint's gather (1: tiles of 8 x 32 nodes, 4: 32 x 32
 * with the sensor nodes staged in LDS; default 4 from 2^21 coefficients on). */
typedef struct {
    int32_t syn_tile;
    int32_t gather_rows;
    int32_t reserved[6];   /* zero */
} fewha_tuning;

fewha_status fewha_get_tuning(const fewha_ctx* ctx, fewha_tuning* t);   /* the shapes in use (syn_tile resolved) */
/* Selects tile shapes (FEWHA_E_INVAL for other values); drops the captured frame graphs. */
fewha_status fewha_set_tuning(fewha_ctx* ctx, const fewha_tuning* t);

/* Autotuner: times every combination of the tile shapes (synthesis 16 / 32 / 64 (FP32) x
 * gather rows 1 / 4) on `reps` applications of M to the carried coefficients, captured into a
 * graph and replayed between two events on `stream`; keeps the fastest in the context and
 * returns it in *best (may be NULL), the mean application time of each candidate in ms[0..n)
 * (order: syn 16 rows 1, syn 16 rows 4, syn 32 rows 1, syn 32 rows 4, syn 64 rows 1, syn 64
 * rows 4) and their count (4 in FP64, 6 in FP32) in *n_out.  The
 * caller stores *best and restores it with fewha_set_tuning on a later context of the same
 * configuration.  Overwrites the scratch vectors (not the carried state); synchronises
 * `stream`. */
fewha_status fewha_autotune(fewha_ctx* ctx, int32_t reps, void* stream, fewha_tuning* best, float* ms, int32_t n,
                            int32_t* n_out);

/* Tiled analysis launches of the context (finest levels first): the largest block each
 * transforms and the number of layers in it. */
fewha_status fewha_wavelet_steps(const fewha_ctx* ctx, int32_t* block_sizes, int32_t* layer_counts, int32_t n,
                                 int32_t* n_out);

/* Release the context (the workspace stays the caller's). */
fewha_status fewha_destroy(fewha_ctx* ctx);

/* Message of the last error on `ctx` (or of the last failed setup when ctx is NULL). */
const char* fewha_last_error(const fewha_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* FEWHA_H */
