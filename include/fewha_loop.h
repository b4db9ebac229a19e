/*
 * fewha_loop.h -- C ABI of the closed-loop wrapper of the augmented wavelet reconstructor
 * (Sec. 5, Alg. 3): every frame turns the measured slopes into the next deformable-mirror
 * (DM) commands by
 *
 *   closed loop:  s_pol = s + H a^(i-1)              (pseudo-open-loop slopes, two-step delay)
 *   frame solve:  c^(i+1) from s_pol                 (fewha_solve_aug on the loop's context)
 *   fitting:      a~ = F W^-1 c^(i+1)
 *   gain control: closed  a^(i+1) = a^(i) + gain (a~ - a^(i-1))
 *                 open    a^(i+1) = (1 - gain) a^(i) + gain a~
 *
 * Readings (the paper is silent on the discrete forms):
 *  - A DM is a square grid of n actuators with spacing d at altitude h; actuator (a, b) sits at
 *    origin + ((b - (n-1)/2) d, (a - (n-1)/2) d), the layer-grid convention.  Its surface is the
 *    bilinear interpolant of the commands, zero outside the grid.
 *  - H (the "Gamma a" of Alg. 3) is the DM-to-sensor map: the DM surfaces at the cone-scaled,
 *    shifted sensor nodes (1 - h_d / H_g) x + theta_g h_d (Sec. 2 propagation), then the
 *    Shack-Hartmann operator; zero on inactive subapertures.
 *  - Fitting F (Sec. 6.1): fit_iter = 0, direct: the layers sit at the DM altitudes (one DM per
 *    layer) and the commands of DM d are layer d's function at its actuators.  fit_iter > 0,
 *    least squares: the commands minimise sum_theta sum_x |sum_d a_d(x + theta h_d) -
 *    sum_l phi_l(x + theta h_l)|^2 over the directions theta and the points x of an n_pts x n_pts
 *    pupil grid (spacing pupil_d / (n_pts - 1), inside the annulus of pupil_d and obstruction);
 *    fit_iter unpreconditioned CG iterations on its normal equations, started from the previous
 *    frame's fitted commands (zero after setup).  Layer functions are zero outside their grids.
 *
 * Conventions: commands are the concatenation over DMs of n_d^2 row-major values, in the
 * element type of the solver context; the loop holds a^(i-1), a^(i) and the last fitted a~.
 * The context must hold one instance; the loop uses it for the frame solve (its carried state
 * advances with every step) and must be destroyed before it.  Device buffers are the caller's;
 * the workspace passed to fewha_loop_setup belongs to the loop until fewha_loop_destroy.
 */
#ifndef FEWHA_LOOP_H
#define FEWHA_LOOP_H

#include <stddef.h>
#include <stdint.h>

#include "fewha.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FEWHA_LOOP_MAX_DM 8
#define FEWHA_LOOP_MAX_DIRS 64

typedef struct fewha_loop fewha_loop;

/* One deformable mirror (Sec. 6, system table). */
typedef struct {
    double height;      /* altitude h_d [m] */
    double spacing;     /* actuator spacing [m] */
    double origin_x;    /* grid centre [m] */
    double origin_y;
    int32_t n;          /* actuators per side, 2..1024 */
    int32_t pad_;
} fewha_dm;

typedef struct {
    int32_t abi_version;     /* FEWHA_ABI_VERSION */
    int32_t n_dm;            /* 1..FEWHA_LOOP_MAX_DM */
    const fewha_dm* dms;     /* host */
    double gain;             /* 0 < gain <= 1 (Sec. 6.1: 0.4) */
    int32_t closed;          /* 1: closed loop (pseudo-open-loop slopes), 0: open loop */
    int32_t fit_iter;        /* 0: direct fitting; 1..64: CG iterations of the least-squares fitting */
    int32_t n_dirs;          /* fitting directions (fit_iter > 0), 1..FEWHA_LOOP_MAX_DIRS */
    int32_t n_pts;           /* pupil grid points per side (fit_iter > 0), 2..512 */
    const double* dirs;      /* host, n_dirs (theta_x, theta_y) pairs [rad] */
    double pupil_d;          /* pupil diameter [m] of the fitting grid */
    double obstruction;      /* central obstruction (diameter ratio) of the fitting grid */
} fewha_loop_config;

/* Device bytes of the loop's workspace for the solver context ctx. */
fewha_status fewha_loop_workspace_size(const fewha_ctx* ctx, const fewha_loop_config* cfg, size_t* bytes);

/* Validate cfg against ctx (one instance; direct fitting: one DM at the altitude of every
 * layer), build the geometry tables into d_workspace (device, 256-byte aligned, >=
 * fewha_loop_workspace_size bytes) and return the loop with all commands zero.  Synchronises
 * `stream`. */
fewha_status fewha_loop_setup(fewha_ctx* ctx, const fewha_loop_config* cfg, void* d_workspace, size_t bytes,
                              void* stream, fewha_loop** out);

/* Number of actuators (sum of n_d^2). */
fewha_status fewha_loop_num_actuators(const fewha_loop* loop, int64_t* n);

/* One frame of Alg. 3: measured slopes d_s (device, S; closed loop: after the DMs) -> the next
 * commands a^(i+1) into d_a (device, actuators, may be NULL); d_info as for fewha_solve_aug.
 * Returns the frame solve's status (FEWHA_E_BREAKDOWN reports an earlier frame, see fewha.h). */
fewha_status fewha_loop_step(fewha_loop* loop, const void* d_s, void* d_a, void* d_info, void* stream);

/* Pieces, for testing:
 *   FEWHA_LOOP_DM_SLOPES: commands (actuators) -> H a (slopes, S; zero on inactive subapertures)
 *   FEWHA_LOOP_FIT:       coefficients (N) -> a~ = F W^-1 c (actuators), the CG started from the
 *                         loop's last fitted commands (which this call does not change) */
typedef enum { FEWHA_LOOP_DM_SLOPES = 0, FEWHA_LOOP_FIT = 1 } fewha_loop_piece_id;
fewha_status fewha_loop_piece(fewha_loop* loop, int32_t piece, const void* d_in, void* d_out, void* stream);

/* Read (which: 0 a^(i-1), 1 a^(i), 2 the last fitted a~) or set all three (NULL leaves one
 * unchanged) of the loop's commands; device buffers of `actuators` elements. */
fewha_status fewha_loop_get_commands(fewha_loop* loop, int32_t which, void* d_out, void* stream);
fewha_status fewha_loop_set_commands(fewha_loop* loop, const void* d_prev, const void* d_cur, const void* d_fit,
                                     void* stream);

fewha_status fewha_loop_destroy(fewha_loop* loop);

/* Message of the last error on `loop` (or of the last failed loop setup when loop is NULL). */
const char* fewha_loop_last_error(const fewha_loop* loop);

#ifdef __cplusplus
}
#endif
#endif /* FEWHA_LOOP_H */
