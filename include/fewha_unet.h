/*
 * fewha_unet.h -- C ABI of the learned warm start of the augmented wavelet reconstructor:
 * a U-Net (4 levels of 32/64/128/256 channels, two 3x3 convolutions with bias and ReLU per
 * level, 2x2 average pooling, 2x nearest upsampling with skip concatenation, a 1x1 output
 * convolution) trained and evaluated by hand-written bfloat16 matrix-core kernels with FP32
 * accumulation.  The paper has no learned component; this is the learned extension of its
 * frame update: from the previous coefficients (as a nodal field) and the preconditioned new
 * residual it predicts a nodal correction of the initial guess of augmented PCG (Alg. 2),
 * which stays the solver and decides how much of the correction to take.
 *
 * Conventions
 *  - Images are grouped by size: group g holds images[g] images of size[g] x size[g] nodes
 *    (size a power of two in [16, 4096], at most 2^25 nodes per group).  Inputs are FP32 NHWC with 4 channels per node, groups one
 *    after the other; outputs are FP32, one value per node, in the same order.
 *  - Parameters are one FP32 vector in the order of the network: for each 3x3 convolution
 *    e0a e0b e1a e1b e2a e2b e3a e3b d2a d2b d1a d1b d0a d0b its weights [3][3][Cin][Cout]
 *    then its bias [Cout] (e0a has Cin = 32: channels 4..31 of its input are zero padding),
 *    then the output weights [32] and bias [1].  The network computes with the bfloat16
 *    rounding of the weights; FP32 master weights and the Adam moments live in the context.
 *  - All device buffers belong to the caller; the workspace passed to fewha_unet_setup
 *    belongs to the context until fewha_unet_destroy.  Calls are stream-ordered; argument
 *    errors are returned synchronously.
 */
#ifndef FEWHA_UNET_H
#define FEWHA_UNET_H

#include <stddef.h>
#include <stdint.h>

#include "fewha.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FEWHA_UNET_MAX_GROUPS 8

typedef struct fewha_unet fewha_unet;

typedef struct {
    int32_t abi_version;        /* FEWHA_ABI_VERSION */
    int32_t n_groups;           /* 1..FEWHA_UNET_MAX_GROUPS */
    int32_t images[FEWHA_UNET_MAX_GROUPS];
    int32_t size[FEWHA_UNET_MAX_GROUPS];
    float lr, beta1, beta2, eps;  /* Adam (Kingma and Ba): lr > 0, 0 <= beta < 1, eps > 0 */
} fewha_unet_config;

/* Device bytes of the workspace (parameters, Adam state, activations, gradients). */
fewha_status fewha_unet_workspace_size(const fewha_unet_config* cfg, size_t* bytes);

/* Context on a 256-byte aligned device workspace; parameters start at zero (set them with
 * fewha_unet_set_params).  Synchronises `stream`. */
fewha_status fewha_unet_setup(const fewha_unet_config* cfg, void* d_workspace, size_t bytes, void* stream,
                              fewha_unet** out);

/* Number of parameters (length of the parameter vector). */
fewha_status fewha_unet_num_params(const fewha_unet* net, int64_t* n);

/* Nodes per call (sum over groups of images x size^2). */
fewha_status fewha_unet_num_nodes(const fewha_unet* net, int64_t* n);

/* Load parameters (device, FP32, network order); resets the Adam moments and step count. */
fewha_status fewha_unet_set_params(fewha_unet* net, const float* d_params, void* stream);

/* Copy the FP32 master parameters (device, network order). */
fewha_status fewha_unet_get_params(fewha_unet* net, float* d_params, void* stream);

/* Forward pass: d_in (device, nodes x 4 FP32) -> d_out (device, nodes FP32). */
fewha_status fewha_unet_forward(fewha_unet* net, const float* d_in, float* d_out, void* stream);

/* Forward pass, mean-squared-error loss against d_target (device, nodes FP32) and the
 * gradients of every parameter (kept in the context; see fewha_unet_get_grads).  d_loss
 * (device, one FP32, may be NULL) receives the loss. */
fewha_status fewha_unet_backward(fewha_unet* net, const float* d_in, const float* d_target, float* d_loss,
                                 void* stream);

/* One Adam step with the gradients of the last fewha_unet_backward. */
fewha_status fewha_unet_adam_step(fewha_unet* net, void* stream);

/* Copy the gradients of the last fewha_unet_backward (device, FP32, network order). */
fewha_status fewha_unet_get_grads(fewha_unet* net, float* d_grads, void* stream);

/* Image groups of the context: images[g], size[g] for g < *n_groups (host arrays of
 * FEWHA_UNET_MAX_GROUPS entries). */
fewha_status fewha_unet_groups(const fewha_unet* net, int32_t* images, int32_t* size, int32_t* n_groups);

/* Normalisation of the warm start: network inputs W^-1 c / scale_c and W^-1 J^-1 r / scale_r
 * (then h_l / 20 km and gamma_l), output times scale_out is the nodal correction. */
typedef struct {
    float scale_c, scale_r, scale_out;
} fewha_warmstart;

/* One frame of Alg. 3 (see fewha_solve_aug) with a learned warm start between the residual
 * update and the Galerkin step: the network's nodal correction d gives the coefficient
 * correction e = W d (W = delta^2 W^-T per layer); one extra operator application gives M e,
 * and the frame takes the step tau = max(0, (e, r) / (e, M e)) that minimises the energy
 * 1/2 c^T M c - b^T c along e: c += tau e, r -= tau M e (info flag bit 2: tau = 0, the
 * correction was not taken).  ctx must hold a single instance whose
 * layers, in order, are the network's images (consecutive equal-size layers form a group).
 * Launches directly (no graph). */
fewha_status fewha_solve_aug_ws(fewha_ctx* ctx, fewha_unet* net, const fewha_warmstart* ws, const void* d_s,
                                void* d_c, void* d_info, void* stream);

/* The warm start's network input for the frame with slopes d_s (device, S) that follows the
 * coefficients d_c (device, N): with r = b - M c (b the right-hand side of d_s), every layer
 * node gets [W^-1 c / scale_c, W^-1 J^-1 r / scale_r, h_l / 20 km, gamma_l] (d_in: device,
 * N x 4 FP32, 16-byte aligned; scale_out unused).  This is the input fewha_solve_aug_ws forms
 * from its own residual; for collecting training samples.  ctx must hold a single instance.
 * Uses the context's scratch vectors; the carried state is not touched. */
fewha_status fewha_warmstart_input(fewha_ctx* ctx, const fewha_warmstart* ws, const void* d_c, const void* d_s,
                                   float* d_in, void* stream);

fewha_status fewha_unet_destroy(fewha_unet* net);
const char* fewha_unet_last_error(const fewha_unet* net);

#ifdef __cplusplus
}
#endif
#endif /* FEWHA_UNET_H */
