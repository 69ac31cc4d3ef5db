/* Learned warm start for the CGD-EnKF solve: a small 1-D convolutional
 * network that predicts the CG starting point z0 of every member from
 * observation-space features, and the kernels that train it on the GPU.
 *
 * The paper has no learned component; the solve it accelerates is the CG of
 * Section 3 (a better z0 shortens the Krylov iteration, Props. 1 and 3 bound
 * the error by the initial error in the Psi-norm).  The library only ever
 * uses the prediction as a warm start with the stall fallback of
 * cgd_options.fallback_on_stall, so a poor prediction costs iterations, never
 * accuracy.
 *
 * Network (fixed architecture): features per member j and observation i
 *   f = (d_ij / s_j, (S S^T)_ii / (N-1), r_i),  s_j = RMS over i of d_ij,
 * four circular conv1d layers of width 5 along i with 3 -> 64 -> 64 -> 64 -> 1
 * channels and ReLU between layers, output net_j; z0_ij = s_j * net_j(i).
 * Operands are BF16 on the MFMA with FP32 accumulation; the parameters are an
 * FP32 vector of cgd_wsnet_param_count() values: for each layer the weights
 * W[o][c][t] (t the tap, o the output and c the input channel) then the
 * bias b[o].
 *
 * No paper source: the network, its features and its training are an
 * extension of the method; the paper's part is the CG it warm-starts.
 *
 * All arrays are device pointers owned by the caller, FP32 unless stated,
 * row-major.  Workspaces are caller-allocated (256-byte aligned).  Calls are
 * stream-ordered and asynchronous (`stream` is a hipStream_t, NULL = the
 * null stream); none allocates.  Errors: CGD_ERR_ARG for
 * invalid sizes or NULL pointers, CGD_ERR_WORKSPACE for a short or
 * misaligned workspace, CGD_ERR_HIP when a launch fails.  Out-of-range
 * observation indices are not reported by these calls (the analysis reports
 * them). */
#ifndef CGD_WSNET_H
#define CGD_WSNET_H

#include <stddef.h>
#include <stdint.h>

#include "cgd_enkf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of FP32 parameters (weights and biases of the four layers). */
size_t cgd_wsnet_param_count(void);

/* Workspace bytes for `batch` members (or training pairs) on a chain of m
 * observations: training = 0 for cgd_wsnet_forward / cgd_wsnet_predict_z0 /
 * cgd_wsnet_features, 1 for cgd_wsnet_train_step.  0 for invalid sizes. */
size_t cgd_wsnet_workspace_bytes(int batch, int m, int training);

/* Features of one analysis (inputs as for cgd_enkf_analysis, FP32):
 * feat [N][m][4] = (d_ij/s_j, diag(SS^T)_i/(N-1), r_i, 0) and scale [N] = s_j,
 * with d_j = y + eps_j - H x_j (eps may be NULL) and HX in double. */
cgd_status cgd_wsnet_features(int n, int m, int N, int k, const float* X_f, const int32_t* idx,
                              const float* w, const float* y, const float* r_diag,
                              const float* eps, float* feat, float* scale, void* workspace,
                              size_t ws_bytes, void* stream);

/* Network output out [batch][m] for features feat [batch][m][4]. */
cgd_status cgd_wsnet_forward(int batch, int m, const float* params, const float* feat,
                             float* out, void* workspace, size_t ws_bytes, void* stream);

/* Inference: the warm start of one analysis, z0 [m][N] (the layout of
 * cgd_options.z0) = s_j * network(features)_j.  Workspace:
 * cgd_wsnet_workspace_bytes(N, m, 0). */
cgd_status cgd_wsnet_infer(int n, int m, int N, int k, const float* X_f, const int32_t* idx,
                           const float* w, const float* y, const float* r_diag, const float* eps,
                           const float* params, float* z0, void* workspace, size_t ws_bytes,
                           void* stream);

/* Loss and gradient without an update: *loss (device FP32) = mean squared
 * error of the network on feat against target, grad (param_count values) its
 * gradient in the parameters.  Workspace: cgd_wsnet_workspace_bytes(batch, m, 1). */
cgd_status cgd_wsnet_loss_grad(int batch, int m, const float* params, const float* feat,
                               const float* target, float* loss, float* grad, void* workspace,
                               size_t ws_bytes, void* stream);

/* One training step on `batch` pairs: forward, mean-squared-error loss
 * against target [batch][m] (the converged z_j / s_j), backward, and one Adam
 * update (betas 0.9, 0.999, eps 1e-8, bias correction with step >= 1) of
 * params with its moment vectors adam_m, adam_v (each param_count values,
 * zero before the first step).  *loss (device FP32) receives the loss before
 * the update.  Workspace: cgd_wsnet_workspace_bytes(batch, m, 1). */
cgd_status cgd_wsnet_train_step(int batch, int m, float* params, float* adam_m, float* adam_v,
                                int step, float lr, const float* feat, const float* target,
                                float* loss, void* workspace, size_t ws_bytes,
                                void* stream);

/* Training target of one analysis: target [N][m] = Z[i][j] / s_j, from the
 * converged solution Z [m][N] (cgd_options.z_out of a zero-start analysis)
 * and the scales s [N] of cgd_wsnet_features.  No workspace. */
cgd_status cgd_wsnet_target(int m, int N, const float* Z, const float* scale, float* target,
                            void* stream);

/* The non-learned comparison start (Jacobi): z0 [m][N] = d_ij / Psi_ii with
 * Psi_ii = (S S^T)_ii/(N-1) + r_i, from the features [N][m][4] and scales
 * of cgd_wsnet_features (d_ij = s_j f0, Psi_ii = f1 + f2).  No workspace. */
cgd_status cgd_wsnet_jacobi_z0(int m, int N, const float* feat, const float* scale, float* z0,
                               void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CGD_WSNET_H */
