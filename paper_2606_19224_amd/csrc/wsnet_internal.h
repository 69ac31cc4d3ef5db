// Internal interface of the warm-start network kernels (wsnet.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

namespace cgd {

// Workspace layout of the network (byte offsets, 256-byte aligned).
struct WsLayout {
  size_t Wf[4], Wb[4], bias[4];   // packed BF16 weights (forward, backward-data), FP32 bias
  size_t act[4], out;             // activations (BF16), network output (FP32)
  size_t g4, ga, gb;              // gradients in the activations (training)
  size_t part, bpart, grad, lpart;
  int nwg;                        // weight-gradient workgroups
  size_t total;
};

size_t wsnet_param_count();
size_t wsnet_param_offset(int layer);
WsLayout wsnet_layout(int B, int M, int training);
hipError_t wsnet_pack(const float* params, unsigned char* ws, const WsLayout& L, hipStream_t s);
hipError_t wsnet_forward(int B, int M, const float* feat, unsigned char* ws, const WsLayout& L,
                         float* out, hipStream_t s);
hipError_t wsnet_loss_grad(int B, int M, const float* params, const float* feat,
                           const float* target, float* loss, float* grad, unsigned char* ws,
                           const WsLayout& L, hipStream_t s);
hipError_t wsnet_train_step(int B, int M, float* params, float* adam_m, float* adam_v, int step,
                            float lr, const float* feat, const float* target, float* loss,
                            unsigned char* ws, const WsLayout& L, hipStream_t s);
hipError_t wsnet_features(int n, int m, int N, int k, const float* Xf, const int32_t* idx,
                          const float* hw, const float* y, const float* rdiag, const float* eps,
                          float* feat, float* scale, float* Dtmp, float* var, double* cpart,
                          int* err, hipStream_t s);
hipError_t wsnet_z0(int m, int N, const float* out, const float* scale, float* z0, hipStream_t s);
hipError_t wsnet_target(int m, int N, const float* Z, const float* scale, float* target,
                        hipStream_t s);
hipError_t wsnet_jacobi_z0(int m, int N, const float* feat, const float* scale, float* z0,
                          hipStream_t s);
// z0 = s_j * net(features) in two launches for N <= 128 (rows pass with the
// forward weights converted alongside, then the fused network); larger N
// take features -> pack -> forward -> scale.  feat and scale are scratch.
hipError_t wsnet_predict_z0(int n, int m, int N, int k, const float* Xf, const int32_t* idx,
                           const float* hw, const float* y, const float* rdiag, const float* eps,
                           const float* params, float* z0, unsigned char* ws, const WsLayout& L,
                           float* Dtmp, float* var, double* cpart, int* err, float* feat,
                           float* scale, hipStream_t s);

}  // namespace cgd
