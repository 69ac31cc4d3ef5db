// Host side of the C ABI declared in include/cgd_wsnet.h.
#include "cgd_wsnet.h"
#include "internal.h"
#include "wsnet_internal.h"

namespace {

using namespace cgd;

// Feature scratch after the network layout: D (m x batch FP32), var (m),
// column partials (row blocks x batch doubles), error word, features
// (batch x m x 4) and scales (batch).
struct FeatLayout {
  size_t D, var, cpart, err, feat, scale, total;
};

FeatLayout feat_layout(size_t base, int B, int m) {
  FeatLayout F;
  size_t o = base;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (bytes + 255) & ~size_t(255);
    return at;
  };
  const size_t nblk = (size_t)(m + 7) / 8;  // row blocks of 8 or more rows
  F.D = take(4 * (size_t)m * B);
  F.var = take(4 * (size_t)m);
  F.cpart = take(8 * nblk * B);
  F.err = take(16);
  F.feat = take(16 * (size_t)m * B);
  F.scale = take(4 * (size_t)B);
  F.total = o;
  return F;
}

bool sizes_ok(int B, int m) {
  return B >= 1 && m >= 1 && (long long)B * m * 64 < (1LL << 31);
}

bool ws_ok(const void* ws, size_t have, size_t need) {
  return ws && have >= need && ((uintptr_t)ws & 255) == 0;
}

}  // namespace

extern "C" {

size_t cgd_wsnet_param_count(void) { return wsnet_param_count(); }

size_t cgd_wsnet_workspace_bytes(int batch, int m, int training) {
  if (!sizes_ok(batch, m) || (training != 0 && training != 1)) return 0;
  const WsLayout L = wsnet_layout(batch, m, training);
  return training ? L.total : feat_layout(L.total, batch, m).total;
}

cgd_status cgd_wsnet_features(int n, int m, int N, int k, const float* X_f, const int32_t* idx,
                              const float* w, const float* y, const float* r_diag,
                              const float* eps, float* feat, float* scale, void* workspace,
                              size_t ws_bytes, void* stream) {
  if (n < 1 || k < 1 || N < 2 || !sizes_ok(N, m)) return CGD_ERR_ARG;
  if (!X_f || !idx || !w || !y || !r_diag || !feat || !scale) return CGD_ERR_ARG;
  const WsLayout L = wsnet_layout(N, m, 0);
  const FeatLayout F = feat_layout(L.total, N, m);
  if (!ws_ok(workspace, ws_bytes, F.total)) return CGD_ERR_WORKSPACE;
  unsigned char* b = (unsigned char*)workspace;
  if (wsnet_features(n, m, N, k, X_f, idx, w, y, r_diag, eps, feat, scale, (float*)(b + F.D),
                     (float*)(b + F.var), (double*)(b + F.cpart), (int*)(b + F.err),
                     (hipStream_t)stream) != hipSuccess)
    return CGD_ERR_HIP;
  return CGD_OK;
}

cgd_status cgd_wsnet_forward(int batch, int m, const float* params, const float* feat,
                             float* out, void* workspace, size_t ws_bytes, void* stream) {
  if (!sizes_ok(batch, m) || !params || !feat || !out) return CGD_ERR_ARG;
  const WsLayout L = wsnet_layout(batch, m, 0);
  if (!ws_ok(workspace, ws_bytes, L.total)) return CGD_ERR_WORKSPACE;
  unsigned char* b = (unsigned char*)workspace;
  if (wsnet_pack(params, b, L, (hipStream_t)stream) != hipSuccess) return CGD_ERR_HIP;
  if (wsnet_forward(batch, m, feat, b, L, out, (hipStream_t)stream) != hipSuccess) return CGD_ERR_HIP;
  return CGD_OK;
}

cgd_status cgd_wsnet_infer(int n, int m, int N, int k, const float* X_f,
                                const int32_t* idx, const float* w, const float* y,
                                const float* r_diag, const float* eps, const float* params,
                                float* z0, void* workspace, size_t ws_bytes, void* stream) {
  if (n < 1 || k < 1 || N < 2 || !sizes_ok(N, m)) return CGD_ERR_ARG;
  if (!X_f || !idx || !w || !y || !r_diag || !params || !z0) return CGD_ERR_ARG;
  const WsLayout L = wsnet_layout(N, m, 0);
  const FeatLayout F = feat_layout(L.total, N, m);
  if (!ws_ok(workspace, ws_bytes, F.total)) return CGD_ERR_WORKSPACE;
  unsigned char* b = (unsigned char*)workspace;
  if (wsnet_predict_z0(n, m, N, k, X_f, idx, w, y, r_diag, eps, params, z0, b, L,
                       (float*)(b + F.D), (float*)(b + F.var), (double*)(b + F.cpart),
                       (int*)(b + F.err), (float*)(b + F.feat), (float*)(b + F.scale),
                       (hipStream_t)stream) != hipSuccess)
    return CGD_ERR_HIP;
  return CGD_OK;
}

cgd_status cgd_wsnet_loss_grad(int batch, int m, const float* params, const float* feat,
                               const float* target, float* loss, float* grad, void* workspace,
                               size_t ws_bytes, void* stream) {
  if (!sizes_ok(batch, m) || !params || !feat || !target || !loss || !grad) return CGD_ERR_ARG;
  const WsLayout L = wsnet_layout(batch, m, 1);
  if (!ws_ok(workspace, ws_bytes, L.total)) return CGD_ERR_WORKSPACE;
  if (wsnet_loss_grad(batch, m, params, feat, target, loss, grad, (unsigned char*)workspace, L,
                      (hipStream_t)stream) != hipSuccess)
    return CGD_ERR_HIP;
  return CGD_OK;
}

cgd_status cgd_wsnet_train_step(int batch, int m, float* params, float* adam_m, float* adam_v,
                                int step, float lr, const float* feat, const float* target,
                                float* loss, void* workspace, size_t ws_bytes,
                                void* stream) {
  if (!sizes_ok(batch, m) || step < 1 || !(lr > 0.f)) return CGD_ERR_ARG;
  if (!params || !adam_m || !adam_v || !feat || !target || !loss) return CGD_ERR_ARG;
  const WsLayout L = wsnet_layout(batch, m, 1);
  if (!ws_ok(workspace, ws_bytes, L.total)) return CGD_ERR_WORKSPACE;
  if (wsnet_train_step(batch, m, params, adam_m, adam_v, step, lr, feat, target, loss,
                       (unsigned char*)workspace, L, (hipStream_t)stream) != hipSuccess)
    return CGD_ERR_HIP;
  return CGD_OK;
}

cgd_status cgd_wsnet_target(int m, int N, const float* Z, const float* scale, float* target,
                            void* stream) {
  if (N < 1 || !sizes_ok(N, m) || !Z || !scale || !target) return CGD_ERR_ARG;
  return wsnet_target(m, N, Z, scale, target, (hipStream_t)stream) == hipSuccess ? CGD_OK
                                                                                 : CGD_ERR_HIP;
}

cgd_status cgd_wsnet_jacobi_z0(int m, int N, const float* feat, const float* scale, float* z0,
                               void* stream) {
  if (N < 1 || !sizes_ok(N, m) || !feat || !scale || !z0) return CGD_ERR_ARG;
  return wsnet_jacobi_z0(m, N, feat, scale, z0, (hipStream_t)stream) == hipSuccess
             ? CGD_OK
             : CGD_ERR_HIP;
}

}  // extern "C"
