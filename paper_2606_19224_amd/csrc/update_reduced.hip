// Ensemble update, CGD-EnKF-Reduced and input validation kernels (gfx950).
#include "internal.h"
#include "mfma_util.h"
#include "update_tile.h"

namespace cgd {

namespace {

// X_a = X_f + A W  (mode 0, Algorithm 1 with W = S^T Z/(N-1), A = X_f - xbar 1^T)
// X_a = X_f W      (mode 1, Algorithm 2)
// Each workgroup owns RBX whole rows: it stages them in LDS before writing,
// so X_a may alias X_f.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(int n, int N, int RBX, const T* Xf, T* Xa,
                                                   const double* Wd, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* tile = (double*)smem_raw;  // RBX * N
  double* mean = tile + (size_t)RBX * N;
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * RBX, rows = min(RBX, n - i0), ne = rows * N;
  if (rows <= 0) return;
  for (int e = tid; e < ne; e += kBlock) tile[e] = (double)Xf[(size_t)i0 * N + e];
  __syncthreads();
  if (mode == 0) {
    for (int i = tid; i < rows; i += kBlock) {
      double s = 0;
      for (int j = 0; j < N; ++j) s += tile[i * N + j];
      mean[i] = s / N;
    }
  }
  __syncthreads();
  for (int e = tid; e < ne; e += kBlock) {
    const int i = e / N, j = e - i * N;
    double acc = 0.0;
    if (mode == 0) {
      const double mu = mean[i];
      for (int kk = 0; kk < N; ++kk) acc += (tile[i * N + kk] - mu) * Wd[(size_t)kk * N + j];
      acc += tile[e];
    } else {
      for (int kk = 0; kk < N; ++kk) acc += tile[i * N + kk] * Wd[(size_t)kk * N + j];
    }
    Xa[(size_t)i0 * N + e] = (T)acc;
  }
}

// The same update on the 16x16x4 MFMA for N <= 128 (FP32) or N <= 64 (FP64):
// one workgroup per 64-row tile (see update_tile.h).
template <typename T, int NP>
__global__ __launch_bounds__(kBlock) void k_update_mfma(int n, int N, const T* Xf, T* Xa,
                                                        const double* Wd, int mode) {
  using C = UCfg<T, NP>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* As = (T*)smem_raw;
  T* Wt = As + (size_t)C::RBX * C::LD;
  double* mean = (double*)(Wt + (size_t)NP * C::LD);
  update_load_w<T, NP, kBlock>(N, Wd, mode, Wt);
  update_tile<T, NP, kBlock>(n, N, Xf, Xa, mode, blockIdx.x * C::RBX, As, Wt, mean);
}

template <typename T, int NP>
hipError_t launch_update_mfma(int n, int N, const T* Xf, T* Xa, const double* Wd, int mode,
                              hipStream_t s) {
  using C = UCfg<T, NP>;
  const hipError_t e = hipFuncSetAttribute((const void*)k_update_mfma<T, NP>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_update_mfma<T, NP>), dim3((n + C::RBX - 1) / C::RBX), dim3(kBlock), C::lds,
                     s, n, N, Xf, Xa, Wd, mode);
  return hipGetLastError();
}

// Reduced mode, step 1 (Algorithm 2 setup, Table 2 "N x N matrix form"):
// per row block, HX, zbar, P = (HX - zbar 1^T)/l_i and Yt = ((y - zbar) 1^T + E)/l_i
// with l_i = sqrt((N-1) r_i); partial [P^T P | P^T Yt] (N x 2N) per workgroup.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_red_gram(int n, int m, int N, int k, int RB, int nblk,
                                                     const T* Xf, const int32_t* idx,
                                                     const T* hw, const T* y, const T* rdiag,
                                                     const T* eps, double* part, int* err) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lp = (double*)smem_raw;           // RB * N
  double* ly = lp + (size_t)RB * N;         // RB * N
  double* lz = ly + (size_t)RB * N;         // RB
  const int tid = threadIdx.x, wg = blockIdx.x, nwg = gridDim.x;
  double* out = part + (size_t)wg * 2 * N * N;
  for (int b = wg; b < nblk; b += nwg) {
    const bool first = (b == wg);
    const int i0 = b * RB, rows = min(RB, m - i0), ne = rows * N;
    for (int e = tid; e < ne; e += kBlock) {
      const int i = e / N, j = e - i * N, gi = i0 + i;
      double h = 0;
      for (int t = 0; t < k; ++t) {
        const int c = idx[(size_t)gi * k + t];
        if ((unsigned)c < (unsigned)n)
          h += (double)hw[(size_t)gi * k + t] * (double)Xf[(size_t)c * N + j];
        else
          atomicOr(err, 2);
      }
      lp[e] = h;
    }
    __syncthreads();
    for (int i = tid; i < rows; i += kBlock) {
      double s = 0;
      for (int j = 0; j < N; ++j) s += lp[i * N + j];
      lz[i] = s / N;
    }
    __syncthreads();
    for (int e = tid; e < ne; e += kBlock) {
      const int i = e / N, gi = i0 + i;
      const double l = sqrt((double)(N - 1) * (double)rdiag[gi]);
      const double zb = lz[i];
      double yt = (double)y[gi] - zb;
      if (eps) yt += (double)eps[(size_t)i0 * N + e];
      lp[e] = (lp[e] - zb) / l;
      ly[e] = yt / l;
    }
    __syncthreads();
    for (int o = tid; o < 2 * N * N; o += kBlock) {
      const int half = o / (N * N), oo = o - half * N * N;
      const int kk = oo / N, j = oo - kk * N;
      const double* v = half ? ly : lp;
      double acc = 0;
      for (int i = 0; i < rows; ++i) acc += lp[i * N + kk] * v[i * N + j];
      out[o] = first ? acc : out[o] + acc;
    }
    __syncthreads();
  }
}

// G = I + sum_w P^T P,  B = I + sum_w P^T Yt  (fixed summation order).
__global__ __launch_bounds__(kBlock) void k_red_sum(int N, int nwg, const double* part, double* G,
                                                    double* B) {
  const int o = blockIdx.x * kBlock + threadIdx.x;
  if (o >= 2 * N * N) return;
  double acc = 0;
  for (int w = 0; w < nwg; ++w) acc += part[(size_t)w * 2 * N * N + o];
  const int half = o / (N * N), oo = o - half * N * N;
  const int kk = oo / N, j = oo - kk * N;
  acc += (kk == j) ? 1.0 : 0.0;
  (half ? B : G)[oo] = acc;
}

__device__ inline double bsum(double v, double* red) {
  const int tid = threadIdx.x;
  __syncthreads();
  red[tid] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double o = red[0];
  __syncthreads();
  return o;
}

// CGD-EnKF-Reduced solve: one workgroup per column j of B runs textbook CG
// on the N x N SPD system G w = b_j from w = 0 (Lemma 1: at most N steps in
// exact arithmetic).  Vectors live in LDS; G is read from L2 (symmetric, so
// q_k = sum_l G[l][k] p_l reads rows coalesced).
__global__ __launch_bounds__(kBlock) void k_small_cg(int N, const double* G, const double* B,
                                                     double* W, int* iters, double tol, int maxit) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* x = (double*)smem_raw;
  double* r = x + N;
  double* p = r + N;
  double* q = p + N;
  double* red = q + N;
  const int tid = threadIdx.x, j = blockIdx.x;
  double part = 0;
  for (int kk = tid; kk < N; kk += kBlock) {
    const double b = B[(size_t)kk * N + j];
    x[kk] = 0;
    r[kk] = b;
    p[kk] = b;
    part += b * b;
  }
  double rho = bsum(part, red);
  const double thr = tol * sqrt(rho);
  int it = 0;
  while (sqrt(rho) > thr && it < maxit && rho > 0.0) {
    part = 0;
    for (int kk = tid; kk < N; kk += kBlock) {
      double acc = 0;
      for (int l = 0; l < N; ++l) acc += G[(size_t)l * N + kk] * p[l];
      q[kk] = acc;
      part += p[kk] * acc;
    }
    const double pq = bsum(part, red);
    const double alpha = rho / pq;
    part = 0;
    for (int kk = tid; kk < N; kk += kBlock) {
      x[kk] += alpha * p[kk];
      r[kk] -= alpha * q[kk];
      part += r[kk] * r[kk];
    }
    const double rho_new = bsum(part, red);
    const double beta = rho_new / rho;
    for (int kk = tid; kk < N; kk += kBlock) p[kk] = r[kk] + beta * p[kk];
    __syncthreads();
    rho = rho_new;
    ++it;
    if (!isfinite(alpha) || !isfinite(beta)) break;
  }
  for (int kk = tid; kk < N; kk += kBlock) W[(size_t)kk * N + j] = x[kk];
  if (tid == 0) iters[j] = it;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_validate(int n, int m, int N, int k, const T* Xf,
                                                     const int32_t* idx, const T* hw, const T* y,
                                                     const T* rdiag, const T* eps, const T* z0,
                                                     int* flags) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  const size_t t0 = (size_t)blockIdx.x * kBlock + threadIdx.x;
  int f = 0;
  for (size_t e = t0; e < (size_t)n * N; e += stride)
    if (!isfinite((double)Xf[e])) f |= VF_NONFINITE;
  for (size_t e = t0; e < (size_t)m * k; e += stride) {
    if (idx[e] < 0 || idx[e] >= n) f |= VF_INDEX;
    if (!isfinite((double)hw[e])) f |= VF_NONFINITE;
  }
  for (size_t e = t0; e < (size_t)m; e += stride) {
    if (!isfinite((double)y[e]) || !isfinite((double)rdiag[e])) f |= VF_NONFINITE;
    if (!(rdiag[e] > (T)0)) f |= VF_NONPOS_R;
  }
  if (eps)
    for (size_t e = t0; e < (size_t)m * N; e += stride)
      if (!isfinite((double)eps[e])) f |= VF_NONFINITE;
  if (z0)
    for (size_t e = t0; e < (size_t)m * N; e += stride)
      if (!isfinite((double)z0[e])) f |= VF_NONFINITE;
  if (f) atomicOr(flags, f);
}

inline int update_rows(int N) {
  int r = (int)((32 * 1024) / (sizeof(double) * (size_t)N + 8));
  if (r > 64) r = 64;
  return r < 1 ? 1 : r;
}

}  // namespace

template <typename T>
hipError_t launch_update(int n, int N, const T* Xf, T* Xa, const double* Wd, int mode,
                         hipStream_t s) {
  if (N <= 16) return launch_update_mfma<T, 16>(n, N, Xf, Xa, Wd, mode, s);
  if (N <= 32) return launch_update_mfma<T, 32>(n, N, Xf, Xa, Wd, mode, s);
  if (N <= 64) return launch_update_mfma<T, 64>(n, N, Xf, Xa, Wd, mode, s);
  if constexpr (sizeof(T) == 4)
    if (N <= 128) return launch_update_mfma<T, 128>(n, N, Xf, Xa, Wd, mode, s);
  // larger ensembles: one double FMA chain per element
  const int RBX = update_rows(N);
  const size_t sh = sizeof(double) * ((size_t)RBX * N + RBX);
  hipLaunchKernelGGL(k_update<T>, dim3((n + RBX - 1) / RBX), dim3(kBlock), sh, s, n, N, RBX, Xf,
                     Xa, Wd, mode);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reduced(int n, int m, int N, int k, const T* Xf, T* Xa, const int32_t* idx,
                          const T* hw, const T* y, const T* rdiag, const T* eps, double tol,
                          int maxit, void* ws, const Layout& L, int* iters_out, hipStream_t s) {
  unsigned char* base = (unsigned char*)ws;
  double* part = (double*)(base + L.rpart);
  double* G = (double*)(base + L.rG);
  double* B = (double*)(base + L.rB);
  double* Wd = (double*)(base + L.Wd);
  int* iters = iters_out ? iters_out : (int*)(base + L.riters);
  const int nwg = L.nwg_max;
  const size_t sh = sizeof(double) * (2 * (size_t)L.RB * N + L.RB);
  int* err = (int*)(base + L.err);
  hipError_t e = launch_zero_u32((unsigned*)err, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_red_gram<T>, dim3(nwg), dim3(kBlock), sh, s, n, m, N, k, L.RB, L.nblk, Xf,
                     idx, hw, y, rdiag, eps, part, err);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_red_sum, dim3((2 * N * N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, N,
                     nwg, part, G, B);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_small_cg, dim3(N), dim3(kBlock), sizeof(double) * (4 * (size_t)N + kBlock),
                     s, N, G, B, Wd, iters, tol, maxit);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (iters != (int*)(base + L.riters))
    if ((e = hipMemcpyAsync(base + L.riters, iters, sizeof(int) * N, hipMemcpyDeviceToDevice, s)) !=
        hipSuccess)
      return e;
  return launch_update<T>(n, N, Xf, Xa, Wd, 1, s);
}

template <typename T>
hipError_t launch_validate(int n, int m, int N, int k, const T* Xf, const int32_t* idx,
                           const T* hw, const T* y, const T* rdiag, const T* eps, const T* z0,
                           int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_validate<T>, dim3(512), dim3(kBlock), 0, s, n, m, N, k, Xf, idx, hw, y,
                     rdiag, eps, z0, flags);
  return hipGetLastError();
}

#define CGD_INST(T)                                                                              \
  template hipError_t launch_update<T>(int, int, const T*, T*, const double*, int, hipStream_t); \
  template hipError_t launch_reduced<T>(int, int, int, int, const T*, T*, const int32_t*,        \
                                        const T*, const T*, const T*, const T*, double, int,     \
                                        void*, const Layout&, int*, hipStream_t);                \
  template hipError_t launch_validate<T>(int, int, int, int, const T*, const int32_t*, const T*, \
                                         const T*, const T*, const T*, const T*, int*,           \
                                         hipStream_t);
CGD_INST(double)
CGD_INST(float)

}  // namespace cgd
