// Non-diagonal observation covariance R = L L^T with a lower-bidiagonal L
// (Section 5.1; the tridiagonal Toeplitz R of Section 5.3 and Example 2).
//
// The analysis whitens the observation space by L: with S~ = L^{-1} S and
// D~ = L^{-1} D the innovation system L^{-1} Psi L^{-T} (L^T z) = L^{-1} d
// has the matrix I + S~ S~^T/(N-1), and W = S^T Z/(N-1) = S~^T Z~/(N-1).  So
// the solvers run unchanged on a problem whose observations are S~ itself:
// rows X' = S~ (already centred), H = I, y' = 0, perturbations
// E' = D~ + S~ (so that y' + E' - H X' = D~) and R' = I, with the update
// applied to the real X_f.  This is CG preconditioned by M = R (the L^{-1}
// scaling of Algorithm 2 applied to the full system), exact for any R with
// such a factor.  The kernels here build that problem, map a warm start to
// the whitened variables (z~0 = L^T z0) and a solution back
// (z = L^{-T} z~), and factor a symmetric tridiagonal R.
//
// L is given as 2m-1 values: its diagonal (m), then its subdiagonal (m-1),
// e[i] = L[i+1][i].
#include "internal.h"

namespace cgd {

namespace {

constexpr int kWB = 256;

// Row i: HX (double) from X_f, idx, w; S = HX - mean (centred rows), D =
// y + eps - HX; both in double.  One thread per row.
template <typename T>
__global__ __launch_bounds__(kWB) void k_tri_rows(int n, int m, int N, int k, const T* Xf,
                                                  const int32_t* idx, const T* hw, const T* y,
                                                  const T* eps, double* Sd, double* Dd,
                                                  int* err) {
  const int i = blockIdx.x * kWB + threadIdx.x;
  if (i >= m) return;
  double sum = 0.0;
  for (int j = 0; j < N; ++j) {
    double h = 0.0;
    for (int t = 0; t < k; ++t) {
      const int c = idx[(size_t)i * k + t];
      if ((unsigned)c < (unsigned)n)
        h += (double)hw[(size_t)i * k + t] * (double)Xf[(size_t)c * N + j];
      else
        atomicOr(err, 2);
    }
    Sd[(size_t)i * N + j] = h;
    sum += h;
  }
  const double mean = sum / N, yi = (double)y[i];
  for (int j = 0; j < N; ++j) {
    const size_t g = (size_t)i * N + j;
    const double h = Sd[g];
    Sd[g] = h - mean;
    Dd[g] = yi - h + (eps ? (double)eps[g] : 0.0);
  }
}

// Member j: S~ = L^{-1} S and D~ = L^{-1} D by forward substitution down the
// rows (x_0 = b_0 / d_0, x_i = (b_i - e_{i-1} x_{i-1}) / d_i), in double;
// writes X'[i][j] = S~_ij and E'[i][j] = D~_ij + S~_ij.  Thread j < N also
// fills rows j, j + N, ... of the constant arrays idx' = i, w' = 1, y' = 0,
// R' = 1.  The loads of a row are independent of the recurrence, so U rows
// are requested ahead.
template <typename T>
__global__ __launch_bounds__(kWB) void k_tri_fwd(int m, int N, const T* Lf, const double* Sd,
                                                 const double* Dd, T* Xp, T* Ep, int32_t* idxp,
                                                 T* wp, T* yp, T* rp) {
  const int j = blockIdx.x * kWB + threadIdx.x;
  if (j >= N) return;
  for (int i = j; i < m; i += N) {
    idxp[i] = i;
    wp[i] = (T)1;
    yp[i] = (T)0;
    rp[i] = (T)1;
  }
  const T* dg = Lf;
  const T* sub = Lf + m;
  constexpr int U = 8;
  double xs = 0.0, xd = 0.0;
  for (int i0 = 0; i0 < m; i0 += U) {
    double bs[U], bd[U], di[U], ei[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u;
      const bool live = i < m;
      bs[u] = live ? Sd[(size_t)i * N + j] : 0.0;
      bd[u] = live ? Dd[(size_t)i * N + j] : 0.0;
      di[u] = live ? (double)dg[i] : 1.0;
      ei[u] = (live && i > 0) ? (double)sub[i - 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u;
      if (i < m) {
        xs = (bs[u] - ei[u] * xs) / di[u];
        xd = (bd[u] - ei[u] * xd) / di[u];
        Xp[(size_t)i * N + j] = (T)xs;
        Ep[(size_t)i * N + j] = (T)(xd + xs);
      }
    }
  }
}

// Warm start in the whitened variables: z~0 = L^T z0, row i =
// d_i z0_i + e_i z0_{i+1} (the last row has no second term).
template <typename T>
__global__ __launch_bounds__(kWB) void k_tri_z0(int m, int N, const T* Lf, const T* z0, T* zt) {
  const long total = (long)m * N;
  for (long e = (long)blockIdx.x * kWB + threadIdx.x; e < total; e += (long)gridDim.x * kWB) {
    const int i = (int)(e / N);
    double v = (double)Lf[i] * (double)z0[e];
    if (i + 1 < m) v += (double)Lf[m + i] * (double)z0[e + N];
    zt[e] = (T)v;
  }
}

// A solution back from the whitened variables, in place: z = L^{-T} z~ by
// backward substitution (z_{m-1} = z~_{m-1} / d_{m-1},
// z_i = (z~_i - e_i z_{i+1}) / d_i).  One thread per member.
template <typename T>
__global__ __launch_bounds__(kWB) void k_tri_back(int m, int N, const T* Lf, T* z) {
  const int j = blockIdx.x * kWB + threadIdx.x;
  if (j >= N) return;
  double x = 0.0;
  for (int i = m - 1; i >= 0; --i) {
    const double e = i + 1 < m ? (double)Lf[m + i] : 0.0;
    x = ((double)z[(size_t)i * N + j] - e * x) / (double)Lf[i];
    z[(size_t)i * N + j] = (T)x;
  }
}

// Cholesky factor of the symmetric tridiagonal R (diagonal r, off-diagonal
// o): d_0 = sqrt(r_0), e_i = o_i / d_i, d_{i+1} = sqrt(r_{i+1} - e_i^2), in
// double.  A pivot that is not positive or not finite leaves d_0 = -1 (the
// host checks d_0); `bad` is unused.
template <typename T>
__global__ void k_tri_chol(int m, const T* r, const T* o, T* Lf, int* bad) {
  (void)bad;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double p = (double)r[0];
  int b = !(p > 0.0) || !isfinite(p);
  double d = sqrt(p);
  const double d0 = d;
  for (int i = 0; i + 1 < m; ++i) {
    const double e = (double)o[i] / d;
    p = (double)r[i + 1] - e * e;
    if (!(p > 0.0) || !isfinite(p)) b = 1;
    d = sqrt(p);
    Lf[m + i] = (T)e;
    Lf[i + 1] = (T)d;
  }
  Lf[0] = b ? (T)-1 : (T)d0;
}

}  // namespace

template <typename T>
hipError_t launch_tri_whiten(int n, int m, int N, int k, const T* Xf, const int32_t* idx,
                             const T* hw, const T* y, const T* eps, const T* Lf, const T* z0,
                             const TriBuffers<T>& tb, int* err, hipStream_t s) {
  hipError_t e = launch_zero_u32((unsigned*)err, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tri_rows<T>, dim3((m + kWB - 1) / kWB), dim3(kWB), 0, s, n, m, N, k, Xf,
                     idx, hw, y, eps, tb.Sd, tb.Dd, err);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tri_fwd<T>, dim3((N + kWB - 1) / kWB), dim3(kWB), 0, s, m, N, Lf,
                     (const double*)tb.Sd, (const double*)tb.Dd, tb.Xp, tb.Ep, tb.idxp, tb.wp,
                     tb.yp, tb.rp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (z0) {
    long nb = ((long)m * N + kWB - 1) / kWB;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_tri_z0<T>, dim3((unsigned)nb), dim3(kWB), 0, s, m, N, Lf, z0, tb.zt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void k_or_u32(int* dst, const int* src) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && *src) atomicOr(dst, *src);
}

hipError_t launch_or_u32(int* dst, const int* src, hipStream_t s) {
  hipLaunchKernelGGL(k_or_u32, dim3(1), dim3(64), 0, s, dst, src);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tri_back(int m, int N, const T* Lf, T* z, hipStream_t s) {
  hipLaunchKernelGGL(k_tri_back<T>, dim3((N + kWB - 1) / kWB), dim3(kWB), 0, s, m, N, Lf, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tri_chol(int m, const T* r, const T* o, T* Lf, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_tri_chol<T>, dim3(1), dim3(64), 0, s, m, r, o, Lf, bad);
  return hipGetLastError();
}

#define CGD_TRI_INST(T)                                                                          \
  template hipError_t launch_tri_whiten<T>(int, int, int, int, const T*, const int32_t*,         \
                                           const T*, const T*, const T*, const T*, const T*,     \
                                           const TriBuffers<T>&, int*, hipStream_t);             \
  template hipError_t launch_tri_back<T>(int, int, const T*, T*, hipStream_t);                   \
  template hipError_t launch_tri_chol<T>(int, const T*, const T*, T*, int*, hipStream_t);
CGD_TRI_INST(double)
CGD_TRI_INST(float)

}  // namespace cgd
