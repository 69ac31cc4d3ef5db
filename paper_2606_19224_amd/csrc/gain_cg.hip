// Explicit-gain CGD-EnKF (Figure 2; Section 3.1, eqs. K_KF_T and
// K_KF_T_rewrite) on gfx950: every column i of K^T (one per state variable)
// solves Psi_z (K^T e_i) = Psi_x^T e_i by its own CG recurrence from zero,
// then X_a = X_f + K (Y - Z).  The n right-hand sides are b_i = S a_i/(N-1)
// (a_i the anomaly row of state i), so the work is that of Algorithm 1 with
// n columns in place of N.
//
// Launches: the error word's clear, k_kt_rows (padded rows of S, D, diag(R)
// and A/(N-1)), k_kt_cg (one workgroup per 16 columns of K^T over all m rows;
// no workgroup waits for another).  In k_kt_cg each CG step is one pass over
// the rows with both S-products on the 16x16x4 MFMA (see k_kt_cg).  The
// vectors of a workgroup's 16 columns live in the workspace, row-major with
// 16 columns per row.
#include "modes.h"
#include "mfma_util.h"

namespace cgd {

namespace {

constexpr int kKtWaves = 8;
constexpr int kKtBlock = 64 * kKtWaves;
constexpr int kKtRowAlign = 16 * kKtWaves;  // m padded so every wave owns whole 16-row blocks

int kt_np(int N) { return N <= 16 ? 16 : N <= 32 ? 32 : N <= 64 ? 64 : 128; }
int kt_mp(int m) { return (m + kKtRowAlign - 1) / kKtRowAlign * kKtRowAlign; }
int kt_nn(int n) { return (n + 15) / 16 * 16; }

// Observation rows first (blocks [0, mp/RPB)), then state rows:
//   S[i] = H X_f row - zbar, D[i] = y_i + eps_i - H X_f row, rd[i] = r_i
//   (zero past N; rows past m zero, rd = 1);
//   A[i] = (X_f row - xbar)/(N-1) (zero past N and past n, up to nn rows).
// One group of NP/4 lanes per row, 4 members per lane.  An index out of range
// sets bit 2 of *err.
template <typename T, int NP>
__global__ __launch_bounds__(kBlock) void k_kt_rows(int n, int m, int N, int k, int mp, int nn,
                                                    const T* Xf, const int32_t* idx,
                                                    const T* hw, const T* y, const T* rdiag,
                                                    const T* eps, T* S, T* D, T* rd, T* A,
                                                    int* err) {
  constexpr int LPR = NP / 4, RPB = kBlock / LPR;
  const int tid = threadIdx.x, q = tid % LPR;
  const int mblk = mp / RPB;
  const bool obs = (int)blockIdx.x < mblk;
  const int i = (obs ? (int)blockIdx.x : (int)blockIdx.x - mblk) * RPB + tid / LPR;
  double h[4] = {0.0, 0.0, 0.0, 0.0};
  bool bad = false;
  if (obs) {
    if (i < m) {
      for (int t = 0; t < k; ++t) {
        const int c = idx[(size_t)i * k + t];
        if ((unsigned)c >= (unsigned)n) {
          bad = true;
          continue;
        }
        const double wt = (double)hw[(size_t)i * k + t];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (4 * q + u < N) h[u] += wt * (double)Xf[(size_t)c * N + 4 * q + u];
      }
    }
  } else if (i < n) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (4 * q + u < N) h[u] = (double)Xf[(size_t)i * N + 4 * q + u];
  }
  // every lane takes part in the group sum; empty rows carry zeros
  const double mean = group_sum<LPR>((h[0] + h[1]) + (h[2] + h[3])) / N;
  if (bad) atomicOr(err, 2);
  if (obs) {
    const bool live = i < m;
    const double yv = live ? (double)y[i] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = 4 * q + u;
      double sv = 0.0, dv = 0.0;
      if (live && j < N) {
        sv = h[u] - mean;
        dv = yv + (eps ? (double)eps[(size_t)i * N + j] : 0.0) - h[u];
      }
      S[(size_t)i * NP + j] = (T)sv;
      D[(size_t)i * NP + j] = (T)dv;
    }
    if (q == 0) rd[i] = live ? rdiag[i] : (T)1;
  } else if (i < nn) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = 4 * q + u;
      const double av = (i < n && j < N) ? (h[u] - mean) / (N - 1) : 0.0;
      A[(size_t)i * NP + j] = (T)av;
    }
  }
}

// 16 rows rb.. of S times g (NP x 16 in LDS, g[j][c] at j * 16 + c, kept in
// double and rounded to T for the MFMA): lane (lr, lk) supplies
// S[rb + lr][lk NP/4 + t] (a contiguous run) and g[lk NP/4 + t][lr] for
// t < NP/4, so the summation over j is split into four contiguous quarters,
// one per lane group.  Result rows frag_row(lk, v), column lr.
template <typename T, int NP>
__device__ __attribute__((always_inline)) inline typename Vec4<T>::type
kt_sg(const T* S, const double* g, int rb, int lr, int lk) {
  constexpr int KS = NP / 4, CH = KS < 8 ? KS : 8;  // S in chunks of 8 (register pressure)
  using V = typename Vec4<T>::type;
  const T* srow = S + (size_t)(rb + lr) * NP + lk * KS;
  V acc = {0, 0, 0, 0};
#pragma unroll
  for (int t0 = 0; t0 < KS; t0 += CH) {
    T sv[CH];
    vload<CH>(srow + t0, sv);
#pragma unroll
    for (int t = 0; t < CH; ++t) acc = mfma4(sv[t], (T)g[(lk * KS + t0 + t) * 16 + lr], acc);
  }
  return acc;
}

__device__ inline double lane_col_sum(double v) {  // over the four lanes of one column
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// One pass over the rows per CG step, the recurrence of Algorithm 1's solver
// rearranged so that alpha of the next step is known when the pass ends (the
// same iterates in exact arithmetic).  With r_i = diag(R), a pass applies the
// direction p = r + beta p_prev (formed as the rows are read) whose
// g = S^T p is held in LDS:
//   q = S g/(N-1) + r o p,  z += alpha p,  r' = r - alpha q,
// and forms for the next step
//   g' = S^T r' (MFMA),  rho = |r'|^2,  a = sum r_i r'^2,  b = sum r_i r' p,
//   c = sum r_i p^2;
// then beta' = rho/rho_prev, S^T p' = g' + beta' g and
//   p'^T Psi p' = |S^T p'|^2/(N-1) + a + 2 beta' b + beta'^2 c.
template <typename T, int NP>
__global__ __launch_bounds__(kKtBlock) void k_kt_cg(int n, int m, int mp, int N, const T* S,
                                                    const T* D, const T* rd, const T* A,
                                                    const T* Xf, T* Xa, T* Zv, T* Rv, T* Pv,
                                                    T* kt, double tol, int maxit, int* iters,
                                                    double* hist, int* status) {
  using V = typename Vec4<T>::type;
  constexpr int NB = NP / 16;
  // per-wave partials of S^T r' (and of K D), then g = S^T p: kt_lds<T>(NP) bytes
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T (*gp)[NP * 16] = reinterpret_cast<T (*)[NP * 16]>(smem_raw);
  double* gd = reinterpret_cast<double*>(smem_raw + sizeof(T) * kKtWaves * NP * 16);
  __shared__ double cr[kKtWaves][4][16];
  __shared__ double s_alpha[16], s_beta[16], s_rho[16], s_thr[16], s_a[16], s_b[16], s_c[16];
  __shared__ int s_it[16], s_act[16], s_st[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int cb = blockIdx.x;
  const size_t vb = (size_t)cb * mp * 16;
  T* Z = Zv + vb;
  T* R = Rv + vb;
  T* P = Pv + vb;
  const int rows = mp / kKtWaves, r0 = wv * rows;
  const double inv = 1.0 / (N - 1);

  // One pass over this wave's rows.  init: r = S g with g the block's 16
  // anomaly rows (already / (N-1)), p = z = 0.  Leaves the wave's partials of
  // S^T r' in gp[wv] and of rho, a, b, c in cr[wv].
  auto pass = [&](bool init) {
    const double alpha = s_alpha[lr], beta = s_beta[lr];
    V acc[NB];
#pragma unroll
    for (int x = 0; x < NB; ++x) acc[x] = V{0, 0, 0, 0};
    double s_rr = 0.0, s_ra = 0.0, s_rb = 0.0, s_rc = 0.0;
    for (int rb = r0; rb < r0 + rows; rb += 16) {
      const V qv = kt_sg<T, NP>(S, gd, rb, lr, lk);
      T rn[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rb + frag_row<T>(lk, v);
        const size_t e = (size_t)row * 16 + lr;
        const double ri = (double)rd[row];
        if (init) {
          rn[v] = qv[v];
          R[e] = rn[v];
          P[e] = (T)0;
          Z[e] = (T)0;
          s_rr += (double)rn[v] * (double)rn[v];
          s_ra += ri * (double)rn[v] * (double)rn[v];
        } else {
          const double rv = (double)R[e];
          const T pn = (T)fma(beta, (double)P[e], rv);
          const double qd = (double)qv[v] * inv + ri * (double)pn;
          const T zn = (T)((double)Z[e] + alpha * (double)pn);
          rn[v] = (T)(rv - alpha * qd);
          Z[e] = zn;
          R[e] = rn[v];
          P[e] = pn;
          const double rr = (double)rn[v], pp = (double)pn;
          s_rr += rr * rr;
          s_ra += ri * rr * rr;
          s_rb += ri * rr * pp;
          s_rc += ri * pp * pp;
        }
      }
      // S^T r' over these 16 rows: k-step v takes the rows frag_row(lk, v), whose
      // r' this lane already holds for column lr
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T* srow = S + (size_t)(rb + frag_row<T>(lk, v)) * NP + lr;
#pragma unroll
        for (int x = 0; x < NB; ++x) acc[x] = mfma4(srow[16 * x], rn[v], acc[x]);
      }
    }
#pragma unroll
    for (int x = 0; x < NB; ++x)
#pragma unroll
      for (int v = 0; v < 4; ++v) gp[wv][(16 * x + frag_row<T>(lk, v)) * 16 + lr] = acc[x][v];
    s_rr = lane_col_sum(s_rr);
    s_ra = lane_col_sum(s_ra);
    s_rb = lane_col_sum(s_rb);
    s_rc = lane_col_sum(s_rc);
    if (lane < 16) {
      cr[wv][0][lane] = s_rr;
      cr[wv][1][lane] = s_ra;
      cr[wv][2][lane] = s_rb;
      cr[wv][3][lane] = s_rc;
    }
  };

  // After a pass: per column the stop test and beta (16 threads), then
  // g = S^T r' + beta g (all threads), then alpha from |g|^2 (wave 0).
  // Returns whether any column of the block is still running.
  auto decide = [&](bool init) -> bool {
    __syncthreads();
    if (tid < 16) {
      const int c = tid;
      double sum[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double t = 0.0;
        for (int w = 0; w < kKtWaves; ++w) t += cr[w][u][c];
        sum[u] = t;
      }
      const double rho = sum[0];
      if (init) {
        const double thr = tol * sqrt(rho);
        const bool live = cb * 16 + c < n;
        const bool act = live && rho > 0.0 && sqrt(rho) > thr && maxit > 0;
        s_thr[c] = thr;
        s_it[c] = 0;
        s_act[c] = act;
        s_beta[c] = 0.0;
        s_st[c] = act ? COL_RUNNING
                      : (!isfinite(rho) ? COL_NONFINITE
                                        : (rho == 0.0 || sqrt(rho) <= thr) ? COL_CONVERGED
                                                                            : COL_MAXIT);
      } else if (s_act[c]) {
        const int it = ++s_it[c];
        const double a = s_alpha[c];
        // alpha_k |r_k|^2 = |e_k|_Psi^2 - |e_{k+1}|_Psi^2 (Hestenes-Stiefel)
        if (hist) hist[(size_t)(it - 1) * n + cb * 16 + c] = a * s_rho[c];
        int st = COL_RUNNING;
        if (!isfinite(a) || !isfinite(rho))
          st = COL_NONFINITE;
        else if (rho == 0.0 || sqrt(rho) <= s_thr[c])
          st = COL_CONVERGED;
        else if (it >= maxit)
          st = COL_MAXIT;
        s_beta[c] = st == COL_RUNNING ? rho / s_rho[c] : 0.0;
        s_st[c] = st;
        s_act[c] = st == COL_RUNNING;
      } else {
        s_beta[c] = 0.0;
      }
      s_rho[c] = rho;
      s_a[c] = sum[1];
      s_b[c] = sum[2];
      s_c[c] = sum[3];
    }
    const bool any = __syncthreads_or(tid < 16 && s_act[tid]);
    for (int e = tid; e < NP * 16; e += kKtBlock) {
      double t = (double)gp[0][e];
#pragma unroll
      for (int w = 1; w < kKtWaves; ++w) t += (double)gp[w][e];
      gd[e] = t + s_beta[e & 15] * gd[e];
    }
    __syncthreads();
    if (wv == 0) {
      // |g_c|^2 over four quarters of j, one per lane group
      const int c = lane & 15, qq = lane >> 4;
      double gg = 0.0;
      for (int j = qq * (NP / 4); j < (qq + 1) * (NP / 4); ++j) gg += gd[j * 16 + c] * gd[j * 16 + c];
      gg = lane_col_sum(gg);
      if (lane < 16) {
        const double bt = s_beta[c];
        const double pap = gg * inv + s_a[c] + 2.0 * bt * s_b[c] + bt * bt * s_c[c];
        s_alpha[c] = s_act[c] ? s_rho[c] / pap : 0.0;
      }
    }
    __syncthreads();
    return any;
  };

  // ---- b = S (A_rows/(N-1))^T: g = the block's 16 anomaly rows, transposed ----
  for (int e = tid; e < NP * 16; e += kKtBlock) {
    const int c = e / NP, j = e - c * NP;
    gd[j * 16 + c] = (double)A[(size_t)(cb * 16 + c) * NP + j];
  }
  if (tid < 16) {
    s_alpha[tid] = 0.0;
    s_beta[tid] = 0.0;
  }
  __syncthreads();
  pass(true);
  bool any = decide(true);
  while (any) {
    pass(false);
    any = decide(false);
  }

  // ---- results: iterations, status, K^T, and this block's rows of X_a ----
  if (tid < 16 && cb * 16 + tid < n) {
    if (iters) iters[cb * 16 + tid] = s_it[tid];
    status[cb * 16 + tid] = s_st[tid];
  }
  if (kt) {
    for (int e = tid; e < m * 16; e += kKtBlock) {
      const int row = e >> 4, c = e & 15;
      if (cb * 16 + c < n) kt[(size_t)row * n + cb * 16 + c] = Z[e];
    }
  }
  // X_a rows cb*16 + c: X_f + sum_i K^T[i][c] D[i][:] (A operand z^T, B operand D)
  V acc[NB];
#pragma unroll
  for (int x = 0; x < NB; ++x) acc[x] = V{0, 0, 0, 0};
  for (int r4 = r0; r4 < r0 + rows; r4 += 4) {
    const int row = r4 + lk;
    const T zv = Z[(size_t)row * 16 + lr];
#pragma unroll
    for (int x = 0; x < NB; ++x) acc[x] = mfma4(zv, D[(size_t)row * NP + 16 * x + lr], acc[x]);
  }
#pragma unroll
  for (int x = 0; x < NB; ++x)
#pragma unroll
    for (int v = 0; v < 4; ++v) gp[wv][frag_row<T>(lk, v) * NP + 16 * x + lr] = acc[x][v];
  __syncthreads();
  for (int e = tid; e < 16 * NP; e += kKtBlock) {
    const int c = e / NP, j = e - c * NP, i = cb * 16 + c;
    if (i >= n || j >= N) continue;
    double s = (double)gp[0][e];
#pragma unroll
    for (int w = 1; w < kKtWaves; ++w) s += (double)gp[w][e];
    Xa[(size_t)i * N + j] = (T)((double)Xf[(size_t)i * N + j] + s);
  }
}

template <typename T>
constexpr size_t kt_lds(int NP) {
  return sizeof(T) * (size_t)kKtWaves * NP * 16 + sizeof(double) * (size_t)NP * 16;
}

template <typename T, int NP>
hipError_t launch_kt_np(int n, int m, int N, int k, const T* Xf, T* Xa, const int32_t* idx,
                        const T* hw, const T* y, const T* rdiag, const T* eps, double tol,
                        int maxit, T* kt, int* iters, double* hist, const KtLayout& L,
                        void* ws, hipStream_t s) {
  unsigned char* b = (unsigned char*)ws;
  T* S = (T*)(b + L.S);
  T* Dm = (T*)(b + L.D);
  T* rd = (T*)(b + L.rd);
  T* A = (T*)(b + L.A);
  int* err = (int*)(b + L.err);
  hipError_t e = launch_zero_u32((unsigned*)err, 1, s);
  if (e != hipSuccess) return e;
  constexpr int RPB = kBlock / (NP / 4);
  const int blocks = L.mp / RPB + (L.nn + RPB - 1) / RPB;
  hipLaunchKernelGGL((k_kt_rows<T, NP>), dim3(blocks), dim3(kBlock), 0, s, n, m, N, k, L.mp,
                     L.nn, Xf, idx, hw, y, rdiag, eps, S, Dm, rd, A, err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const void* fn = (const void*)k_kt_cg<T, NP>;
  if ((e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kt_lds<T>(NP))) != hipSuccess)
    return e;
  hipLaunchKernelGGL((k_kt_cg<T, NP>), dim3(L.nn / 16), dim3(kKtBlock), kt_lds<T>(NP), s, n, m,
                     L.mp, N,
                     (const T*)S, (const T*)Dm, (const T*)rd, (const T*)A, Xf, Xa,
                     (T*)(b + L.Z), (T*)(b + L.R), (T*)(b + L.P), kt, tol, maxit, iters, hist,
                     (int*)(b + L.status));
  return hipGetLastError();
}

}  // namespace

KtLayout kt_layout(int n, int m, int N, int prec) {
  KtLayout L{};
  if (n < 1 || m < 1 || N < 2 || N > 128) return L;
  if (prec != CGD_FP64 && prec != CGD_FP32) return L;
  const size_t esz = prec == CGD_FP64 ? 8 : 4;
  L.NP = kt_np(N);
  L.mp = kt_mp(m);
  L.nn = kt_nn(n);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (bytes + 255) & ~size_t(255);
    return at;
  };
  L.S = take(esz * L.mp * L.NP);
  L.D = take(esz * L.mp * L.NP);
  L.rd = take(esz * L.mp);
  L.A = take(esz * L.nn * L.NP);
  L.Z = take(esz * L.nn * L.mp);
  L.R = take(esz * L.nn * L.mp);
  L.P = take(esz * L.nn * L.mp);
  L.status = take(sizeof(int) * L.nn);
  L.iters = take(sizeof(int) * L.nn);
  L.err = take(sizeof(int) * 4);
  L.total = o;
  return L;
}

template <typename T>
hipError_t launch_kt(int n, int m, int N, int k, const T* Xf, T* Xa, const int32_t* idx,
                     const T* hw, const T* y, const T* rdiag, const T* eps, double tol, int maxit,
                     T* kt, int* iters, double* hist, const KtLayout& L, void* ws,
                     hipStream_t s) {
  switch (L.NP) {
    case 16:
      return launch_kt_np<T, 16>(n, m, N, k, Xf, Xa, idx, hw, y, rdiag, eps, tol, maxit, kt,
                                 iters, hist, L, ws, s);
    case 32:
      return launch_kt_np<T, 32>(n, m, N, k, Xf, Xa, idx, hw, y, rdiag, eps, tol, maxit, kt,
                                 iters, hist, L, ws, s);
    case 64:
      return launch_kt_np<T, 64>(n, m, N, k, Xf, Xa, idx, hw, y, rdiag, eps, tol, maxit, kt,
                                 iters, hist, L, ws, s);
    case 128:
      return launch_kt_np<T, 128>(n, m, N, k, Xf, Xa, idx, hw, y, rdiag, eps, tol, maxit, kt,
                                  iters, hist, L, ws, s);
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_kt<double>(int, int, int, int, const double*, double*, const int32_t*,
                                      const double*, const double*, const double*,
                                      const double*, double, int, double*, int*, double*,
                                      const KtLayout&, void*, hipStream_t);
template hipError_t launch_kt<float>(int, int, int, int, const float*, float*, const int32_t*,
                                     const float*, const float*, const float*, const float*,
                                     double, int, float*, int*, double*, const KtLayout&, void*,
                                     hipStream_t);

}  // namespace cgd
