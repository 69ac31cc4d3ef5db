// Ensemble update, CGD-EnKF-Reduced and input validation kernels (gfx950).
#include "modes.h"
#include "mfma_util.h"
#include "update_tile.h"

namespace cgd {

namespace {

// X_a = X_f + A W  (mode 0, Algorithm 1 with W = S^T Z/(N-1), A = X_f - xbar 1^T)
// X_a = X_f W      (mode 1, Algorithm 2)
// Each workgroup owns RBX whole rows: it stages them in LDS before writing,
// so X_a may alias X_f.  With `skip`, nothing is written when bit 2 of *skip
// is set (the solver's start-up census gave up: W was never formed).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(int n, int N, int RBX, const T* Xf, T* Xa,
                                                   const double* Wd, int mode, const int* skip) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (skip && (*skip & 4)) return;
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

// The same update on the 16x16x4 MFMA for N <= 128 (FP32) or N <= 64 (FP64),
// 64-row tiles (see update_tile.h): each workgroup brings W into LDS once
// and then takes every gridDim.x-th tile.
template <typename T, int NP>
__global__ __launch_bounds__(kBlock) void k_update_mfma(int n, int N, const T* Xf, T* Xa,
                                                        const double* Wd, int mode,
                                                        const int* skip) {
  using C = UCfg<T, NP>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (skip && (*skip & 4)) return;
  T* Wt = (T*)smem_raw;
  T* As = Wt + (size_t)NP * C::LD;
  T* Xr = As + (size_t)C::RBX * C::LD;
  double* mean = (double*)(Xr + (size_t)C::RBX * C::LD);
  update_load_w<T, NP, kBlock>(N, Wd, mode, Wt);
  update_tiles_stream<T, NP, kBlock, C::RBX>(n, N, Xf, Xa, mode, As, mode == 0 ? Xr : As, Wt, mean);
}

// The same update with the A' operand read from global memory straight into
// the MFMA's registers: no tile of X_f passes through LDS and no barrier is
// taken per tile.  W'^T sits in LDS (from Wd as update_load_w forms it, or, WT,
// already transposed in T as k_red_update takes it).  Each wave takes 16-row
// blocks in turn over the whole grid (workgroups first, then their waves); lane (lr, lk) holds row lr's columns
// lk NP/4 .. lk NP/4 + NP/4 - 1 (16-byte loads: N a multiple of 16/sizeof(T),
// X_f and X_a 16-byte aligned), the permutation of the summation index the B
// operand uses too.  Mode 0 centres each row with its mean (the lane's part
// plus two shuffles across the row's four lanes).  X_f is read again for the
// output elements before the block's stores, so X_a may alias X_f.
constexpr int kUpdWaves = 8;

template <typename T, int NP, bool WT>
__global__ __launch_bounds__(64 * kUpdWaves) void k_update_rows(int n, int N, const T* Xf, T* Xa,
                                                               const double* Wd, const T* Wtg,
                                                               int mode, const int* skip) {
  using U = UCfg<T, NP>;
  using V = typename Vec4<T>::type;
  constexpr int KQ = NP / 4, TJ = NP / 16, VU = 16 / (int)sizeof(T), BS = 64 * kUpdWaves;
  constexpr int CH = KQ < 8 ? KQ : 8;  // B operand loads in chunks (register pressure)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (skip && (*skip & 4)) return;
  T* Wt = (T*)smem_raw;  // NP x LD
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15, lk = lane >> 4;
  if constexpr (WT) {
    for (int e = tid; e < NP * NP / VU; e += BS) {
      const int row = e / (NP / VU), c = (e - row * (NP / VU)) * VU;
      T v[VU];
      vload<VU>(Wtg + (size_t)row * NP + c, v);
#pragma unroll
      for (int u = 0; u < VU; ++u) Wt[row * U::LD + c + u] = v[u];
    }
  } else {
    update_load_w<T, NP, BS>(N, Wd, mode, Wt);
  }
  __syncthreads();
  // blocks go round the workgroups first, then their waves, so that a small n
  // still spreads over the whole grid
  const int nb = (n + 15) / 16, step = gridDim.x * kUpdWaves;
  for (int b = blockIdx.x + gridDim.x * wv; b < nb; b += step) {
    const int i0 = b * 16, row = i0 + lr;
    // A' operand: this lane's quarter of row lr, zero past N and past n
    T av[KQ];
#pragma unroll
    for (int c = 0; c < KQ; c += VU) {
      const int col = lk * KQ + c;
      if (row < n && col < N) {
        vload<VU>(Xf + (size_t)row * N + col, *reinterpret_cast<T(*)[VU]>(&av[c]));
      } else {
#pragma unroll
        for (int u = 0; u < VU; ++u) av[c + u] = (T)0;
      }
    }
    if (mode == 0) {
      double sum = 0.0;
#pragma unroll
      for (int t = 0; t < KQ; ++t) sum += (double)av[t];
      sum += __shfl_xor(sum, 16);
      sum += __shfl_xor(sum, 32);
      const double mu = sum / N;
#pragma unroll
      for (int t = 0; t < KQ; ++t)
        av[t] = lk * KQ + t < N ? (T)((double)av[t] - mu) : (T)0;
    }
    // every X_f element of the block's rows is in registers (av) or read below
    // before this wave stores any of them
#pragma unroll 2
    for (int tj = 0; tj < TJ; ++tj) {
      // X_f at this lane's output elements of the tile (rows frag_row(lk, i),
      // column lr), requested before the tile's products
      T xo[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = i0 + frag_row<T>(lk, i), col = tj * 16 + lr;
        xo[i] = (r < n && col < N) ? Xf[(size_t)r * N + col] : (T)0;
      }
      V acc = {0, 0, 0, 0};
      const T* wrow = Wt + (tj * 16 + lr) * U::LD + lk * KQ;
#pragma unroll
      for (int t0 = 0; t0 < KQ; t0 += CH) {
        T bv[CH];
        vload<CH>(wrow + t0, bv);
#pragma unroll
        for (int t = 0; t < CH; ++t) acc = mfma4(av[t0 + t], bv[t], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = i0 + frag_row<T>(lk, i), col = tj * 16 + lr;
        if (r < n && col < N) Xa[(size_t)r * N + col] = (T)((double)xo[i] + (double)acc[i]);
      }
    }
  }
}

// Whether k_update_rows applies and pays: N a multiple of the 16-byte vector,
// both arrays 16-byte aligned, and enough 16-row blocks that a full grid of
// 8-wave workgroups gives every wave one (n >= 32768 on 256 CUs).  Below that
// the LDS-tiled updates, which share a tile among four waves, measured
// faster (twin workload, n = 4096: 25985 against about 28000 reduced analyses/s).
constexpr int kUpdRowsMinN = 16 * kUpdWaves * 256;
template <typename T>
bool update_rows_ok(int n, int N, const T* Xf, const T* Xa) {
  return n >= kUpdRowsMinN && N % (16 / (int)sizeof(T)) == 0 && ((uintptr_t)Xf & 15) == 0 &&
         ((uintptr_t)Xa & 15) == 0;
}

template <typename T, int NP, bool WT>
hipError_t launch_update_rows(int n, int N, const T* Xf, T* Xa, const double* Wd, const T* Wt,
                              int mode, const int* skip, hipStream_t s) {
  using U = UCfg<T, NP>;
  constexpr size_t lds = sizeof(T) * (size_t)NP * U::LD;
  const void* fn = (const void*)k_update_rows<T, NP, WT>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  // as many workgroups as run at once (each loads W' once), at most one per block
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
      return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_update_rows<T, NP, WT>,
                                                          64 * kUpdWaves, lds)) != hipSuccess)
      return e;
    resident = per * cus > 0 ? per * cus : 1;
  }
  const int nb = (n + 15) / 16;
  const int grid = nb < resident ? nb : resident;
  hipLaunchKernelGGL((k_update_rows<T, NP, WT>), dim3(grid), dim3(64 * kUpdWaves), lds, s, n, N,
                     Xf, Xa, Wd, Wt, mode, skip);
  return hipGetLastError();
}

template <typename T, int NP>
hipError_t launch_update_mfma(int n, int N, const T* Xf, T* Xa, const double* Wd, int mode,
                              const int* skip, hipStream_t s) {
  using C = UCfg<T, NP>;
  const void* fn = (const void*)k_update_mfma<T, NP>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::lds_xr);
  if (e != hipSuccess) return e;
  // as many workgroups as run at once (each loads W once), at most one per tile
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
      return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_update_mfma<T, NP>, kBlock,
                                                          C::lds_xr)) != hipSuccess)
      return e;
    resident = per * cus > 0 ? per * cus : 1;
  }
  const int tiles = (n + C::RBX - 1) / C::RBX;
  const int grid = tiles < resident ? tiles : resident;
  hipLaunchKernelGGL((k_update_mfma<T, NP>), dim3(grid), dim3(kBlock), C::lds_xr, s, n, N, Xf,
                     Xa, Wd, mode, skip);
  return hipGetLastError();
}

// Reduced mode, step 1 (Algorithm 2 setup, Table 2 "N x N matrix form"):
// per row block, HX, zbar, P = (HX - zbar 1^T)/l_i and Yt = ((y - zbar) 1^T + E)/l_i
// with l_i = sqrt((N-1) r_i); partial [P^T P | P^T Yt] (N x 2N) per workgroup.
// SEN (the sEnKF of Appendix A, Algorithm 3): l_i^2 = ||s_i||^2 + (N-1) r_i,
// the i-th diagonal entry of Zhat Zhat^T + (N-1) R, and Yt = (Y - HX)/l_i, so
// that the right half is Zhat^T diag(Zhat Zhat^T + (N-1) R)^{-1} (Y - Z); the
// left half is not formed.
template <typename T, bool SEN>
__global__ __launch_bounds__(kBlock) void k_red_gram(int n, int m, int N, int k, int RB, int nblk,
                                                     const T* Xf, const int32_t* idx,
                                                     const T* hw, const T* y, const T* rdiag,
                                                     const T* eps, double* part, int* err) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lp = (double*)smem_raw;           // RB * N
  double* ly = lp + (size_t)RB * N;         // RB * N
  double* lz = ly + (size_t)RB * N;         // RB: zbar_i
  double* ll = lz + RB;                     // RB: l_i
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
      const double zb = s / N;
      double l2 = (double)(N - 1) * (double)rdiag[i0 + i];
      if constexpr (SEN) {
        double ss = 0;
        for (int j = 0; j < N; ++j) ss += (lp[i * N + j] - zb) * (lp[i * N + j] - zb);
        l2 += ss;
      }
      lz[i] = zb;
      ll[i] = sqrt(l2);
    }
    __syncthreads();
    for (int e = tid; e < ne; e += kBlock) {
      const int i = e / N, gi = i0 + i;
      const double l = ll[i];
      const double zb = lz[i];
      double yt = (double)y[gi] - (SEN ? lp[e] : zb);
      if (eps) yt += (double)eps[(size_t)i0 * N + e];
      lp[e] = (lp[e] - zb) / l;
      ly[e] = yt / l;
    }
    __syncthreads();
    for (int o = tid + (SEN ? N * N : 0); o < 2 * N * N; o += kBlock) {
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
// o0 = N * N forms B only; dadd is the diagonal added (1, or 0 for the sEnKF).
__global__ __launch_bounds__(kBlock) void k_red_sum(int N, int nwg, const double* part, double* G,
                                                    double* B, int o0, double dadd) {
  const int o = o0 + blockIdx.x * kBlock + threadIdx.x;
  if (o >= 2 * N * N) return;
  double acc = 0;
  for (int w = 0; w < nwg; ++w) acc += part[(size_t)w * 2 * N * N + o];
  const int half = o / (N * N), oo = o - half * N * N;
  const int kk = oo / N, j = oo - kk * N;
  acc += (kk == j) ? dadd : 0.0;
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

// Final status of one column of the N x N CG: a non-finite coefficient or
// residual, else converged when the residual test holds (also on the last
// allowed step, and for b_j = 0), else stopped at maxit.
__device__ inline int small_cg_status(bool nonfinite, double rho, double thr) {
  if (nonfinite || !isfinite(rho)) return COL_NONFINITE;
  if (rho == 0.0 || sqrt(rho) <= thr) return COL_CONVERGED;
  return COL_MAXIT;
}

// CGD-EnKF-Reduced solve: one workgroup per column j of B runs textbook CG
// on the N x N SPD system G w = b_j from w = 0 (Lemma 1: at most N steps in
// exact arithmetic).  Vectors live in LDS; G is read from L2 (symmetric, so
// q_k = sum_l G[l][k] p_l reads rows coalesced).
__global__ __launch_bounds__(kBlock) void k_small_cg(int N, const double* G, const double* B,
                                                     double* W, int* iters, int* status,
                                                     double tol, int maxit) {
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
  bool nonfinite = false;
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
    if (!isfinite(alpha) || !isfinite(beta)) {
      nonfinite = true;
      break;
    }
  }
  for (int kk = tid; kk < N; kk += kBlock) W[(size_t)kk * N + j] = x[kk];
  if (tid == 0) {
    iters[j] = it;
    status[j] = small_cg_status(nonfinite, rho, thr);
  }
}

// ---------------------------------------------------------------------------
// Reduced mode on the MFMA, N <= 128 (Algorithm 2 with the formation costs of
// Table 2).  NP is N rounded up to 32, 64 or 128; Q is mpad x 2 NP (mpad = m
// rounded up to 32), row i = [P_i | Yt_i] with
//   P_i  = (HX_i - zbar_i 1^T) / l_i,  Yt_i = (y_i - zbar_i + E_i) / l_i,
//   l_i  = sqrt((N-1) r_i),  zbar_i = HX_i 1 / N,
// zero in the padding columns and rows.  [P^T P | P^T Yt] = Q[:, :NP]^T Q is
// a tall-skinny product over the m rows, summed in parts over row chunks
// that a later launch adds in a fixed order, with the identity.  For NP <= 64
// one launch builds each chunk of Q in LDS and multiplies it there
// (k_red_pg); for NP = 128 Q goes through memory: k_red_prep writes it, and
// each k_red_gemm workgroup takes one chunk of KC rows and one TS x TS output
// tile (the upper tiles of the symmetric left half, every tile of the right
// half).
// ---------------------------------------------------------------------------

template <int NP> struct RedCfg {
  static constexpr int QW = 2 * NP;
  static constexpr int TS = NP >= 64 ? 64 : 32;   // output tile
  static constexpr int MB = TS / 32;              // 16x16 MFMA blocks per wave and direction
  static constexpr int TT = NP / TS;              // tiles across the left half
  static constexpr int NTG = TT * (TT + 1) / 2;   // upper tiles of the left half
  static constexpr int NTILE = NTG + TT * TT;
  static constexpr int LPR = NP / 4;              // prep: lanes per row, 4 columns each
  static constexpr int RPB = kBlock / LPR;        // prep: rows per workgroup
};

// Row i of Q from X_f, idx, w, y, r and E (one group of NP/4 lanes per row).
// Every workgroup writes its error word errw[blockIdx.x] (2: an index out of
// range, else 0), so no word needs clearing beforehand.  The grid is
// mpad / RPB workgroups.  SEN: the sEnKF's row scaling (see k_red_gram).
template <typename T, int NP, bool SEN>
__global__ __launch_bounds__(kBlock) void k_red_prep(int n, int m, int N, int k, const T* Xf,
                                                     const int32_t* idx, const T* hw, const T* y,
                                                     const T* rdiag, const T* eps, T* Q,
                                                     int* errw) {
  using C = RedCfg<NP>;
  __shared__ int bad;
  const int tid = threadIdx.x, q = tid % C::LPR;
  const int i = blockIdx.x * C::RPB + tid / C::LPR;
  const bool live = i < m;
  if (tid == 0) bad = 0;
  __syncthreads();
  // the row's own inputs load alongside the gather
  double yv = 0.0, rv = 1.0, ev[4] = {0.0, 0.0, 0.0, 0.0};
  if (live) {
    yv = (double)y[i];
    rv = (double)rdiag[i];
    if (eps) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * q + u < N) ev[u] = (double)eps[(size_t)i * N + 4 * q + u];
    }
  }
  // the entries of the operator row four at a time: their indices and weights
  // first, then every X_f load (an index out of range reads row 0 with weight
  // 0), summed in the order of t
  double h[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t0 = 0; t0 < k; t0 += 4) {
    int c[4];
    double wt[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int t = t0 + v;
      c[v] = 0;
      wt[v] = 0.0;
      if (live && t < k) {
        const int cx = idx[(size_t)i * k + t];
        if ((unsigned)cx < (unsigned)n) {
          c[v] = cx;
          wt[v] = (double)hw[(size_t)i * k + t];
        } else if (q == 0) {
          atomicOr(&bad, 2);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T* xr = Xf + (size_t)c[v] * N;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * q + u < N) h[u] += wt[v] * (double)xr[4 * q + u];
    }
  }
  // every lane takes part in the group sum; rows past m carry zeros
  const double zb = group_sum<C::LPR>((h[0] + h[1]) + (h[2] + h[3])) / N;
  __syncthreads();
  if (tid == 0) errw[blockIdx.x] = bad;
  double l2 = (double)(N - 1) * rv;
  if constexpr (SEN) {
    double ss = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (4 * q + u < N) ss += (h[u] - zb) * (h[u] - zb);
    l2 += group_sum<C::LPR>(ss);
  }
  const double l = sqrt(l2), yz = yv - zb;
  T* qr = Q + (size_t)i * C::QW;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = 4 * q + u;
    double pm = 0.0, yt = 0.0;
    if (live && j < N) {
      pm = (h[u] - zb) / l;
      yt = (yz + ev[u] - (SEN ? h[u] - zb : 0.0)) / l;
    }
    qr[j] = (T)pm;
    qr[NP + j] = (T)yt;
  }
}

// Gather and product in one launch for NP <= 64.  Workgroup s builds rows
// s KC .. s KC + KC - 1 of Q in LDS (zero past m), stored by column (a run of
// KC rows per column, padded to spread the banks), then forms its part of
// Q[:, :NP]^T Q on the MFMA: each wave a quarter of the NP x 2NP output, the
// summation over the chunk's rows split into four runs of KC/4, one per lane
// group (the same bijection for both operands).  errw[s] as in k_red_prep.
// SEN: the sEnKF's row scaling, and only the right half Q[:, :NP]^T Q[:, NP:]
// (each wave a quarter of it).
constexpr int kRedFusedRows = 32;  // KC of the fused launch

template <typename T, int NP, bool SEN>
__global__ __launch_bounds__(kBlock) void k_red_pg(int n, int m, int N, int k, const T* Xf,
                                                   const int32_t* idx, const T* hw, const T* y,
                                                   const T* rdiag, const T* eps, T* part,
                                                   int* errw) {
  using C = RedCfg<NP>;
  using V = typename Vec4<T>::type;
  constexpr int KC = kRedFusedRows, KQ = KC / 4, LQ = KC + 16 / (int)sizeof(T);
  constexpr int PASS = KC / C::RPB;                 // rows per thread
  constexpr int MA = NP / 32, MB = SEN ? NP / 32 : NP / 16;  // 16x16 blocks per wave (a, b)
  static_assert(PASS * C::RPB == KC && KQ % 4 == 0, "chunk shape");
  __shared__ __align__(16) T qt[2 * NP * LQ];
  __shared__ int bad;
  const int tid = threadIdx.x, q = tid % C::LPR, rw = tid / C::LPR;
  const int r0 = blockIdx.x * KC;
  if (tid == 0) bad = 0;
  __syncthreads();
  // ---- Q rows of the chunk: every load of the thread's rows first ----
  double yv[PASS], rv[PASS], ev[PASS][4], h[PASS][4];
#pragma unroll
  for (int u = 0; u < PASS; ++u) {
    const int i = r0 + u * C::RPB + rw;
    const bool live = i < m;
    yv[u] = live ? (double)y[i] : 0.0;
    rv[u] = live ? (double)rdiag[i] : 1.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      h[u][c] = 0.0;
      ev[u][c] = (live && eps && 4 * q + c < N) ? (double)eps[(size_t)i * N + 4 * q + c] : 0.0;
    }
  }
  for (int t = 0; t < k; ++t) {
    int col[PASS];
    double wt[PASS];
#pragma unroll
    for (int u = 0; u < PASS; ++u) {
      const int i = r0 + u * C::RPB + rw;
      col[u] = 0;
      wt[u] = 0.0;
      if (i < m) {
        const int cx = idx[(size_t)i * k + t];
        if ((unsigned)cx < (unsigned)n) {
          col[u] = cx;
          wt[u] = (double)hw[(size_t)i * k + t];
        } else if (q == 0) {
          atomicOr(&bad, 2);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < PASS; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (4 * q + c < N) h[u][c] += wt[u] * (double)Xf[(size_t)col[u] * N + 4 * q + c];
  }
#pragma unroll
  for (int u = 0; u < PASS; ++u) {
    const int i = r0 + u * C::RPB + rw, rr = u * C::RPB + rw;
    const bool live = i < m;
    const double zb = group_sum<C::LPR>((h[u][0] + h[u][1]) + (h[u][2] + h[u][3])) / N;
    double l2 = (double)(N - 1) * rv[u];
    if constexpr (SEN) {
      double ss = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (4 * q + c < N) ss += (h[u][c] - zb) * (h[u][c] - zb);
      l2 += group_sum<C::LPR>(ss);
    }
    const double l = sqrt(l2), yz = yv[u] - zb;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = 4 * q + c;
      double pm = 0.0, yt = 0.0;
      if (live && j < N) {
        pm = (h[u][c] - zb) / l;
        yt = (yz + ev[u][c] - (SEN ? h[u][c] - zb : 0.0)) / l;
      }
      qt[j * LQ + rr] = (T)pm;
      qt[(NP + j) * LQ + rr] = (T)yt;
    }
  }
  __syncthreads();
  if (tid == 0) errw[blockIdx.x] = bad;
  // ---- the chunk's part of the product ----
  const int lane = tid & 63, wv = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int a0 = (wv >> 1) * (NP / 2), b0 = SEN ? NP + (wv & 1) * (NP / 2) : (wv & 1) * NP;
  T av[MA][KQ], bv[MB][KQ];
#pragma unroll
  for (int x = 0; x < MA; ++x) vload<KQ>(qt + (a0 + 16 * x + lr) * LQ + lk * KQ, av[x]);
#pragma unroll
  for (int z = 0; z < MB; ++z) vload<KQ>(qt + (b0 + 16 * z + lr) * LQ + lk * KQ, bv[z]);
  V acc[MA][MB];
#pragma unroll
  for (int x = 0; x < MA; ++x)
#pragma unroll
    for (int z = 0; z < MB; ++z) acc[x][z] = V{0, 0, 0, 0};
#pragma unroll
  for (int u = 0; u < KQ; ++u)
#pragma unroll
    for (int x = 0; x < MA; ++x)
#pragma unroll
      for (int z = 0; z < MB; ++z) acc[x][z] = mfma4(av[x][u], bv[z][u], acc[x][z]);
  T* out = part + (size_t)blockIdx.x * NP * C::QW;
#pragma unroll
  for (int x = 0; x < MA; ++x)
#pragma unroll
    for (int z = 0; z < MB; ++z)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out[(size_t)(a0 + 16 * x + frag_row<T>(lk, i)) * C::QW + b0 + 16 * z + lr] = acc[x][z][i];
}

// part[s] (NP x 2NP, tile entries only) = Q[rows of chunk s, :NP]^T Q[rows of chunk s, :].
// Grid (NTILE - t0, S), tile t0 + blockIdx.x (t0 = NTG: the right half only); four waves per tile, each a (TS/2) x (TS/2) quarter of
// MB x MB MFMA blocks.  The next 32 rows load while the current ones multiply.
template <typename T, int NP>
__global__ __launch_bounds__(kBlock) void k_red_gemm(int KC, int mpad, int t0, const T* Q,
                                                     T* part) {
  using C = RedCfg<NP>;
  using V = typename Vec4<T>::type;
  constexpr int MB = C::MB, HS = C::TS / 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
  int t = blockIdx.x + t0, ta = 0, tb;
  if (t < C::NTG) {
    while (t >= C::TT - ta) t -= C::TT - ta++;
    tb = ta + t;
  } else {
    t -= C::NTG;
    ta = t / C::TT;
    tb = C::TT + t % C::TT;
  }
  const int ca = ta * C::TS + (wv >> 1) * HS + lr, cb = tb * C::TS + (wv & 1) * HS + lr;
  const int r0 = blockIdx.y * KC, r1 = min(mpad, r0 + KC);
  V acc[MB][MB];
#pragma unroll
  for (int x = 0; x < MB; ++x)
#pragma unroll
    for (int z = 0; z < MB; ++z) acc[x][z] = V{0, 0, 0, 0};
  T an[8][MB], bn[8][MB];
  auto load = [&](int r) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const T* row = Q + (size_t)(r + 4 * u + lk) * C::QW;
#pragma unroll
      for (int x = 0; x < MB; ++x) {
        an[u][x] = row[ca + 16 * x];
        bn[u][x] = row[cb + 16 * x];
      }
    }
  };
  load(r0);
  for (int r = r0; r < r1; r += 32) {
    T ac[8][MB], bc[8][MB];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int x = 0; x < MB; ++x) {
        ac[u][x] = an[u][x];
        bc[u][x] = bn[u][x];
      }
    if (r + 32 < r1) load(r + 32);
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int x = 0; x < MB; ++x)
#pragma unroll
        for (int z = 0; z < MB; ++z) acc[x][z] = mfma4(ac[u][x], bc[u][z], acc[x][z]);
  }
  T* out = part + (size_t)blockIdx.y * NP * C::QW;
#pragma unroll
  for (int x = 0; x < MB; ++x)
#pragma unroll
    for (int z = 0; z < MB; ++z)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out[(size_t)(ca - lr + 16 * x + frag_row<T>(lk, i)) * C::QW + cb + 16 * z] = acc[x][z][i];
}

// G = I + sum_s part_s[:, :NP] and B = I + sum_s part_s[:, NP:], restricted
// to N x N (I scaled by dadd: 0 for the sEnKF, which passes NR = 0 and so
// forms B only); a left-half entry below the diagonal tiles is read from its
// mirror.  Eight lanes share an output: lane q adds the parts q, q + 8, ...
// in order, then a fixed lane tree adds the eight.  G is written as the
// solve keeps it in LDS: NR rows of stride LG, zero outside N x N; B is
// N x N.  Workgroup 0 also folds the gather's error
// words into err.
template <typename T, int NP>
__global__ __launch_bounds__(kBlock) void k_red_sum2(int N, int NR, int LG, int S,
                                                     const T* part, double* Gp, double* B,
                                                     const int* errw, int nerr, int* err,
                                                     double dadd) {
  using C = RedCfg<NP>;
  const int tid = threadIdx.x, q = tid & 7;
  if (blockIdx.x == 0) {
    __shared__ int flags;
    if (tid == 0) flags = 0;
    __syncthreads();
    int f = 0;
    for (int e = tid; e < nerr; e += kBlock) f |= errw[e];
    if (f) atomicOr(&flags, f);
    __syncthreads();
    if (tid == 0) *err = flags;
  }
  const int o = blockIdx.x * (kBlock / 8) + tid / 8, ng = NR * LG, total = ng + N * N;
  const bool right = o >= ng;
  int a = 0, b = 0;
  bool live = o < total;
  if (live) {
    if (!right) {
      a = o / LG;
      b = o - a * LG;
      live = a < N && b < N;
    } else {
      a = (o - ng) / N;
      b = (o - ng) - a * N;
    }
  }
  double acc = 0.0;
  if (live) {
    const bool mirror = !right && a / C::TS > b / C::TS;
    const T* src = part + (size_t)(mirror ? b : a) * C::QW + (right ? NP : 0) + (mirror ? a : b);
    const size_t stride = (size_t)NP * C::QW;
#pragma unroll 4
    for (int s = q; s < S; s += 8) acc += (double)src[s * stride];
  }
  acc = group_sum<8>(acc);
  if (q == 0 && o < total) {
    if (live && a == b) acc += dadd;
    if (right)
      B[o - ng] = acc;
    else
      Gp[o] = acc;
  }
}

// sEnKF: Zhat^T diag(...)^{-1} (Y - Z) = sum_s part_s[:, NP:] restricted to
// N x N, written transposed in the update's element type as k_red_update
// takes W' - I: Wt[b][a] (NP x NP, zero outside N x N).  Eight lanes share an
// output as in k_red_sum2; workgroup 0 folds the gather's error words and
// zeros the N iteration counts (iters0, if given: no CG runs).
template <typename T, int NP>
__global__ __launch_bounds__(kBlock) void k_senkf_sum(int N, int S, const T* part, T* Wt,
                                                      const int* errw, int nerr, int* err,
                                                      int* iters0) {
  using C = RedCfg<NP>;
  const int tid = threadIdx.x, q = tid & 7;
  if (blockIdx.x == 0) {
    if (iters0)
      for (int e = tid; e < N; e += kBlock) iters0[e] = 0;
    __shared__ int flags;
    if (tid == 0) flags = 0;
    __syncthreads();
    int f = 0;
    for (int e = tid; e < nerr; e += kBlock) f |= errw[e];
    if (f) atomicOr(&flags, f);
    __syncthreads();
    if (tid == 0) *err = flags;
  }
  const int o = blockIdx.x * (kBlock / 8) + tid / 8;  // all eight lanes of a group share o
  if (o >= NP * NP) return;
  const int b = o / NP, a = o - b * NP;
  double acc = 0.0;
  if (a < N && b < N) {
    const T* src = part + (size_t)a * C::QW + NP + b;
    const size_t stride = (size_t)NP * C::QW;
#pragma unroll 4
    for (int s = q; s < S; s += 8) acc += (double)src[s * stride];
  }
  acc = group_sum<8>(acc);
  if (q == 0) Wt[o] = (T)acc;
}

// CGD-EnKF-Reduced solve for N <= 64 RPL: textbook CG on G w = b_j from
// w = 0 (Lemma 1: at most N steps in exact arithmetic), one workgroup per
// column.  G comes as the sum launch lays it out (LG = 64 RPL rows of stride
// LG, zero outside N x N); each wave keeps a quarter of its rows in
// registers (reading G from LDS every step cost 0.43 us a step at N = 128).
// Each wave carries the whole recurrence (lane l holds rows l + 64 u of w,
// r, p, q), the same values in every wave, but forms only a quarter of
// q = G p: the rows of G from LG/4 wv on, with its own copy of p in LDS.  The four partial q meet
// in LDS (two buffers, alternate steps) behind one barrier per step and
// every wave adds them in the same order, so all waves take the same
// decisions.  Writes W (FP64, row-major) and Wt = (W - I)^T in the update's
// element type (NP x NP, zero outside N x N); workgroups j >= N only clear
// their row of Wt.
template <typename T, int RPL>
__global__ __launch_bounds__(kBlock) void k_small_cg_w(int N, int NP, const double* Gp,
                                                       const double* B, double* W, T* Wt,
                                                       int* iters, int* iters2, int* status,
                                                       double tol, int maxit) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int LG = 64 * RPL, NW = kBlock / 64, QR = LG / NW;
  static_assert(QR % 16 == 0, "rows per wave");
  double* ps = (double*)smem_raw;             // NW x LG
  double* qp = ps + (size_t)NW * LG;          // 2 x NW x LG
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, j = blockIdx.x;
  if (j >= N) {
    for (int e = tid; e < NP; e += kBlock) Wt[(size_t)j * NP + e] = (T)0;
    return;
  }
  // This wave's QR rows of G (G is symmetric: row l, column i = lane + 64 u),
  // kept in registers for the whole solve (QR x RPL doubles per lane), so
  // that a step reads no G from LDS.
  double gr[QR][RPL];
#pragma unroll
  for (int t = 0; t < QR; ++t)
#pragma unroll
    for (int u = 0; u < RPL; ++u) gr[t][u] = Gp[(size_t)(wv * QR + t) * LG + lane + 64 * u];
  double x[RPL], r[RPL], p[RPL];
  double part = 0.0;
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int i = lane + 64 * u;
    const double b = i < N ? B[(size_t)i * N + j] : 0.0;
    x[u] = 0.0;
    r[u] = b;
    p[u] = b;
    part += b * b;
  }
  double rho = wave_sum(part);
  const double thr = tol * sqrt(rho);
  double* myp = ps + wv * LG;
  int it = 0, buf = 0;
  bool nonfinite = false;
  while (sqrt(rho) > thr && it < maxit && rho > 0.0) {
#pragma unroll
    for (int u = 0; u < RPL; ++u) myp[lane + 64 * u] = p[u];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // this wave's quarter of q = G p, four accumulation chains
    double qa[4][RPL];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int u = 0; u < RPL; ++u) qa[c][u] = 0.0;
#pragma unroll
    for (int c = 0; c < QR / 16; ++c) {
      const int l0 = wv * QR + 16 * c;
      v2d pv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) pv[t] = *reinterpret_cast<const v2d*>(myp + l0 + 2 * t);
#pragma unroll
      for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int u = 0; u < RPL; ++u) qa[t & 3][u] += gr[16 * c + t][u] * pv[t >> 1][t & 1];
    }
    double* qw = qp + (size_t)(buf * NW + wv) * LG;
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      qw[lane + 64 * u] = (qa[0][u] + qa[1][u]) + (qa[2][u] + qa[3][u]);
    __syncthreads();
    const double* qb = qp + (size_t)buf * NW * LG;
    buf ^= 1;
    double q[RPL];
    part = 0.0;
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int i = lane + 64 * u;
      q[u] = (qb[i] + qb[LG + i]) + (qb[2 * LG + i] + qb[3 * LG + i]);
      part += p[u] * q[u];
    }
    const double alpha = rho / wave_sum(part);
    part = 0.0;
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      x[u] += alpha * p[u];
      r[u] -= alpha * q[u];
      part += r[u] * r[u];
    }
    const double rho_new = wave_sum(part);
    const double beta = rho_new / rho;
#pragma unroll
    for (int u = 0; u < RPL; ++u) p[u] = r[u] + beta * p[u];
    rho = rho_new;
    ++it;
    // alpha and beta are the same in every lane and wave, so the exit is uniform
    if (!isfinite(alpha) || !isfinite(beta)) {
      nonfinite = true;
      break;
    }
  }
  if (wv != 0) return;
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int i = lane + 64 * u;
    if (i < N) W[(size_t)i * N + j] = x[u];
    if (i < NP) Wt[(size_t)j * NP + i] = (T)(i < N ? x[u] - (i == j ? 1.0 : 0.0) : 0.0);
  }
  if (lane == 0) {
    iters[j] = it;
    if (iters2) iters2[j] = it;
    status[j] = small_cg_status(nonfinite, rho, thr);
  }
}

// X_a = X_f + X_f (W - I) on the MFMA with W'^T = Wt read as prepared by the
// solve; RB-row tiles so that small n still spreads over the chip.
template <typename T, int NP, int RB>
__global__ __launch_bounds__(kBlock) void k_red_update(int n, int N, const T* Xf, T* Xa,
                                                       const T* Wtg) {
  using U = UCfg<T, NP, RB>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Wt = (T*)smem_raw;
  T* As = Wt + (size_t)NP * U::LD;
  double* mean = (double*)(As + (size_t)U::RBX * U::LD);
  // W'^T once per workgroup (16-byte loads, all in flight at once)
  constexpr int VW = 16 / (int)sizeof(T), NWL = NP * NP / VW / kBlock;
  static_assert(NWL * VW * kBlock == NP * NP, "W loads");
  const int tid = threadIdx.x;
  T wl[NWL][VW];
#pragma unroll
  for (int u = 0; u < NWL; ++u) {
    const int e = u * kBlock + tid, row = e / (NP / VW), c = (e - row * (NP / VW)) * VW;
    vload<VW>(Wtg + (size_t)row * NP + c, wl[u]);
  }
#pragma unroll
  for (int u = 0; u < NWL; ++u) {
    const int e = u * kBlock + tid, row = e / (NP / VW), c = (e - row * (NP / VW)) * VW;
#pragma unroll
    for (int v = 0; v < VW; ++v) Wt[row * U::LD + c + v] = wl[u][v];
  }
  update_tiles_stream<T, NP, kBlock, RB>(n, N, Xf, Xa, 1, As, As, Wt, mean);
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
                         hipStream_t s, const int* skip) {
  if (update_rows_ok(n, N, Xf, Xa)) {
    if (N <= 16) return launch_update_rows<T, 16, false>(n, N, Xf, Xa, Wd, nullptr, mode, skip, s);
    if (N <= 32) return launch_update_rows<T, 32, false>(n, N, Xf, Xa, Wd, nullptr, mode, skip, s);
    if (N <= 64) return launch_update_rows<T, 64, false>(n, N, Xf, Xa, Wd, nullptr, mode, skip, s);
    if constexpr (sizeof(T) == 4)
      if (N <= 128)
        return launch_update_rows<T, 128, false>(n, N, Xf, Xa, Wd, nullptr, mode, skip, s);
  }
  if (N <= 16) return launch_update_mfma<T, 16>(n, N, Xf, Xa, Wd, mode, skip, s);
  if (N <= 32) return launch_update_mfma<T, 32>(n, N, Xf, Xa, Wd, mode, skip, s);
  if (N <= 64) return launch_update_mfma<T, 64>(n, N, Xf, Xa, Wd, mode, skip, s);
  if constexpr (sizeof(T) == 4)
    if (N <= 128) return launch_update_mfma<T, 128>(n, N, Xf, Xa, Wd, mode, skip, s);
  // larger ensembles: one double FMA chain per element
  const int RBX = update_rows(N);
  const size_t sh = sizeof(double) * ((size_t)RBX * N + RBX);
  hipLaunchKernelGGL(k_update<T>, dim3((n + RBX - 1) / RBX), dim3(kBlock), sh, s, n, N, RBX, Xf,
                     Xa, Wd, mode, skip);
  return hipGetLastError();
}

int reduced_shape(int m, int N, int* NP, int* mpad, int* KC, int* S) {
  if (N < 2 || N > 128 || m < 1 || m > (1 << 30)) return 0;
  const int np = N <= 32 ? 32 : N <= 64 ? 64 : 128;
  if (np <= 64) {
    // gather and product fused: chunks of kRedFusedRows rows, no Q in memory
    *NP = np;
    *KC = kRedFusedRows;
    *S = (m + kRedFusedRows - 1) / kRedFusedRows;
    *mpad = *S * kRedFusedRows;
    return 1;
  }
  const int tiles = np == 32 ? RedCfg<32>::NTILE : np == 64 ? RedCfg<64>::NTILE : RedCfg<128>::NTILE;
  const long mp = ((long)m + 31) / 32 * 32, blocks = mp / 32;
  // about 512 workgroups, chunks of at least 64 rows
  long sc = (512 + tiles - 1) / tiles;
  const long smax = (mp + 63) / 64;
  if (sc > smax) sc = smax;
  if (sc < 1) sc = 1;
  const long kc = (blocks + sc - 1) / sc * 32;
  *NP = np;
  *mpad = (int)mp;
  *KC = (int)kc;
  *S = (int)((mp + kc - 1) / kc);
  return 1;
}

namespace {

template <typename T, int NP, int RB>
hipError_t launch_red_update(int n, int N, const T* Xf, T* Xa, const T* Wt, hipStream_t s) {
  using U = UCfg<T, NP, RB>;
  hipError_t e = hipFuncSetAttribute((const void*)k_red_update<T, NP, RB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)U::lds);
  if (e != hipSuccess) return e;
  // persistent: as many workgroups as run at once (each loads W once), at
  // most one per tile
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
      return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_red_update<T, NP, RB>, kBlock,
                                                          U::lds)) != hipSuccess)
      return e;
    resident = per * cus > 0 ? per * cus : 1;
  }
  const int tiles = (n + RB - 1) / RB;
  const int grid = tiles < resident ? tiles : resident;
  hipLaunchKernelGGL((k_red_update<T, NP, RB>), dim3(grid), dim3(kBlock), U::lds, s, n, N, Xf,
                     Xa, Wt);
  return hipGetLastError();
}

// The tallest row tile that fits the LDS and still gives every CU a workgroup.
template <typename T, int NP>
hipError_t launch_red_update_np(int n, int N, const T* Xf, T* Xa, const T* Wt, hipStream_t s) {
  if (update_rows_ok(n, N, Xf, (const T*)Xa))
    return launch_update_rows<T, NP, true>(n, N, Xf, Xa, nullptr, Wt, 1, nullptr, s);
  constexpr size_t lmax = 160 * 1024;
  if constexpr (UCfg<T, NP, 64>::lds <= lmax)
    if (n >= 64 * 256) return launch_red_update<T, NP, 64>(n, N, Xf, Xa, Wt, s);
  if constexpr (UCfg<T, NP, 32>::lds <= lmax)
    if (n >= 32 * 256) return launch_red_update<T, NP, 32>(n, N, Xf, Xa, Wt, s);
  static_assert(UCfg<T, NP, 16>::lds <= lmax, "update tile");
  return launch_red_update<T, NP, 16>(n, N, Xf, Xa, Wt, s);
}

template <typename T, int NP>
hipError_t launch_reduced_mfma(int n, int m, int N, int k, const T* Xf, T* Xa, const T* Xg, int ng,
                               const int32_t* idx, const T* hw, const T* y, const T* rdiag,
                               const T* eps, double tol, int maxit, void* ws, const Layout& L,
                               int* iters_out, hipStream_t s) {
  using C = RedCfg<NP>;
  unsigned char* base = (unsigned char*)ws;
  T* Q = (T*)(base + L.rQ);
  T* part = (T*)(base + L.rpart);
  double* Gp = (double*)(base + L.rG);
  double* B = (double*)(base + L.rB);
  double* Wd = (double*)(base + L.Wd);
  T* Wt = (T*)(base + L.rWt);
  int* iters = (int*)(base + L.riters);
  int* stat = (int*)(base + L.rstat);
  int* err = (int*)(base + L.err);
  int* errw = (int*)(base + L.rerr);
  const int LG = NP < 64 ? 64 : NP, RPL = LG / 64, NR = LG;
  hipError_t e;
  int nprep;
  if constexpr (NP <= 64) {
    nprep = L.rS;
    hipLaunchKernelGGL((k_red_pg<T, NP, false>), dim3(L.rS), dim3(kBlock), 0, s, ng, m, N, k, Xg,
                       idx, hw, y, rdiag, eps, part, errw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    nprep = L.rmpad / C::RPB;
    hipLaunchKernelGGL((k_red_prep<T, NP, false>), dim3(nprep), dim3(kBlock), 0, s, ng, m, N, k,
                       Xg, idx, hw, y, rdiag, eps, Q, errw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_red_gemm<T, NP>), dim3(C::NTILE, L.rS), dim3(kBlock), 0, s, L.rKC,
                       L.rmpad, 0, (const T*)Q, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int nsum = NR * LG + N * N, per = kBlock / 8;
  hipLaunchKernelGGL((k_red_sum2<T, NP>), dim3((nsum + per - 1) / per), dim3(kBlock), 0, s, N, NR,
                     LG, L.rS, (const T*)part, Gp, B, (const int*)errw, nprep, err, 1.0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds = sizeof(double) * (3 * (kBlock / 64) * (size_t)LG);
  if (RPL == 1) {
    if ((e = hipFuncSetAttribute((const void*)k_small_cg_w<T, 1>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
        hipSuccess)
      return e;
    hipLaunchKernelGGL((k_small_cg_w<T, 1>), dim3(NP), dim3(kBlock), lds, s, N, NP,
                       (const double*)Gp, (const double*)B, Wd, Wt, iters, iters_out, stat, tol,
                       maxit);
  } else {
    if ((e = hipFuncSetAttribute((const void*)k_small_cg_w<T, 2>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
        hipSuccess)
      return e;
    hipLaunchKernelGGL((k_small_cg_w<T, 2>), dim3(NP), dim3(kBlock), lds, s, N, NP,
                       (const double*)Gp, (const double*)B, Wd, Wt, iters, iters_out, stat, tol,
                       maxit);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_red_update_np<T, NP>(n, N, Xf, Xa, Wt, s);
}

}  // namespace

template <typename T>
hipError_t launch_reduced(int n, int m, int N, int k, const T* Xf, T* Xa, const T* Xg, int ng,
                          const int32_t* idx, const T* hw, const T* y, const T* rdiag,
                          const T* eps, double tol, int maxit, void* ws, const Layout& L,
                          int* iters_out, hipStream_t s) {
  if (L.rNP == 32)
    return launch_reduced_mfma<T, 32>(n, m, N, k, Xf, Xa, Xg, ng, idx, hw, y, rdiag, eps, tol, maxit, ws,
                                      L, iters_out, s);
  if (L.rNP == 64)
    return launch_reduced_mfma<T, 64>(n, m, N, k, Xf, Xa, Xg, ng, idx, hw, y, rdiag, eps, tol, maxit, ws,
                                      L, iters_out, s);
  if (L.rNP == 128)
    return launch_reduced_mfma<T, 128>(n, m, N, k, Xf, Xa, Xg, ng, idx, hw, y, rdiag, eps, tol, maxit,
                                       ws, L, iters_out, s);
  // N > 128: one workgroup per row block with scalar FP64 sums, then the
  // workgroup-per-column solve
  unsigned char* base = (unsigned char*)ws;
  double* part = (double*)(base + L.rpart);
  double* G = (double*)(base + L.rG);
  double* B = (double*)(base + L.rB);
  double* Wd = (double*)(base + L.Wd);
  int* iters = iters_out ? iters_out : (int*)(base + L.riters);
  const int nwg = L.nwg_max;
  const size_t sh = sizeof(double) * (2 * (size_t)L.RB * N + 2 * L.RB);
  int* err = (int*)(base + L.err);
  hipError_t e = launch_zero_u32((unsigned*)err, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_red_gram<T, false>), dim3(nwg), dim3(kBlock), sh, s, ng, m, N, k, L.RB,
                     L.nblk, Xg, idx, hw, y, rdiag, eps, part, err);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_red_sum, dim3((2 * N * N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, N,
                     nwg, part, G, B, 0, 1.0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_small_cg, dim3(N), dim3(kBlock), sizeof(double) * (4 * (size_t)N + kBlock),
                     s, N, G, B, Wd, iters, (int*)(base + L.rstat), tol, maxit);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (iters != (int*)(base + L.riters))
    if ((e = hipMemcpyAsync(base + L.riters, iters, sizeof(int) * N, hipMemcpyDeviceToDevice, s)) !=
        hipSuccess)
      return e;
  return launch_update<T>(n, N, Xf, Xa, Wd, 1, s);
}

// sEnKF analysis (Appendix A, Algorithm 3) with the reduced mode's layout:
// W = Zhat^T diag(Zhat Zhat^T + (N-1) R)^{-1} (Y - Z) from the SEN variants of
// its gather and product kernels and the partial sums (no solve), then
// X_a = X_f + X_f W, Algorithm 3's own form, on the reduced mode's update.
template <typename T, int NP>
hipError_t launch_senkf_mfma(int n, int m, int N, int k, const T* Xf, T* Xa, const int32_t* idx,
                             const T* hw, const T* y, const T* rdiag, const T* eps, void* ws,
                             const Layout& L, int* iters0, hipStream_t s) {
  using C = RedCfg<NP>;
  unsigned char* base = (unsigned char*)ws;
  T* Q = (T*)(base + L.rQ);
  T* part = (T*)(base + L.rpart);
  int* err = (int*)(base + L.err);
  int* errw = (int*)(base + L.rerr);
  hipError_t e;
  int nprep;
  if constexpr (NP <= 64) {
    nprep = L.rS;
    hipLaunchKernelGGL((k_red_pg<T, NP, true>), dim3(L.rS), dim3(kBlock), 0, s, n, m, N, k, Xf,
                       idx, hw, y, rdiag, eps, part, errw);
  } else {
    nprep = L.rmpad / C::RPB;
    hipLaunchKernelGGL((k_red_prep<T, NP, true>), dim3(nprep), dim3(kBlock), 0, s, n, m, N, k, Xf,
                       idx, hw, y, rdiag, eps, Q, errw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_red_gemm<T, NP>), dim3(C::NTILE - C::NTG, L.rS), dim3(kBlock), 0, s,
                       L.rKC, L.rmpad, C::NTG, (const T*)Q, part);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int per = kBlock / 8;
  T* Wt = (T*)(base + L.rWt);
  hipLaunchKernelGGL((k_senkf_sum<T, NP>), dim3((NP * NP + per - 1) / per), dim3(kBlock), 0, s,
                     N, L.rS, (const T*)part, Wt, (const int*)errw, nprep, err, iters0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_red_update_np<T, NP>(n, N, Xf, Xa, Wt, s);
}

template <typename T>
hipError_t launch_senkf(int n, int m, int N, int k, const T* Xf, T* Xa, const int32_t* idx,
                        const T* hw, const T* y, const T* rdiag, const T* eps, void* ws,
                        const Layout& L, int* iters0, hipStream_t s) {
  if (L.rNP == 32)
    return launch_senkf_mfma<T, 32>(n, m, N, k, Xf, Xa, idx, hw, y, rdiag, eps, ws, L, iters0, s);
  if (L.rNP == 64)
    return launch_senkf_mfma<T, 64>(n, m, N, k, Xf, Xa, idx, hw, y, rdiag, eps, ws, L, iters0, s);
  if (L.rNP == 128)
    return launch_senkf_mfma<T, 128>(n, m, N, k, Xf, Xa, idx, hw, y, rdiag, eps, ws, L, iters0,
                                     s);
  // N > 128: the row-block partials with FP64 sums
  unsigned char* base = (unsigned char*)ws;
  double* part = (double*)(base + L.rpart);
  double* G = (double*)(base + L.rG);
  double* B = (double*)(base + L.rB);
  int* err = (int*)(base + L.err);
  const size_t sh = sizeof(double) * (2 * (size_t)L.RB * N + 2 * L.RB);
  hipError_t e = launch_zero_u32((unsigned*)err, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_red_gram<T, true>), dim3(L.nwg_max), dim3(kBlock), sh, s, n, m, N, k,
                     L.RB, L.nblk, Xf, idx, hw, y, rdiag, eps, part, err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_red_sum, dim3((N * N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, N,
                     L.nwg_max, part, G, B, N * N, 0.0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (iters0 && (e = launch_zero_u32((unsigned*)iters0, N, s)) != hipSuccess) return e;
  return launch_update<T>(n, N, Xf, Xa, B, 0, s, nullptr);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_unscale_rows(int m, int N, T* z, const T* rdiag) {
  const long total = (long)m * N;
  for (long e = (long)blockIdx.x * kBlock + threadIdx.x; e < total; e += (long)gridDim.x * kBlock)
    z[e] = (T)((double)z[e] / sqrt((double)rdiag[e / N]));
}

template <typename T>
hipError_t launch_unscale_rows(int m, int N, T* z, const T* rdiag, hipStream_t s) {
  const long total = (long)m * N;
  long nb = (total + kBlock - 1) / kBlock;
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL(k_unscale_rows<T>, dim3((unsigned)nb), dim3(kBlock), 0, s, m, N, z, rdiag);
  return hipGetLastError();
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
  template hipError_t launch_update<T>(int, int, const T*, T*, const double*, int, hipStream_t, \
                                       const int*);                                           \
  template hipError_t launch_reduced<T>(int, int, int, int, const T*, T*, const T*, int,        \
                                        const int32_t*, const T*, const T*, const T*, const T*,  \
                                        double, int, void*, const Layout&, int*, hipStream_t);   \
  template hipError_t launch_validate<T>(int, int, int, int, const T*, const int32_t*, const T*, \
                                         const T*, const T*, const T*, const T*, int*,           \
                                         hipStream_t);                                           \
  template hipError_t launch_unscale_rows<T>(int, int, T*, const T*, hipStream_t);            \
  template hipError_t launch_senkf<T>(int, int, int, int, const T*, T*, const int32_t*, const T*, \
                                      const T*, const T*, const T*, void*, const Layout&, int*,   \
                                      hipStream_t);
CGD_INST(double)
CGD_INST(float)

}  // namespace cgd
