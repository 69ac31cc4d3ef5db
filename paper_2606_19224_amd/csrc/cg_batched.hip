// Batched CGD-EnKF analyses: many independent filters in one persistent launch.
//
// Each workgroup takes whole problems from an atomic queue (the host orders
// them by decreasing cost, so the longest start first) and solves each one
// alone, with no cross-workgroup synchronisation: the observation rows of
// its problem stream through LDS in blocks of 64 and every CG iteration is
// one fused pass over them (Sections 3.1-3.3):
//   p = r + beta p,  q = S_B G/(N-1) + R p,  z += alpha p,  r -= alpha q,
//   and the next iteration's S_B^T r and column sums, accumulated across
// blocks in registers.  Both block products run on the 16x16x4 MFMA.  The
// per-column decisions (alpha, beta, stop) are the same as in the other
// solvers and are taken by one thread per column.
#include "internal.h"
#include "mfma_util.h"

namespace cgd {

namespace {

constexpr int BRB = 64;  // observation rows per block

template <typename T, int NP>
struct BCfg {
  static constexpr int PAD = 16 / (int)sizeof(T);
  static constexpr int LDA = NP + PAD;     // row stride of S and Gs
  static constexpr int LDR = BRB + PAD;    // row stride of Rt
  static constexpr int TJ = NP / 16, TI = BRB / 16;
  static constexpr int NQ = TI * TJ, TQ = (NQ + 3) / 4;
  static constexpr int NG = TJ * TJ, TG = (NG + 3) / 4;
  static constexpr int KQ = NP / 4, KG = BRB / 4;
  static constexpr int JG = TJ > 4 ? TJ / 4 : 1;
};

template <typename T, int NP>
struct __align__(16) BLds {
  using C = BCfg<T, NP>;
  T S[BRB * C::LDA];
  T Rt[NP * C::LDR];
  T Gs[NP * C::LDA];   // G [j][k] (in place: old G, then new G)
  double Gr[NP * NP];  // S^T r over all rows [j][k], accumulated in double
  double acc[4][4][NP];
  double alpha[NP], beta[NP];
  int mode[NP];
  double rho[NP], rhoprev[NP], dn[NP], ad[NP], av[NP], bv[NP], cv[NP];
  int active[NP], fresh[NP], iters[NP], status[NP];
  T rv[BRB];
  double zb[BRB];
};

template <typename T>
constexpr size_t blds_bytes() {
  return sizeof(BLds<T, 64>) > sizeof(BLds<T, 32>)
             ? (sizeof(BLds<T, 64>) > sizeof(BLds<T, 16>) ? sizeof(BLds<T, 64>) : sizeof(BLds<T, 16>))
             : (sizeof(BLds<T, 32>) > sizeof(BLds<T, 16>) ? sizeof(BLds<T, 32>) : sizeof(BLds<T, 16>));
}

template <typename T, int NP>
__device__ void solve_one(const BProb<T>& P, double tol, int maxit, unsigned char* smem, int* err) {
  using C = BCfg<T, NP>;
  using V = typename Vec4<T>::type;
  BLds<T, NP>& L = *reinterpret_cast<BLds<T, NP>*>(smem);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int N = P.N, m = P.m, k = P.k;
  const int nblk = (m + BRB - 1) / BRB;
  const T inv = (T)(1.0 / (double)(N - 1));

  T zr[C::TQ][4], pr[C::TQ][4], rr[C::TQ][4];
  V gacc[C::TG];
  double cs[C::JG][4];
  auto elem_row = [&](int s, int i) { return ((wv + 4 * s) / C::TJ) * 16 + frag_row<T>(lk, i); };
  auto elem_col = [&](int s) { return ((wv + 4 * s) % C::TJ) * 16 + lr; };
  // Each lane owns the same Gram positions in gram_acc and pass_end, so the
  // double accumulator needs no barrier of its own.
  auto gram_slot = [&](int s, int i) {
    const int g = wv + 4 * s, tk = g / C::TJ, tj = g - tk * C::TJ;
    return (tj * 16 + lr) * NP + tk * 16 + frag_row<T>(lk, i);
  };
  auto pass_begin = [&]() {
#pragma unroll
    for (int s = 0; s < C::TG; ++s) {
      gacc[s] = V{0, 0, 0, 0};
      if (sizeof(T) == 4 && wv + 4 * s < C::NG)
#pragma unroll
        for (int i = 0; i < 4; ++i) L.Gr[gram_slot(s, i)] = 0.0;
    }
#pragma unroll
    for (int g = 0; g < C::JG; ++g)
#pragma unroll
      for (int f = 0; f < 4; ++f) cs[g][f] = 0.0;
  };
  auto cs_add = [&](int s, int f, double v) {
    if (wv + 4 * s < C::NQ) cs[s % C::JG][f] += v;
  };
  // S_B^T Rt^T for this wave's tiles (block in LDS).  FP64 accumulates
  // across blocks in the MFMA registers; FP32 takes each 64-row block
  // product from the MFMA and adds it to a double accumulator in LDS, since
  // a running FP32 sum over thousands of rows loses the digits that the
  // later CG iterations depend on.
  auto gram_acc = [&]() {
#pragma unroll
    for (int s = 0; s < C::TG; ++s) {
      const int g = wv + 4 * s;
      if (g < C::NG) {
        const int tk = g / C::TJ, tj = g - tk * C::TJ;
        T bv[C::KG];
        vload<C::KG>(L.Rt + (tj * 16 + lr) * C::LDR + lk * C::KG, bv);
        V c = sizeof(T) == 8 ? gacc[s] : V{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < C::KG; ++u)
          c = mfma4(L.S[(lk * C::KG + u) * C::LDA + tk * 16 + lr], bv[u], c);
        if constexpr (sizeof(T) == 8) {
          gacc[s] = c;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            L.Gr[gram_slot(s, i)] += (double)c[i];
        }
      }
    }
  };
  // End of a pass: reduced S^T r into L.Gr, column sums into fields 0..nf-1 of L.acc[0].
  auto pass_end = [&](int nf) {
    for (int e = lane; e < 4 * NP; e += 64) (&L.acc[wv][0][0])[e] = 0.0;
#pragma unroll
    for (int g = 0; g < C::JG; ++g)
      for (int f = 0; f < nf; ++f) {
        double v = cs[g][f];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (lk == 0) L.acc[wv][f][((wv + 4 * g) % C::TJ) * 16 + lr] = v;
      }
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int s = 0; s < C::TG; ++s)
        if (wv + 4 * s < C::NG)
#pragma unroll
          for (int i = 0; i < 4; ++i) L.Gr[gram_slot(s, i)] = gacc[s][i];
    }
    __syncthreads();
    for (int e = tid; e < nf * NP; e += kBlock) {
      const int f = e / NP, j = e - f * NP;
      const double v = (L.acc[0][f][j] + L.acc[1][f][j]) + (L.acc[2][f][j] + L.acc[3][f][j]);
      (f == 0 ? L.rho : f == 1 ? L.av : f == 2 ? L.bv : L.cv)[j] = v;
    }
    __syncthreads();
  };

  // ---------------- gather pass ----------------
  pass_begin();
  for (int blk = 0; blk < nblk; ++blk) {
    const int i0 = blk * BRB, rows = min(BRB, m - i0);
    // HX, S = HX - zbar and D = y + eps - HX in double, rounded once (the
    // FP32 cancellation in HX - zbar would be amplified by the conditioning
    // of Psi).  HX is gathered twice rather than held in registers, which
    // this kernel has none left for; the second gather hits in L2.
    auto gather = [&](int i, int j) {
      double h = 0.0;
      const int gi = i0 + i;
      for (int t = 0; t < k; ++t) {
        const int c = P.idx[(size_t)gi * k + t];
        if ((unsigned)c < (unsigned)P.n)
          h += (double)P.hw[(size_t)gi * k + t] * (double)P.Xf[(size_t)c * N + j];
        else
          atomicOr(err, 2);
      }
      return h;
    };
    for (int e = tid; e < BRB * NP; e += kBlock) {
      const int i = e / NP, j = e - i * NP;
      L.S[i * C::LDA + j] = (i < rows && j < N) ? (T)gather(i, j) : (T)0;
    }
    __syncthreads();
    for (int i = tid; i < BRB; i += kBlock) {
      double s = 0;
      for (int j = 0; j < N; ++j) s += (double)L.S[i * C::LDA + j];
      L.zb[i] = s / N;
      L.rv[i] = i < rows ? P.rdiag[i0 + i] : (T)0;
    }
    __syncthreads();
    for (int e = tid; e < BRB * NP; e += kBlock) {
      const int i = e / NP, j = e - i * NP;
      T s = 0, d = 0;
      if (i < rows && j < N) {
        const size_t g = (size_t)(i0 + i) * N + j;
        const double hd = gather(i, j);
        s = (T)(hd - L.zb[i]);
        double dd = (double)P.y[i0 + i] - hd;
        if (P.eps) dd += (double)P.eps[g];
        d = (T)dd;
        P.S[g] = s;
        P.D[g] = d;
        P.R[g] = d;
        P.P[g] = (T)0;
        P.Z[g] = (T)0;
      }
      L.S[i * C::LDA + j] = s;
      L.Rt[j * C::LDR + i] = d;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < C::TQ; ++s) {
      double d2 = 0, ad2 = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = elem_row(s, i);
        const bool ok = wv + 4 * s < C::NQ;
        const double d = ok ? (double)L.Rt[elem_col(s) * C::LDR + row] : 0.0;
        d2 += d * d;
        ad2 += (ok ? (double)L.rv[row] : 0.0) * d * d;
      }
      cs_add(s, 0, d2);
      cs_add(s, 1, ad2);
    }
    gram_acc();
    __syncthreads();
  }
  pass_end(2);
  for (int j = tid; j < NP; j += kBlock) {
    L.dn[j] = L.rho[j];
    L.ad[j] = L.av[j];
    L.av[j] = L.ad[j];
    L.bv[j] = 0.0;
    L.cv[j] = 0.0;
    L.active[j] = j < N ? 1 : 0;
    L.fresh[j] = 1;
    L.iters[j] = 0;
    L.status[j] = COL_RUNNING;
    L.rhoprev[j] = 0.0;
  }
  for (int e = tid; e < NP * C::LDA; e += kBlock) L.Gs[e] = (T)0;
  __syncthreads();

  // ---------------- CG iterations ----------------
  for (int kit = 0;; ++kit) {
    // per-column decision (thread j), G updated in place: G = S^T r + beta G
    int moving = 0;
    if (tid < N) {
      const int j = tid;
      int mode = MODE_FROZEN;
      double alpha = 0.0, beta = 0.0;
      if (L.active[j]) {
        const double rho = L.rho[j], dn = L.dn[j];
        if (sqrt(rho) <= tol * sqrt(dn)) {
          L.active[j] = 0;
          L.iters[j] = kit;
          L.status[j] = COL_CONVERGED;
        } else if (kit >= maxit) {
          L.active[j] = 0;
          L.iters[j] = kit;
          L.status[j] = COL_MAXIT;
        } else {
          beta = L.fresh[j] ? 0.0 : rho / L.rhoprev[j];
          double gg = 0.0;
          for (int kk = 0; kk < NP; ++kk) {
            double g = L.Gr[j * NP + kk];
            if (beta != 0.0) g += beta * (double)L.Gs[j * C::LDA + kk];
            const T gt = (T)g;
            L.Gs[j * C::LDA + kk] = gt;
            gg += (double)gt * (double)gt;
          }
          alpha = rho / (gg / (N - 1) + L.av[j] + 2.0 * beta * L.bv[j] + beta * beta * L.cv[j]);
          L.rhoprev[j] = rho;
          L.fresh[j] = 0;
          mode = MODE_STEP;
          if (!isfinite(alpha) || !isfinite(beta)) {
            L.active[j] = 0;
            L.iters[j] = kit;
            L.status[j] = COL_NONFINITE;
            mode = MODE_FROZEN;
            alpha = 0.0;
            beta = 0.0;
          }
        }
      }
      L.alpha[j] = alpha;
      L.beta[j] = beta;
      L.mode[j] = mode;
      moving = mode != MODE_FROZEN;
    } else if (tid < NP) {
      L.alpha[tid] = 0.0;
      L.beta[tid] = 0.0;
      L.mode[tid] = MODE_FROZEN;
    }
    if (!__syncthreads_or(moving)) break;

    pass_begin();
    for (int blk = 0; blk < nblk; ++blk) {
      const int i0 = blk * BRB, rows = min(BRB, m - i0);
      for (int e = tid; e < BRB * NP; e += kBlock) {
        const int i = e / NP, j = e - i * NP;
        L.S[i * C::LDA + j] = (i < rows && j < N) ? P.S[(size_t)(i0 + i) * N + j] : (T)0;
      }
      for (int i = tid; i < BRB; i += kBlock) L.rv[i] = i < rows ? P.rdiag[i0 + i] : (T)0;
      // this lane's elements of r, p, z
#pragma unroll
      for (int s = 0; s < C::TQ; ++s) {
        const int col = elem_col(s);
        const bool ok = wv + 4 * s < C::NQ && col < N;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = elem_row(s, i);
          if (ok && row < rows) {
            const size_t g = (size_t)(i0 + row) * N + col;
            rr[s][i] = P.R[g];
            pr[s][i] = P.P[g];
            zr[s][i] = P.Z[g];
          } else {
            rr[s][i] = 0;
            pr[s][i] = 0;
            zr[s][i] = 0;
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < C::TQ; ++s) {
        const int t = wv + 4 * s, col = elem_col(s);
        const int md = t < C::NQ ? L.mode[col] : MODE_FROZEN;
        const T be = (T)L.beta[col];
#pragma unroll
        for (int i = 0; i < 4; ++i) pr[s][i] = (md == MODE_STEP) ? rr[s][i] + be * pr[s][i] : (T)0;
      }
      V qacc[C::TQ];
#pragma unroll
      for (int s = 0; s < C::TQ; ++s) {
        const int t = wv + 4 * s;
        V c = {0, 0, 0, 0};
        if (t < C::NQ) {
          const int ti = t / C::TJ, tj = t - ti * C::TJ;
          T av[C::KQ], bv[C::KQ];
          vload<C::KQ>(L.S + (ti * 16 + lr) * C::LDA + lk * C::KQ, av);
          vload<C::KQ>(L.Gs + (tj * 16 + lr) * C::LDA + lk * C::KQ, bv);
#pragma unroll
          for (int u = 0; u < C::KQ; ++u) c = mfma4(av[u], bv[u], c);
        }
        qacc[s] = c;
      }
#pragma unroll
      for (int s = 0; s < C::TQ; ++s) {
        const int t = wv + 4 * s, col = elem_col(s);
        const int md = t < C::NQ ? L.mode[col] : MODE_FROZEN;
        const T al = (T)L.alpha[col];
        double r2 = 0, ar2 = 0, arp = 0, ap2 = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = elem_row(s, i);
          const T rv = t < C::NQ ? L.rv[row] : (T)0;
          if (md == MODE_STEP) {
            const T q = qacc[s][i] * inv + rv * pr[s][i];
            zr[s][i] += al * pr[s][i];
            rr[s][i] -= al * q;
            if (row < rows && col < N) {
              const size_t g = (size_t)(i0 + row) * N + col;
              P.R[g] = rr[s][i];
              P.P[g] = pr[s][i];
              P.Z[g] = zr[s][i];
            }
          }
          const double r = rr[s][i], p = pr[s][i];
          r2 += r * r;
          ar2 += (double)rv * r * r;
          arp += (double)rv * r * p;
          ap2 += (double)rv * p * p;
          if (t < C::NQ) L.Rt[col * C::LDR + row] = rr[s][i];
        }
        cs_add(s, 0, r2);
        cs_add(s, 1, ar2);
        cs_add(s, 2, arp);
        cs_add(s, 3, ap2);
      }
      __syncthreads();
      gram_acc();
      __syncthreads();
    }
    pass_end(4);
  }

  // ---------------- finish: W = S^T Z/(N-1) in double ----------------
  v4d wacc[C::TG];
#pragma unroll
  for (int s = 0; s < C::TG; ++s) wacc[s] = v4d{0, 0, 0, 0};
  for (int blk = 0; blk < nblk; ++blk) {
    const int i0 = blk * BRB, rows = min(BRB, m - i0);
    for (int e = tid; e < BRB * NP; e += kBlock) {
      const int i = e / NP, j = e - i * NP;
      const bool ok = i < rows && j < N;
      const size_t g = (size_t)(i0 + i) * N + j;
      L.S[i * C::LDA + j] = ok ? P.S[g] : (T)0;
      L.Rt[j * C::LDR + i] = ok ? P.Z[g] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < C::TG; ++s) {
      const int g = wv + 4 * s;
      if (g < C::NG) {
        const int tk = g / C::TJ, tj = g - tk * C::TJ;
        v4d c = wacc[s];
        for (int u = 0; u < C::KG; ++u)
          c = mfma4((double)L.S[(lk * C::KG + u) * C::LDA + tk * 16 + lr],
                    (double)L.Rt[(tj * 16 + lr) * C::LDR + lk * C::KG + u], c);
        wacc[s] = c;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < C::TG; ++s) {
    const int g = wv + 4 * s;
    if (g < C::NG) {
      const int tk = g / C::TJ, tj = g - tk * C::TJ;
      const int j = tj * 16 + lr;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kk = tk * 16 + frag_row<double>(lk, i);
        if (kk < N && j < N) P.Wd[(size_t)kk * N + j] = wacc[s][i] / (double)(N - 1);
      }
    }
  }
  for (int j = tid; j < N; j += kBlock) {
    P.iters[j] = L.iters[j];
    P.status[j] = L.status[j];
    if (P.iters_out) P.iters_out[j] = L.iters[j];
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_batched(const BProb<T>* probs, int count,
                                                       unsigned* queue, double tol, int maxit,
                                                       int* err) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int b = s_next;
    __syncthreads();
    if (b >= count) return;
    const BProb<T> P = probs[b];
    const int NP = P.N <= 16 ? 16 : (P.N <= 32 ? 32 : 64);
    if (NP == 16)
      solve_one<T, 16>(P, tol, maxit, smem_raw, err);
    else if (NP == 32)
      solve_one<T, 32>(P, tol, maxit, smem_raw, err);
    else
      solve_one<T, 64>(P, tol, maxit, smem_raw, err);
  }
}

// X_a = X_f + A W for every problem; blocks listed in a (problem, first row) table.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_batched(const BProb<T>* probs, const int2* table,
                                                           int RBX) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* tile = (double*)smem_raw;
  const int2 ent = table[blockIdx.x];
  const BProb<T>& P = probs[ent.x];
  const int N = P.N, n = P.n, tid = threadIdx.x;
  double* mean = tile + (size_t)RBX * N;
  const int i0 = ent.y, rows = min(RBX, n - i0), ne = rows * N;
  for (int e = tid; e < ne; e += kBlock) tile[e] = (double)P.Xf[(size_t)i0 * N + e];
  __syncthreads();
  for (int i = tid; i < rows; i += kBlock) {
    double s = 0;
    for (int j = 0; j < N; ++j) s += tile[i * N + j];
    mean[i] = s / N;
  }
  __syncthreads();
  for (int e = tid; e < ne; e += kBlock) {
    const int i = e / N, j = e - i * N;
    const double mu = mean[i];
    double acc = 0.0;
    for (int kk = 0; kk < N; ++kk) acc += (tile[i * N + kk] - mu) * P.Wd[(size_t)kk * N + j];
    P.Xa[(size_t)i0 * N + e] = (T)(tile[e] + acc);
  }
}

}  // namespace

template <typename T>
size_t batched_lds() {
  return blds_bytes<T>();
}

template <typename T>
int batched_coresident() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t sh = blds_bytes<T>();
  if (hipFuncSetAttribute((const void*)k_cg_batched<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)sh) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cg_batched<T>, kBlock, sh) != hipSuccess)
    return 0;
  return per * cus;
}

template <typename T>
hipError_t launch_batched(const BProb<T>* probs, int count, unsigned* queue, const int2* table,
                          int nupdate, int RBX, int nwg, double tol, int maxit, int* err,
                          hipEvent_t* ev, hipStream_t s) {
  hipError_t e = launch_zero_u32(queue, 1, s);
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
  const size_t sh = blds_bytes<T>();
  if ((e = hipFuncSetAttribute((const void*)k_cg_batched<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_cg_batched<T>, dim3(nwg), dim3(kBlock), sh, s, probs, count, queue, tol,
                     maxit, err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  const size_t shu = sizeof(double) * ((size_t)RBX * 64 + RBX);
  hipLaunchKernelGGL(k_update_batched<T>, dim3(nupdate), dim3(kBlock), shu, s, probs, table, RBX);
  return hipGetLastError();
}

template size_t batched_lds<float>();
template size_t batched_lds<double>();
template int batched_coresident<float>();
template int batched_coresident<double>();
template hipError_t launch_batched<float>(const BProb<float>*, int, unsigned*, const int2*, int,
                                          int, int, double, int, int*, hipEvent_t*, hipStream_t);
template hipError_t launch_batched<double>(const BProb<double>*, int, unsigned*, const int2*, int,
                                           int, int, double, int, int*, hipEvent_t*, hipStream_t);

}  // namespace cgd
