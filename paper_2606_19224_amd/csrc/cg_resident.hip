// Resident block-CG solver of the CGD-EnKF analysis (gfx950, MFMA).
//
// Same mathematics as the streaming solver (cg_solver.hip): gather, then N
// independent CG recurrences on Psi = S S^T/(N-1) + diag(r) sharing every
// product with S (Sections 3.1-3.3), one cross-workgroup reduction per
// iteration, then W = S^T Z/(N-1).  What changes is where the data lives:
//
//  * each workgroup owns ONE block of RB observation rows for the whole
//    solve (a cooperative launch makes all of them co-resident);
//  * its S block stays in LDS, and z, p, r of its rows stay in registers,
//    laid out exactly as the output fragments of the 16x16x4 MFMA that
//    computes Q = S_B G, so the CG vector updates are register-local;
//  * both contractions (Q = S_B G and the partial S_B^T R_B) run on MFMA
//    (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64), N padded to NP;
//  * workgroups exchange partial sums through per-workgroup epoch flags
//    (release store / acquire poll), never through a contended atomic:
//      arrive[w] = e   partials of workgroup w for exchange e are written
//      done[o]   = e   owner o has reduced its columns and published G, alpha, beta
//    Column j is owned by workgroup j % nwg.  Every wait is bounded; a wait
//    that runs out sets an error flag instead of hanging.
#include "internal.h"

namespace cgd {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef v4f type; };
template <> struct Vec4<double> { typedef v4d type; };

// Row (within a 16x16 output tile) of accumulator register i in lane group
// lk = lane / 16; the column is lane % 16.  The f32 16x16x4 MFMA returns
// rows 4*lk + i, the f64 one rows lk + 4*i (checked on gfx950).
template <typename A> __device__ constexpr int frag_row(int lk, int i);
template <> __device__ constexpr int frag_row<float>(int lk, int i) { return 4 * lk + i; }
template <> __device__ constexpr int frag_row<double>(int lk, int i) { return lk + 4 * i; }

constexpr long kSpinLimit = 1L << 25;

// All threads' prior global writes, then the flag.
__device__ inline void publish(unsigned* flag, unsigned epoch) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until flags[0..count) >= epoch, then make their writers' data visible.
__device__ inline void wait_flags(const unsigned* flags, int count, unsigned epoch, int* err) {
  for (int i = threadIdx.x; i < count; i += kBlock) {
    long spins = 0;
    while (__hip_atomic_load(&flags[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        atomicOr(err, 1);
        break;
      }
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename T, int NP, int RB>
struct Cfg {
  static constexpr int LD = NP + (sizeof(T) == 4 ? 4 : 2);  // padded LDS row stride
  static constexpr int TJ = NP / 16, TI = RB / 16;
  static constexpr int NQ = TI * TJ, TQ = (NQ + 3) / 4;       // Q tiles, per wave
  static constexpr int NG = TJ * TJ, TG = (NG + 3) / 4;       // Gram tiles, per wave
};

template <typename T, int NP, int RB>
struct __align__(16) Lds {
  T S[RB * Cfg<T, NP, RB>::LD];
  T R[RB * Cfg<T, NP, RB>::LD];
  T G[NP * Cfg<T, NP, RB>::LD];
  double acc[4][4][NP];    // [wave][scalar][column] partial column sums
  double alpha[NP], beta[NP];
  int mode[NP];
  T rv[RB];
  T zb[RB];
  double red[kBlock];
  int misc[8];
};

// Q tiles of this wave: acc[s] = S_B(tile rows, :) * B(:, tile cols), B from
// an LDS matrix B[k][j] with row stride LD (or, for FP64 W, from global).
template <typename T, int NP, int RB, typename BF>
__device__ inline void q_product(const T* Sl, BF bload, typename Vec4<T>::type (&acc)[Cfg<T, NP, RB>::TQ]) {
  using C = Cfg<T, NP, RB>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int s = 0; s < C::TQ; ++s) {
    const int t = wv + 4 * s;
    typename Vec4<T>::type c = {0, 0, 0, 0};
    if (t < C::NQ) {
      const int ti = t / C::TJ, tj = t - ti * C::TJ;
      const T* arow = Sl + (ti * 16 + lr) * C::LD + lk;
#pragma unroll 4
      for (int k0 = 0; k0 < NP; k0 += 4) c = mfma4(arow[k0], bload(k0 + lk, tj * 16 + lr), c);
    }
    acc[s] = c;
  }
}

// Gram tiles of this wave: acc[s] = S_B^T V_B for tile (tk, tj), V from LDS.
template <typename T, typename A, int NP, int RB>
__device__ inline void gram_product(const T* Sl, const T* Vl, typename Vec4<A>::type (&acc)[Cfg<T, NP, RB>::TG]) {
  using C = Cfg<T, NP, RB>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int s = 0; s < C::TG; ++s) {
    const int g = wv + 4 * s;
    typename Vec4<A>::type c = {0, 0, 0, 0};
    if (g < C::NG) {
      const int tk = g / C::TJ, tj = g - tk * C::TJ;
#pragma unroll 4
      for (int i0 = 0; i0 < RB; i0 += 4) {
        const int row = (i0 + lk) * C::LD;
        c = mfma4((A)Sl[row + tk * 16 + lr], (A)Vl[row + tj * 16 + lr], c);
      }
    }
    acc[s] = c;
  }
}

// Store this wave's Gram tiles as out[j * NP + k] (column j contiguous).
template <typename T, typename A, int NP, int RB>
__device__ inline void store_gram(const typename Vec4<A>::type (&acc)[Cfg<T, NP, RB>::TG], A* out) {
  using C = Cfg<T, NP, RB>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int s = 0; s < C::TG; ++s) {
    const int g = wv + 4 * s;
    if (g < C::NG) {
      const int tk = g / C::TJ, tj = g - tk * C::TJ;
      A* dst = out + (size_t)(tj * 16 + lr) * NP + tk * 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[frag_row<A>(lk, i)] = acc[s][i];
    }
  }
}

template <typename T, int NP, int RB>
__global__ __launch_bounds__(kBlock) void k_cg_resident(CGArgs<T> a) {
  using C = Cfg<T, NP, RB>;
  using V = typename Vec4<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Lds<T, NP, RB>& L = *reinterpret_cast<Lds<T, NP, RB>*>(smem_raw);
  const int tid = threadIdx.x, wg = blockIdx.x, nwg = gridDim.x;
  const int lane = tid & 63, wv = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int N = a.N, m = a.m;
  const int i0 = wg * RB, rows = min(RB, m - i0);
  const int nown = min(N, nwg);           // owner workgroups
  const bool owner = wg < N;
  const T inv = (T)(1.0 / (double)(N - 1));
  const bool warm = a.z0 != nullptr;
  unsigned* arrive = a.arrive;
  unsigned* done = a.done;
  unsigned epoch = 0;

  // registers: z, p, r of the elements this lane owns (Q fragment layout)
  T zr[C::TQ][4], pr[C::TQ][4], rr[C::TQ][4];

  // ---------------- initial column state ----------------
  for (int j = wg; j < N; j += nwg) {
    if (tid == 0) {
      a.coli[CI_ACTIVE * N + j] = 1;
      a.coli[CI_WARM * N + j] = warm ? 1 : 0;
      a.coli[CI_FRESH * N + j] = 1;
      a.coli[CI_ITERS * N + j] = 0;
      a.coli[CI_STATUS * N + j] = COL_RUNNING;
      a.coli[CI_FALLBACK * N + j] = 0;
    }
  }

  // ---------------- gather: S, D into LDS, r = d into registers ----------------
  for (int e = tid; e < RB * NP; e += kBlock) {
    const int i = e / NP, j = e - i * NP;
    T h = 0;
    if (i < rows && j < N) {
      const int gi = i0 + i;
      for (int t = 0; t < a.k; ++t) {
        const int c = a.idx[(size_t)gi * a.k + t];
        if ((unsigned)c < (unsigned)a.n)
          h += a.hw[(size_t)gi * a.k + t] * a.Xf[(size_t)c * N + j];
        else
          atomicOr(a.err, 2);
      }
    }
    L.R[i * C::LD + j] = h;
  }
  __syncthreads();
  for (int i = tid; i < RB; i += kBlock) {
    T s = 0;
    for (int j = 0; j < N; ++j) s += L.R[i * C::LD + j];
    L.zb[i] = s / (T)N;
    L.rv[i] = i < rows ? a.rdiag[i0 + i] : (T)0;
  }
  __syncthreads();
  for (int e = tid; e < RB * NP; e += kBlock) {
    const int i = e / NP, j = e - i * NP;
    T s = 0, d = 0;
    if (i < rows && j < N) {
      const size_t g = (size_t)(i0 + i) * N + j;
      const T h = L.R[i * C::LD + j];
      s = h - L.zb[i];
      d = a.y[i0 + i] - h;
      if (a.eps) d += a.eps[g];
      a.D[g] = d;
    }
    L.S[i * C::LD + j] = s;
    L.R[i * C::LD + j] = d;
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < C::TQ; ++s) {
    const int t = wv + 4 * s;
    const int ti = t / C::TJ, tj = t - ti * C::TJ;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      T d = 0, z = 0;
      if (t < C::NQ) {
        const int row = ti * 16 + frag_row<T>(lk, i), col = tj * 16 + lr;
        d = L.R[row * C::LD + col];
        if (warm && row < rows && col < N) z = a.z0[(size_t)(i0 + row) * N + col];
      }
      rr[s][i] = d;
      zr[s][i] = z;
      pr[s][i] = 0;
    }
  }

  // Column sums of this wave's fragments into L.acc[wv][f][col] (f < nf).
  auto colsum_begin = [&]() {
    for (int e = lane; e < 4 * NP; e += 64) (&L.acc[wv][0][0])[e] = 0.0;
    __syncthreads();
  };
  auto colsum_add = [&](int s, int f, double v) {
    // v: this lane's sum over its 4 rows of tile s; reduce over lk
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    const int t = wv + 4 * s;
    if (lk == 0 && t < C::NQ) {
      const int tj = t % C::TJ;
      L.acc[wv][f][tj * 16 + lr] += v;
    }
  };
  // Sum the 4 waves' column sums and write the workgroup's scalar partials.
  auto colsum_flush = [&](int f0, int nf, int dst0) {
    __syncthreads();
    for (int e = tid; e < nf * NP; e += kBlock) {
      const int f = e / NP, j = e - f * NP;
      const double v = L.acc[0][f0 + f][j] + L.acc[1][f0 + f][j] + L.acc[2][f0 + f][j] +
                       L.acc[3][f0 + f][j];
      a.partS[((size_t)wg * PS_NS + dst0 + f) * NP + j] = v;
    }
  };

  typename Vec4<T>::type gacc[C::TG];
  // partials of S^T d and (warm) S^T z0; scalars rho = a-sum etc. from r = d
  {
    colsum_begin();
#pragma unroll
    for (int s = 0; s < C::TQ; ++s) {
      double r2 = 0, ar2 = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = wv + 4 * s, row = (t / C::TJ) * 16 + frag_row<T>(lk, i);
        const double rv = (t < C::NQ) ? (double)L.rv[row] : 0.0;
        const double r = rr[s][i];
        r2 += r * r;
        ar2 += rv * r * r;
      }
      colsum_add(s, 0, r2);
      colsum_add(s, 1, ar2);
    }
    gram_product<T, T, NP, RB>(L.S, L.R, gacc);
    store_gram<T, T, NP, RB>(gacc, a.partG + (size_t)wg * NP * NP);
    colsum_flush(0, 2, PS_DN);  // PS_DN, PS_AD
    colsum_flush(0, 2, PS_RHO); // PS_RHO, PS_A (zero start: r = d)
    for (int j = tid; j < NP; j += kBlock) {
      a.partS[((size_t)wg * PS_NS + PS_B) * NP + j] = 0.0;
      a.partS[((size_t)wg * PS_NS + PS_C) * NP + j] = 0.0;
    }
    if (warm) {
      __syncthreads();
      // Z0 tile into R (reuse) for S^T z0
#pragma unroll
      for (int s = 0; s < C::TQ; ++s) {
        const int t = wv + 4 * s;
        if (t < C::NQ) {
          const int ti = t / C::TJ, tj = t - ti * C::TJ;
#pragma unroll
          for (int i = 0; i < 4; ++i) L.R[(ti * 16 + frag_row<T>(lk, i)) * C::LD + tj * 16 + lr] = zr[s][i];
        }
      }
      __syncthreads();
      gram_product<T, T, NP, RB>(L.S, L.R, gacc);
      store_gram<T, T, NP, RB>(gacc, a.partG2 + (size_t)wg * NP * NP);
    }
  }
  publish(&arrive[wg], ++epoch);

  if (warm) {
    // owners: Gd = sum S^T d, Gz = sum S^T z0 (into Gt[1]), dn, ad
    if (owner) {
      wait_flags(arrive, nwg, epoch, a.err);
      for (int j = wg; j < N; j += nwg) {
        for (int kk = tid; kk < NP; kk += kBlock) {
          T gd = 0, gz = 0;
          for (int w = 0; w < nwg; ++w) {
            gd += a.partG[((size_t)w * NP + j) * NP + kk];
            gz += a.partG2[((size_t)w * NP + j) * NP + kk];
          }
          a.Gd[(size_t)j * NP + kk] = gd;
          a.Gt[(size_t)NP * NP + (size_t)j * NP + kk] = gz;
        }
        if (tid < 2) {
          double s = 0;
          const int f = tid == 0 ? PS_DN : PS_AD;
          for (int w = 0; w < nwg; ++w) s += a.partS[((size_t)w * PS_NS + f) * NP + j];
          a.col[(tid == 0 ? CF_DN : CF_AD) * N + j] = s;
        }
      }
      publish(&done[wg], epoch);
    }
    wait_flags(done, nown, epoch, a.err);
    // Gz -> LDS as B[k][j]; r0 = d - S Gz/(N-1) - R z0
    for (int e = tid; e < NP * NP; e += kBlock) {
      const int j = e / NP, kk = e - j * NP;
      L.G[kk * C::LD + j] = (j < N) ? a.Gt[(size_t)NP * NP + e] : (T)0;
    }
    __syncthreads();
    V qacc[C::TQ];
    q_product<T, NP, RB>(L.S, [&](int kk, int j) { return L.G[kk * C::LD + j]; }, qacc);
    colsum_begin();
#pragma unroll
    for (int s = 0; s < C::TQ; ++s) {
      const int t = wv + 4 * s;
      const int ti = t / C::TJ, tj = t - ti * C::TJ;
      double r2 = 0, ar2 = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = ti * 16 + frag_row<T>(lk, i);
        const T rv = (t < C::NQ) ? L.rv[row] : (T)0;
        const T r = rr[s][i] - (qacc[s][i] * inv + rv * zr[s][i]);
        rr[s][i] = (t < C::NQ) ? r : (T)0;
        r2 += (double)rr[s][i] * rr[s][i];
        ar2 += (double)rv * rr[s][i] * rr[s][i];
        if (t < C::NQ) L.R[row * C::LD + tj * 16 + lr] = rr[s][i];
      }
      colsum_add(s, 0, r2);
      colsum_add(s, 1, ar2);
    }
    __syncthreads();
    gram_product<T, T, NP, RB>(L.S, L.R, gacc);
    store_gram<T, T, NP, RB>(gacc, a.partG + (size_t)wg * NP * NP);
    colsum_flush(0, 2, PS_RHO);
    publish(&arrive[wg], ++epoch);
  }

  // ---------------- CG iterations ----------------
  for (int kit = 0;; ++kit) {
    // ---- owners: reduce partials, decide alpha/beta, publish G ----
    if (owner) {
      wait_flags(arrive, nwg, epoch, a.err);
      const T* Gold = a.Gt + (size_t)((kit + 1) & 1) * NP * NP;
      T* Gcur = a.Gt + (size_t)(kit & 1) * NP * NP;
      int pending = 0;
      for (int j = wg; j < N; j += nwg) {
        // scalars: 6 kinds x nwg partials, thread (f, w-lane)
        {
          double v = 0;
          const int f = tid >> 5, wl = tid & 31;  // 8 groups of 32
          if (f < PS_NS)
            for (int w = wl; w < nwg; w += 32) v += a.partS[((size_t)w * PS_NS + f) * NP + j];
          L.red[tid] = v;
          __syncthreads();
          if (tid < PS_NS) {
            double s = 0;
            for (int q = 0; q < 32; ++q) s += L.red[tid * 32 + q];
            L.acc[0][0][tid] = s;  // scratch: scalar f at acc[0][0][f]
          }
          __syncthreads();
        }
        if (tid == 0) {
          const double rho = L.acc[0][0][PS_RHO];
          double dn, ad;
          if (kit == 0 && !warm) {
            dn = L.acc[0][0][PS_DN];
            ad = L.acc[0][0][PS_AD];
            a.col[CF_DN * N + j] = dn;
            a.col[CF_AD * N + j] = ad;
          } else {
            dn = a.col[CF_DN * N + j];
            ad = a.col[CF_AD * N + j];
          }
          int mode = MODE_FROZEN;
          double beta = 0.0;
          if (a.coli[CI_ACTIVE * N + j]) {
            const double nr = sqrt(rho), thr = a.tol * sqrt(dn);
            const bool cw = a.coli[CI_WARM * N + j] != 0;
            bool restart = false;
            if (kit == 0 && cw && a.fallback && rho > dn) {
              restart = true;
            } else if (nr <= thr) {
              a.coli[CI_ACTIVE * N + j] = 0;
              a.coli[CI_ITERS * N + j] = kit;
              a.coli[CI_STATUS * N + j] = COL_CONVERGED;
            } else if (kit >= a.maxit) {
              a.coli[CI_ACTIVE * N + j] = 0;
              a.coli[CI_ITERS * N + j] = kit;
              a.coli[CI_STATUS * N + j] = COL_MAXIT;
            } else if (cw && a.fallback && kit >= kStallWindow &&
                       nr > kStallFactor * a.col[(CF_HIST0 + (kit % kStallWindow)) * N + j]) {
              restart = true;
            } else {
              mode = MODE_STEP;
              beta = a.coli[CI_FRESH * N + j] ? 0.0 : rho / a.col[CF_RHOPREV * N + j];
            }
            if (cw) a.col[(CF_HIST0 + (kit % kStallWindow)) * N + j] = nr;
            if (restart) {
              a.coli[CI_WARM * N + j] = 0;
              a.coli[CI_FALLBACK * N + j] = 1;
              if (dn == 0.0 || a.tol >= 1.0) {
                mode = MODE_ZERO;
                a.coli[CI_ACTIVE * N + j] = 0;
                a.coli[CI_ITERS * N + j] = kit;
                a.coli[CI_STATUS * N + j] = COL_CONVERGED;
              } else {
                mode = MODE_RESTART;
              }
            }
          }
          L.red[0] = beta;
          L.red[1] = (double)mode;
          L.red[2] = dn;
          L.red[3] = ad;
        }
        __syncthreads();
        const int mode = (int)L.red[1];
        const double beta = L.red[0], dn = L.red[2], ad = L.red[3];
        const double rho = L.acc[0][0][PS_RHO], av = L.acc[0][0][PS_A];
        const double bv = L.acc[0][0][PS_B], cv = L.acc[0][0][PS_C];
        __syncthreads();
        // G column: thread (kk, group) sums over its share of workgroups
        double part = 0.0;
        {
          constexpr int GRP = kBlock / NP;  // >= 2
          const int kk = tid % NP, gq = tid / NP;
          double gsum = 0.0;
          if ((mode == MODE_STEP) && gq < GRP)
            for (int w = gq; w < nwg; w += GRP) gsum += (double)a.partG[((size_t)w * NP + j) * NP + kk];
          L.red[tid] = gsum;
          __syncthreads();
          if (tid < NP) {
            double g = 0.0;
            if (mode == MODE_STEP) {
              for (int q = 0; q < GRP; ++q) g += L.red[q * NP + tid];
              if (beta != 0.0) g += beta * (double)Gold[(size_t)j * NP + tid];
            } else if (mode == MODE_RESTART) {
              g = (double)a.Gd[(size_t)j * NP + tid];
            }
            const T gt = (T)g;
            if (mode == MODE_STEP || mode == MODE_RESTART) Gcur[(size_t)j * NP + tid] = gt;
            part = (double)gt * (double)gt;
          }
          __syncthreads();
        }
        L.red[tid] = part;
        __syncthreads();
        for (int sft = kBlock / 2; sft > 0; sft >>= 1) {
          if (tid < sft) L.red[tid] += L.red[tid + sft];
          __syncthreads();
        }
        if (tid == 0) {
          const double gg = L.red[0];
          double alpha = 0.0;
          int m2 = mode;
          if (mode == MODE_STEP) {
            alpha = rho / (gg / (N - 1) + av + 2.0 * beta * bv + beta * beta * cv);
            a.col[CF_RHOPREV * N + j] = rho;
          } else if (mode == MODE_RESTART) {
            alpha = dn / (gg / (N - 1) + ad);
            a.col[CF_RHOPREV * N + j] = dn;
          }
          if (mode == MODE_STEP || mode == MODE_RESTART) {
            a.coli[CI_FRESH * N + j] = 0;
            if (!isfinite(alpha) || !isfinite(beta)) {
              a.coli[CI_ACTIVE * N + j] = 0;
              a.coli[CI_ITERS * N + j] = kit;
              a.coli[CI_STATUS * N + j] = COL_NONFINITE;
              m2 = MODE_FROZEN;
              alpha = 0.0;
            }
          }
          a.col[CF_ALPHA * N + j] = alpha;
          a.col[CF_BETA * N + j] = (m2 == MODE_STEP) ? beta : 0.0;
          a.coli[CI_MODE * N + j] = m2;
          if (m2 != MODE_FROZEN) ++pending;
        }
        __syncthreads();
      }
      if (tid == 0) a.pend[wg] = pending;
      publish(&done[wg], epoch);
    }
    // ---- everyone: wait for the owners, then the row update ----
    wait_flags(done, nown, epoch, a.err);
    if (tid == 0) {
      int total = 0;
      for (int o = 0; o < nown; ++o) total += a.pend[o];
      L.misc[0] = total;
    }
    __syncthreads();
    if (L.misc[0] == 0) break;
    {
      const T* Gc = a.Gt + (size_t)(kit & 1) * NP * NP;
      for (int e = tid; e < NP * NP; e += kBlock) {
        const int j = e / NP, kk = e - j * NP;
        L.G[kk * C::LD + j] = (j < N) ? Gc[e] : (T)0;
      }
      for (int j = tid; j < NP; j += kBlock) {
        L.alpha[j] = j < N ? a.col[CF_ALPHA * N + j] : 0.0;
        L.beta[j] = j < N ? a.col[CF_BETA * N + j] : 0.0;
        L.mode[j] = j < N ? a.coli[CI_MODE * N + j] : MODE_FROZEN;
      }
    }
    __syncthreads();
    // p = r + beta p (restart: r = d, z = 0, p = d); frozen columns keep r, p = 0
#pragma unroll
    for (int s = 0; s < C::TQ; ++s) {
      const int t = wv + 4 * s;
      const int col = (t % C::TJ) * 16 + lr;
      const int md = (t < C::NQ) ? L.mode[col] : MODE_FROZEN;
      const T be = (T)L.beta[col];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = (t / C::TJ) * 16 + frag_row<T>(lk, i);
        if (md == MODE_STEP) {
          pr[s][i] = rr[s][i] + be * pr[s][i];
        } else if (md == MODE_RESTART || md == MODE_ZERO) {
          const T d = (row < rows && col < N) ? a.D[(size_t)(i0 + row) * N + col] : (T)0;
          rr[s][i] = d;
          zr[s][i] = 0;
          pr[s][i] = (md == MODE_RESTART) ? d : (T)0;
        } else {
          pr[s][i] = 0;
        }
      }
    }
    V qacc[C::TQ];
    q_product<T, NP, RB>(L.S, [&](int kk, int j) { return L.G[kk * C::LD + j]; }, qacc);
    colsum_begin();
#pragma unroll
    for (int s = 0; s < C::TQ; ++s) {
      const int t = wv + 4 * s;
      const int ti = t / C::TJ, tj = t - ti * C::TJ;
      const int col = tj * 16 + lr;
      const int md = (t < C::NQ) ? L.mode[col] : MODE_FROZEN;
      const T al = (T)L.alpha[col];
      double r2 = 0, ar2 = 0, arp = 0, ap2 = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = ti * 16 + frag_row<T>(lk, i);
        const T rv = (t < C::NQ) ? L.rv[row] : (T)0;
        if (md == MODE_STEP || md == MODE_RESTART) {
          const T q = qacc[s][i] * inv + rv * pr[s][i];
          zr[s][i] += al * pr[s][i];
          rr[s][i] -= al * q;
        }
        const double r = rr[s][i], p = pr[s][i];
        r2 += r * r;
        ar2 += (double)rv * r * r;
        arp += (double)rv * r * p;
        ap2 += (double)rv * p * p;
        if (t < C::NQ) L.R[row * C::LD + col] = rr[s][i];
      }
      colsum_add(s, 0, r2);
      colsum_add(s, 1, ar2);
      colsum_add(s, 2, arp);
      colsum_add(s, 3, ap2);
    }
    __syncthreads();
    gram_product<T, T, NP, RB>(L.S, L.R, gacc);
    store_gram<T, T, NP, RB>(gacc, a.partG + (size_t)wg * NP * NP);
    colsum_flush(0, 4, PS_RHO);  // PS_RHO, PS_A, PS_B, PS_C
    publish(&arrive[wg], ++epoch);
  }

  // ---------------- finish: z_out, W = S^T Z/(N-1) in double ----------------
#pragma unroll
  for (int s = 0; s < C::TQ; ++s) {
    const int t = wv + 4 * s;
    if (t < C::NQ) {
      const int ti = t / C::TJ, tj = t - ti * C::TJ;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = ti * 16 + frag_row<T>(lk, i), col = tj * 16 + lr;
        L.R[row * C::LD + col] = zr[s][i];
        if (row < rows && col < N) {
          const size_t g = (size_t)(i0 + row) * N + col;
          if (a.z_out) a.z_out[g] = zr[s][i];
          a.Z[g] = zr[s][i];
        }
      }
    }
  }
  __syncthreads();
  {
    v4d wacc[C::TG];
    gram_product<T, double, NP, RB>(L.S, L.R, wacc);
    store_gram<T, double, NP, RB>(wacc, a.partW + (size_t)wg * NP * NP);
  }
  publish(&arrive[wg], ++epoch);
  if (owner) {
    wait_flags(arrive, nwg, epoch, a.err);
    for (int j = wg; j < N; j += nwg) {
      constexpr int GRP = kBlock / NP;
      const int kk = tid % NP, gq = tid / NP;
      double s = 0.0;
      if (gq < GRP)
        for (int w = gq; w < nwg; w += GRP) s += a.partW[((size_t)w * NP + j) * NP + kk];
      L.red[tid] = s;
      __syncthreads();
      if (tid < N) {
        double v = 0.0;
        for (int q = 0; q < GRP; ++q) v += L.red[q * NP + tid];
        a.Wd[(size_t)tid * N + j] = v / (double)(N - 1);
      }
      if (tid == 0 && a.iters_out) a.iters_out[j] = a.coli[CI_ITERS * N + j];
      __syncthreads();
    }
    publish(&done[wg], epoch);
  }
  if (!a.want_relres) return;
  wait_flags(done, nown, epoch, a.err);
  // true residual d - S W - R z, double accumulation (FP64 MFMA on widened operands)
  {
    v4d racc[C::TQ];
    const double* Wd = a.Wd;
#pragma unroll
    for (int s = 0; s < C::TQ; ++s) {
      const int t = wv + 4 * s;
      v4d c = {0, 0, 0, 0};
      if (t < C::NQ) {
        const int ti = t / C::TJ, tj = t - ti * C::TJ;
        const int col = tj * 16 + lr;
        for (int k0 = 0; k0 < NP; k0 += 4) {
          const int kk = k0 + lk;
          const double b = (kk < N && col < N) ? Wd[(size_t)kk * N + col] : 0.0;
          c = mfma4((double)L.S[(ti * 16 + lr) * C::LD + kk], b, c);
        }
      }
      racc[s] = c;
    }
    colsum_begin();
#pragma unroll
    for (int s = 0; s < C::TQ; ++s) {
      const int t = wv + 4 * s;
      const int ti = t / C::TJ, tj = t - ti * C::TJ;
      const int col = tj * 16 + lr;
      double r2 = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // racc is in the f64 fragment layout; z is read back from the Z tile
        const int row = ti * 16 + frag_row<double>(lk, i);
        if (t < C::NQ && row < rows && col < N) {
          const double d = (double)a.D[(size_t)(i0 + row) * N + col];
          const double z = (double)L.R[row * C::LD + col];
          const double res = d - racc[s][i] - (double)L.rv[row] * z;
          r2 += res * res;
        }
      }
      colsum_add(s, 0, r2);
    }
    colsum_flush(0, 1, PS_RHO);
  }
  publish(&arrive[wg], ++epoch);
  if (owner) {
    wait_flags(arrive, nwg, epoch, a.err);
    for (int j = wg; j < N; j += nwg) {
      if (tid == 0) {
        double s = 0;
        for (int w = 0; w < nwg; ++w) s += a.partS[((size_t)w * PS_NS + PS_RHO) * NP + j];
        const double dn = a.col[CF_DN * N + j];
        const double rr2 = dn > 0 ? sqrt(s / dn) : 0.0;
        a.relres[j] = rr2;
        if (a.relres_out) a.relres_out[j] = rr2;
      }
    }
  }
}

__global__ void k_fill_u32(unsigned* p, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <typename T, int NP, int RB>
hipError_t launch_one(const CGArgs<T>& a, int nwg, hipStream_t s) {
  const size_t sh = sizeof(Lds<T, NP, RB>);
  const void* fn = (const void*)k_cg_resident<T, NP, RB>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  CGArgs<T> copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(fn, dim3(nwg), dim3(kBlock), args, sh, s);
}

template <typename T, int NP, int RB>
int coresident_one() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t sh = sizeof(Lds<T, NP, RB>);
  const void* fn = (const void*)k_cg_resident<T, NP, RB>;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cg_resident<T, NP, RB>, kBlock, sh) !=
      hipSuccess)
    return 0;
  return per * cus;
}

}  // namespace

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

// Resident variants: (NP, RB) menu per precision.
template <typename T>
int resident_np(int N) {
  if (N <= 16) return 16;
  if (N <= 32) return 32;
  if (N <= 64) return 64;
  if (sizeof(T) == 4 && N <= 128) return 128;
  return 0;
}

template <typename T>
size_t resident_lds(int NP, int RB) {
#define CGD_LDS_CASE(np, rb) if (NP == np && RB == rb) return sizeof(Lds<T, np, rb>);
  CGD_LDS_CASE(16, 16) CGD_LDS_CASE(16, 32) CGD_LDS_CASE(16, 64)
  CGD_LDS_CASE(32, 16) CGD_LDS_CASE(32, 32) CGD_LDS_CASE(32, 64)
  CGD_LDS_CASE(64, 16) CGD_LDS_CASE(64, 32) CGD_LDS_CASE(64, 64)
  if constexpr (sizeof(T) == 4) { CGD_LDS_CASE(128, 16) CGD_LDS_CASE(128, 32) CGD_LDS_CASE(128, 64) }
#undef CGD_LDS_CASE
  return 0;
}

template <typename T>
int resident_coresident(int NP, int RB) {
#define CGD_CO_CASE(np, rb) if (NP == np && RB == rb) return coresident_one<T, np, rb>();
  CGD_CO_CASE(16, 16) CGD_CO_CASE(16, 32) CGD_CO_CASE(16, 64)
  CGD_CO_CASE(32, 16) CGD_CO_CASE(32, 32) CGD_CO_CASE(32, 64)
  CGD_CO_CASE(64, 16) CGD_CO_CASE(64, 32) CGD_CO_CASE(64, 64)
  if constexpr (sizeof(T) == 4) { CGD_CO_CASE(128, 16) CGD_CO_CASE(128, 32) CGD_CO_CASE(128, 64) }
#undef CGD_CO_CASE
  return 0;
}

template <typename T>
hipError_t launch_cg_resident(const CGArgs<T>& a, int NP, int RB, int nwg, hipStream_t s) {
  // reset the exchange flags with a kernel (graph-capture safe)
  const int nflags = 2 * kMaxResidentGrid;
  hipLaunchKernelGGL(k_fill_u32, dim3((nflags + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     a.arrive, nflags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define CGD_L_CASE(np, rb) if (NP == np && RB == rb) return launch_one<T, np, rb>(a, nwg, s);
  CGD_L_CASE(16, 16) CGD_L_CASE(16, 32) CGD_L_CASE(16, 64)
  CGD_L_CASE(32, 16) CGD_L_CASE(32, 32) CGD_L_CASE(32, 64)
  CGD_L_CASE(64, 16) CGD_L_CASE(64, 32) CGD_L_CASE(64, 64)
  if constexpr (sizeof(T) == 4) { CGD_L_CASE(128, 16) CGD_L_CASE(128, 32) CGD_L_CASE(128, 64) }
#undef CGD_L_CASE
  return hipErrorInvalidValue;
}

template int resident_np<float>(int);
template int resident_np<double>(int);
template size_t resident_lds<float>(int, int);
template size_t resident_lds<double>(int, int);
template int resident_coresident<float>(int, int);
template int resident_coresident<double>(int, int);
template hipError_t launch_cg_resident<float>(const CGArgs<float>&, int, int, int, hipStream_t);
template hipError_t launch_cg_resident<double>(const CGArgs<double>&, int, int, int, hipStream_t);

}  // namespace cgd
