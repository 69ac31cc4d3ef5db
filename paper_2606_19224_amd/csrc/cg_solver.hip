// Persistent block-CG solver of the CGD-EnKF analysis (gfx950).
//
// One cooperative launch runs the whole analysis solve:
//   gather      S = H X_f - zbar 1^T, D = y 1^T + E - H X_f          (Sec. 2.3)
//   CG loop     N independent CG recurrences on Psi = S S^T/(N-1) + diag(r),
//               every product with S shared by all N columns          (Sec. 3.1-3.3)
//   finish      W = S^T Z / (N-1) and, on request, the true residual.
//
// Rows of the m x N observation-space arrays are split into blocks of RB
// rows; workgroup w owns blocks w, w + nwg, ...  The three-stage product of
// Section 3.3 (eq. matvec_decomp) maps onto this row-block distribution just
// as the paper's MPI ranks own row blocks: each workgroup forms its partial
// S_B^T v, the partials are summed across the grid in a fixed order (so the
// result is bitwise repeatable), then each workgroup applies S_B G / (N-1) +
// R_B v to its own rows.
//
// One grid reduction per CG iteration.  The row pass of iteration k updates
// z, r and then immediately forms the partials for iteration k+1:
//   S^T r,  rho = r^T r,  a = sum r_i r^2,  b = sum r_i r p,  c = sum r_i p^2
// (r_i = diag(R)).  With beta = rho/rho_prev the next search direction
// p' = r + beta p has  S^T p' = S^T r + beta S^T p  and
//   p'^T Psi p' = |S^T p'|^2/(N-1) + a + 2 beta b + beta^2 c,
// so alpha' = rho / p'^T Psi p' is known before p' is formed.  This is the
// textbook recurrence rearranged, not a different method: in exact
// arithmetic it produces the same iterates.
#include <hip/hip_cooperative_groups.h>

#include "internal.h"

namespace cg_ns = cooperative_groups;

namespace cgd {

namespace {

template <typename T>
struct Smem {
  T* s;        // RB * N
  T* r;        // RB * N
  T* p;        // RB * N
  T* rv;       // RB   diag(R) (or zbar in the gather)
  double* alpha;  // N
  double* beta;   // N
  int* mode;      // N
  double* red;    // kBlock + 16
};

__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~size_t(7); }

template <typename T>
__host__ __device__ inline size_t smem_bytes(int RB, int N) {
  size_t b = align8(sizeof(T) * (size_t)RB * N) * 3 + align8(sizeof(T) * (size_t)RB);
  b += sizeof(double) * 2 * (size_t)N + align8(sizeof(int) * (size_t)N);
  b += sizeof(double) * (kBlock + 16);
  return b;
}

template <typename T>
__device__ inline Smem<T> carve(unsigned char* base, int RB, int N) {
  Smem<T> sm;
  size_t o = 0;
  sm.s = (T*)(base + o); o += align8(sizeof(T) * (size_t)RB * N);
  sm.r = (T*)(base + o); o += align8(sizeof(T) * (size_t)RB * N);
  sm.p = (T*)(base + o); o += align8(sizeof(T) * (size_t)RB * N);
  sm.rv = (T*)(base + o); o += align8(sizeof(T) * (size_t)RB);
  sm.alpha = (double*)(base + o); o += sizeof(double) * N;
  sm.beta = (double*)(base + o); o += sizeof(double) * N;
  sm.mode = (int*)(base + o); o += align8(sizeof(int) * (size_t)N);
  sm.red = (double*)(base + o);
  return sm;
}

// Sum of one double per thread over the workgroup, fixed order.
__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  __syncthreads();
  red[tid] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  double out = red[0];
  __syncthreads();
  return out;
}

// Partial  S_B^T V_B  for the tiles in LDS, written (first block) or added
// into out[j * N + kk] for every (kk, j).
template <typename T, typename Acc, typename Out>
__device__ inline void tile_gram(const T* ls, const T* lv, int rows, int N, Out* out, bool first) {
  for (int o = threadIdx.x; o < N * N; o += kBlock) {
    const int j = o / N, kk = o - j * N;
    Acc acc = 0;
    for (int i = 0; i < rows; ++i) acc += (Acc)ls[i * N + kk] * (Acc)lv[i * N + j];
    out[o] = first ? (Out)acc : (Out)(out[o] + acc);
  }
}

template <typename T>
__device__ void decide(const CGArgs<T>& a, int kit, Smem<T>& sm, double* lsc) {
  const int tid = threadIdx.x, wg = blockIdx.x, nwg = gridDim.x, N = a.N;
  const T* Gold = a.Gt + (size_t)((kit + 1) & 1) * N * N;
  T* Gcur = a.Gt + (size_t)(kit & 1) * N * N;
  int pending = 0;
  for (int j = wg; j < N; j += nwg) {
    __syncthreads();
    if (tid < PS_NS) {
      double s = 0;
      for (int w = 0; w < nwg; ++w) s += a.partS[((size_t)w * PS_NS + tid) * N + j];
      lsc[tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
      double rho = lsc[PS_RHO];
      double dn, ad;
      if (kit == 0 && a.z0 == nullptr) {
        dn = lsc[PS_DN];
        ad = lsc[PS_AD];
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
        const bool warm = a.coli[CI_WARM * N + j] != 0;
        bool restart = false;
        if (kit == 0 && warm && a.fallback && rho > dn) {
          restart = true;
        } else if (nr <= thr) {
          a.coli[CI_ACTIVE * N + j] = 0;
          a.coli[CI_ITERS * N + j] = kit;
          a.coli[CI_STATUS * N + j] = COL_CONVERGED;
        } else if (kit >= a.maxit) {
          a.coli[CI_ACTIVE * N + j] = 0;
          a.coli[CI_ITERS * N + j] = kit;
          a.coli[CI_STATUS * N + j] = COL_MAXIT;
        } else if (warm && a.fallback && kit >= kStallWindow &&
                   nr > kStallFactor * a.col[(CF_HIST0 + (kit % kStallWindow)) * N + j]) {
          restart = true;
        } else {
          mode = MODE_STEP;
          beta = a.coli[CI_FRESH * N + j] ? 0.0 : rho / a.col[CF_RHOPREV * N + j];
        }
        if (warm) a.col[(CF_HIST0 + (kit % kStallWindow)) * N + j] = nr;
        if (restart) {
          a.coli[CI_WARM * N + j] = 0;
          a.coli[CI_FALLBACK * N + j] = 1;
          if (dn == 0.0 || a.tol >= 1.0) {  // converged at z = 0
            mode = MODE_ZERO;
            a.coli[CI_ACTIVE * N + j] = 0;
            a.coli[CI_ITERS * N + j] = kit;
            a.coli[CI_STATUS * N + j] = COL_CONVERGED;
          } else {
            mode = MODE_RESTART;
          }
        }
      }
      lsc[8] = beta;
      lsc[9] = (double)mode;
      lsc[10] = dn;
      lsc[11] = ad;
    }
    __syncthreads();
    const int mode = (int)lsc[9];
    const double beta = lsc[8];
    double part = 0.0;
    if (mode == MODE_STEP || mode == MODE_RESTART) {
      for (int kk = tid; kk < N; kk += kBlock) {
        double g;
        if (mode == MODE_STEP) {
          double gr = 0.0;
          for (int w = 0; w < nwg; ++w) gr += (double)a.partG[((size_t)w * N + j) * N + kk];
          g = gr;
          if (beta != 0.0) g += beta * (double)Gold[(size_t)j * N + kk];
        } else {
          g = (double)a.Gd[(size_t)j * N + kk];
        }
        const T gt = (T)g;
        Gcur[(size_t)j * N + kk] = gt;
        part += (double)gt * (double)gt;
      }
    }
    const double gg = block_sum(part, sm.red);
    if (tid == 0) {
      double alpha = 0.0;
      if (mode == MODE_STEP) {
        const double rho = lsc[PS_RHO];
        const double pi = gg / (N - 1) + lsc[PS_A] + 2.0 * beta * lsc[PS_B] +
                          beta * beta * lsc[PS_C];
        alpha = rho / pi;
        a.col[CF_RHOPREV * N + j] = rho;
      } else if (mode == MODE_RESTART) {
        const double dn = lsc[10];
        alpha = dn / (gg / (N - 1) + lsc[11]);
        a.col[CF_RHOPREV * N + j] = dn;
      }
      int m2 = mode;
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
  }
  if (tid == 0 && pending) atomicAdd(&a.ctr[kit & 1], pending);
}

// Row pass of iteration kit: p = r + beta p, q = S G/(N-1) + R p, z += alpha p,
// r -= alpha q, then the partials for the next decision.
template <typename T>
__device__ void row_pass(const CGArgs<T>& a, int kit, Smem<T>& sm) {
  const int tid = threadIdx.x, wg = blockIdx.x, nwg = gridDim.x, N = a.N, RB = a.RB;
  const T* G = a.Gt + (size_t)(kit & 1) * N * N;
  for (int j = tid; j < N; j += kBlock) {
    sm.alpha[j] = a.col[CF_ALPHA * N + j];
    sm.beta[j] = a.col[CF_BETA * N + j];
    sm.mode[j] = a.coli[CI_MODE * N + j];
  }
  __syncthreads();
  const T inv = (T)(1.0 / (double)(N - 1));
  for (int b = wg; b < a.nblk; b += nwg) {
    const bool first = (b == wg);
    const int i0 = b * RB, rows = min(RB, a.m - i0), ne = rows * N;
    for (int i = tid; i < rows; i += kBlock) sm.rv[i] = effective_r(a, i0 + i);
    for (int e = tid; e < ne; e += kBlock) {
      const int j = e % N;
      const size_t g = (size_t)i0 * N + e;
      const int mode = sm.mode[j];
      T r, p;
      if (mode == MODE_STEP) {
        r = a.R[g];
        p = r + (T)sm.beta[j] * a.P[g];
      } else if (mode == MODE_RESTART || mode == MODE_ZERO) {
        r = a.D[g];
        p = r;
      } else {
        r = a.R[g];
        p = (T)0;
      }
      sm.s[e] = a.S[g];
      sm.r[e] = r;
      sm.p[e] = p;
    }
    __syncthreads();
    for (int e = tid; e < ne; e += kBlock) {
      const int i = e / N, j = e - i * N;
      const int mode = sm.mode[j];
      if (mode == MODE_FROZEN) continue;
      const size_t g = (size_t)i0 * N + e;
      if (mode == MODE_ZERO) {
        a.Z[g] = (T)0;
        a.R[g] = sm.r[e];
        continue;
      }
      T q = 0;
      const T* srow = sm.s + i * N;
      const T* gcol = G + (size_t)j * N;
      for (int kk = 0; kk < N; ++kk) q += srow[kk] * gcol[kk];
      const T p = sm.p[e];
      q = q * inv + sm.rv[i] * p;
      const T al = (T)sm.alpha[j];
      const T z = (mode == MODE_RESTART ? (T)0 : a.Z[g]) + al * p;
      const T r = sm.r[e] - al * q;
      a.Z[g] = z;
      a.R[g] = r;
      a.P[g] = p;
      sm.r[e] = r;
    }
    __syncthreads();
    tile_gram<T, T, T>(sm.s, sm.r, rows, N, a.partG + (size_t)wg * N * N, first);
    for (int j = tid; j < N; j += kBlock) {
      double rho = 0, av = 0, bv = 0, cv = 0;
      for (int i = 0; i < rows; ++i) {
        const double r = sm.r[i * N + j], p = sm.p[i * N + j], rv = sm.rv[i];
        rho += r * r;
        av += rv * r * r;
        bv += rv * r * p;
        cv += rv * p * p;
      }
      double* ps = a.partS + (size_t)wg * PS_NS * N;
      if (first) {
        ps[PS_RHO * N + j] = rho; ps[PS_A * N + j] = av; ps[PS_B * N + j] = bv; ps[PS_C * N + j] = cv;
      } else {
        ps[PS_RHO * N + j] += rho; ps[PS_A * N + j] += av; ps[PS_B * N + j] += bv; ps[PS_C * N + j] += cv;
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_solve(CGArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cg_ns::grid_group grid = cg_ns::this_grid();
  const int tid = threadIdx.x, wg = blockIdx.x, nwg = gridDim.x;
  const int N = a.N, RB = a.RB, m = a.m;
  Smem<T> sm = carve<T>(smem_raw, RB, N);
  __shared__ double lsc[16];
  const bool warm = a.z0 != nullptr;

  // ---- initial column state (each column by its owner) and counters ----
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
  if (wg == 0 && tid < 4) a.ctr[tid] = 0;

  // ---- gather: S, D, Z, R; partials of S^T d (and S^T z0) ----
  for (int b = wg; b < a.nblk; b += nwg) {
    const bool first = (b == wg);
    const int i0 = b * RB, rows = min(RB, m - i0), ne = rows * N;
    // HX in double (rounded copy staged for the row means), S = HX - zbar and
    // D = y + eps - HX in double from a second gather, rounded once
    auto gather = [&](int e) {
      const int i = e / N, j = e - i * N, gi = i0 + i;
      double h = 0.0;
      for (int t = 0; t < a.k; ++t) {
        const int c = a.idx[(size_t)gi * a.k + t];
        if ((unsigned)c < (unsigned)a.ng)
          h += (double)a.hw[(size_t)gi * a.k + t] * (double)a.Xg[(size_t)c * N + j];
        else
          atomicOr(a.err, 2);
      }
      return h;
    };
    for (int e = tid; e < ne; e += kBlock) sm.p[e] = (T)gather(e);
    __syncthreads();
    for (int i = tid; i < rows; i += kBlock) {
      double s = 0;
      for (int j = 0; j < N; ++j) s += (double)sm.p[i * N + j];
      sm.red[i] = s / N;
    }
    __syncthreads();
    for (int e = tid; e < ne; e += kBlock) {
      const int i = e / N, gi = i0 + i;
      const size_t g = (size_t)i0 * N + e;
      const double hd = gather(e);
      const double sc = precond_row_scale(a, gi);
      const T s = (T)((hd - sm.red[i]) * sc);
      double dd = (double)a.y[gi] - hd;
      if (a.eps) dd += (double)a.eps[g];
      const T d = (T)(dd * sc);
      a.S[g] = s;
      a.D[g] = d;
      a.R[g] = d;
      a.P[g] = (T)0;
      const T z = warm ? precond_z0(a, gi, a.z0[g]) : (T)0;
      a.Z[g] = z;
      sm.s[e] = s;
      sm.r[e] = d;
      sm.p[e] = z;
    }
    __syncthreads();
    for (int i = tid; i < rows; i += kBlock) sm.rv[i] = effective_r(a, i0 + i);
    __syncthreads();
    if (warm) tile_gram<T, double, double>(sm.s, sm.p, rows, N, a.partW + (size_t)wg * N * N, first);
    tile_gram<T, T, T>(sm.s, sm.r, rows, N, a.partG + (size_t)wg * N * N, first);
    for (int j = tid; j < N; j += kBlock) {
      double dn = 0, ad = 0;
      for (int i = 0; i < rows; ++i) {
        const double d = sm.r[i * N + j];
        dn += d * d;
        ad += (double)sm.rv[i] * d * d;
      }
      double* ps = a.partS + (size_t)wg * PS_NS * N;
      if (first) {
        ps[PS_DN * N + j] = dn; ps[PS_AD * N + j] = ad;
        ps[PS_RHO * N + j] = dn; ps[PS_A * N + j] = ad;
        ps[PS_B * N + j] = 0; ps[PS_C * N + j] = 0;
      } else {
        ps[PS_DN * N + j] += dn; ps[PS_AD * N + j] += ad;
        ps[PS_RHO * N + j] += dn; ps[PS_A * N + j] += ad;
      }
    }
    __syncthreads();
  }
  grid.sync();

  if (warm) {
    // S^T d -> Gd and ||d||^2, sum r d^2 -> columns; S^T z0 -> Gt[1] (scratch)
    for (int j = wg; j < N; j += nwg) {
      for (int kk = tid; kk < N; kk += kBlock) {
        double gd = 0.0, gz = 0.0;
        for (int w = 0; w < nwg; ++w) {
          gd += (double)a.partG[((size_t)w * N + j) * N + kk];
          gz += a.partW[((size_t)w * N + j) * N + kk];
        }
        a.Gd[(size_t)j * N + kk] = (T)gd;
        a.Gt[(size_t)N * N + (size_t)j * N + kk] = (T)gz;
      }
      if (tid < 2) {
        double s = 0;
        const int f = tid == 0 ? PS_DN : PS_AD;
        for (int w = 0; w < nwg; ++w) s += a.partS[((size_t)w * PS_NS + f) * N + j];
        a.col[(tid == 0 ? CF_DN : CF_AD) * N + j] = s;
      }
    }
    grid.sync();
    // r0 = d - Psi z0, partials of S^T r0 and the scalars
    const T* Gz = a.Gt + (size_t)N * N;
    const T inv = (T)(1.0 / (double)(N - 1));
    for (int b = wg; b < a.nblk; b += nwg) {
      const bool first = (b == wg);
      const int i0 = b * RB, rows = min(RB, m - i0), ne = rows * N;
      for (int i = tid; i < rows; i += kBlock) sm.rv[i] = effective_r(a, i0 + i);
      for (int e = tid; e < ne; e += kBlock) sm.s[e] = a.S[(size_t)i0 * N + e];
      __syncthreads();
      for (int e = tid; e < ne; e += kBlock) {
        const int i = e / N, j = e - i * N;
        const size_t g = (size_t)i0 * N + e;
        T q = 0;
        for (int kk = 0; kk < N; ++kk) q += sm.s[i * N + kk] * Gz[(size_t)j * N + kk];
        const T z = a.Z[g];
        const T r = a.D[g] - (q * inv + sm.rv[i] * z);
        a.R[g] = r;
        sm.r[e] = r;
        sm.p[e] = (T)0;
      }
      __syncthreads();
      tile_gram<T, T, T>(sm.s, sm.r, rows, N, a.partG + (size_t)wg * N * N, first);
      for (int j = tid; j < N; j += kBlock) {
        double rho = 0, av = 0;
        for (int i = 0; i < rows; ++i) {
          const double r = sm.r[i * N + j];
          rho += r * r;
          av += (double)sm.rv[i] * r * r;
        }
        double* ps = a.partS + (size_t)wg * PS_NS * N;
        if (first) {
          ps[PS_RHO * N + j] = rho; ps[PS_A * N + j] = av;
          ps[PS_B * N + j] = 0; ps[PS_C * N + j] = 0;
        } else {
          ps[PS_RHO * N + j] += rho; ps[PS_A * N + j] += av;
        }
      }
      __syncthreads();
    }
    grid.sync();
  }

  // ---- CG iterations: decide (owners) | sync | row pass | sync ----
  for (int kit = 0;; ++kit) {
    decide<T>(a, kit, sm, lsc);
    grid.sync();
    if (__hip_atomic_load(&a.ctr[kit & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
    if (wg == 0 && tid == 0) a.ctr[(kit + 1) & 1] = 0;
    row_pass<T>(a, kit, sm);
    grid.sync();
  }

  // ---- finish: W = S^T Z/(N-1) in double, iteration counts, z_out ----
  for (int b = wg; b < a.nblk; b += nwg) {
    const bool first = (b == wg);
    const int i0 = b * RB, rows = min(RB, m - i0), ne = rows * N;
    for (int e = tid; e < ne; e += kBlock) {
      const size_t g = (size_t)i0 * N + e;
      sm.s[e] = a.S[g];
      const T z = a.Z[g];
      sm.p[e] = z;
      if (a.z_out) a.z_out[g] = z;
    }
    __syncthreads();
    tile_gram<T, double, double>(sm.s, sm.p, rows, N, a.partW + (size_t)wg * N * N, first);
    __syncthreads();
  }
  grid.sync();
  for (int j = wg; j < N; j += nwg) {
    for (int kk = tid; kk < N; kk += kBlock) {
      double acc = 0.0;
      for (int w = 0; w < nwg; ++w) acc += a.partW[((size_t)w * N + j) * N + kk];
      a.Wd[(size_t)kk * N + j] = acc / (double)(N - 1);
    }
    if (tid == 0 && a.iters_out) a.iters_out[j] = a.coli[CI_ITERS * N + j];
  }
  if (!a.want_relres) return;
  grid.sync();
  for (int b = wg; b < a.nblk; b += nwg) {
    const bool first = (b == wg);
    const int i0 = b * RB, rows = min(RB, m - i0), ne = rows * N;
    for (int i = tid; i < rows; i += kBlock) sm.rv[i] = effective_r(a, i0 + i);
    for (int e = tid; e < ne; e += kBlock) sm.s[e] = a.S[(size_t)i0 * N + e];
    __syncthreads();
    // true residual d - S W - R z with double accumulation, one column per thread
    for (int j = tid; j < N; j += kBlock) {
      double acc = 0.0;
      for (int i = 0; i < rows; ++i) {
        const size_t g = (size_t)(i0 + i) * N + j;
        double q = 0.0;
        for (int kk = 0; kk < N; ++kk) q += (double)sm.s[i * N + kk] * a.Wd[(size_t)kk * N + j];
        const double res = (double)a.D[g] - q - (double)sm.rv[i] * (double)a.Z[g];
        acc += res * res;
      }
      double* ps = a.partS + (size_t)wg * PS_NS * N;
      ps[PS_RHO * N + j] = first ? acc : ps[PS_RHO * N + j] + acc;
    }
    __syncthreads();
  }
  grid.sync();
  for (int j = wg; j < N; j += nwg) {
    if (tid == 0) {
      double s = 0;
      for (int w = 0; w < nwg; ++w) s += a.partS[((size_t)w * PS_NS + PS_RHO) * N + j];
      const double dn = a.col[CF_DN * N + j];
      const double rr = dn > 0 ? sqrt(s / dn) : 0.0;
      a.relres[j] = rr;
      if (a.relres_out) a.relres_out[j] = rr;
    }
  }
}

}  // namespace

template <typename T>
int cg_max_coresident(int RB, int N) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cg_solve<T>, kBlock,
                                                   smem_bytes<T>(RB, N)) != hipSuccess)
    return 0;
  return per * cus;
}

template <typename T>
hipError_t launch_cg_solve(const CGArgs<T>& a, int nwg, hipStream_t s) {
  CGArgs<T> copy = a;
  void* args[] = {&copy};
  const size_t sh = smem_bytes<T>(a.RB, a.N);
  if (sh > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_cg_solve<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
  }
  return hipLaunchCooperativeKernel((const void*)k_cg_solve<T>, dim3(nwg), dim3(kBlock), args, sh, s);
}

size_t cg_smem_bytes(int RB, int N, int prec) {
  return prec == CGD_FP64 ? smem_bytes<double>(RB, N) : smem_bytes<float>(RB, N);
}

template hipError_t launch_cg_solve<double>(const CGArgs<double>&, int, hipStream_t);
template hipError_t launch_cg_solve<float>(const CGArgs<float>&, int, hipStream_t);
template int cg_max_coresident<double>(int, int);
template int cg_max_coresident<float>(int, int);

}  // namespace cgd
