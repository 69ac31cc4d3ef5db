// Column-parallel CG solver of the CGD-EnKF analysis (gfx950).
//
// The N right-hand sides of Psi Z = D are independent CG recurrences that
// share only the matrix (Sections 3.1-3.3).  When S is small (m N values fit
// in an XCD's L2 many times over), sharing the matrix is cheaper than
// sharing the recurrences: one workgroup per ensemble member j runs column
// j's recurrence alone and streams S through L2 (the first RL rows stay in
// LDS) once per iteration, with no cross-workgroup traffic inside the CG
// loop.  One launch does the whole analysis:
//
//   1. gather: every workgroup forms a slice of rows of S = HX - zbar 1^T
//      and D = y 1^T + E - HX (HX in double, rounded once) and publishes it;
//   2. after one grid-wide flag exchange, workgroup j solves column j with
//      the one-pass rearranged iteration (per row: p = r + beta p,
//      q = S_i.G/(N-1) + r_i p_i, z += alpha p, r -= alpha q, and the next
//      S^T r accumulated on the fly), deciding alpha, beta and the stop rule
//      itself, and accumulates W_:j = S^T z_j/(N-1) as sum alpha_k G_k
//      (G_k = S^T p_k, starting from S^T z0 for a warm start);
//   3. after a second exchange, every workgroup applies the ensemble update
//      X_a = X_f + A W to its share of 64-row tiles (update_tile.h).
//
// S is stored by the gather in a plane layout so that every load
// instruction of a wave reads 1 KiB of consecutive bytes: lane (g, c) of a
// row step handles row g of the step and columns c*C .. c*C+C-1, and the
// 16-byte chunk v of that run lives at ((v * mp + i) * L + c) * VU.
#include <mutex>
#include <type_traits>
#include <vector>

#include "exchange.h"
#include "internal.h"
#include "mfma_util.h"
#include "update_tile.h"

namespace cgd {

namespace {

constexpr int kCB = 512;              // threads per workgroup
constexpr int kNW = kCB / 64;         // waves per workgroup
// dynamic LDS budget: 160 KiB less the kernel's static LDS (barrier helpers) and a margin
constexpr size_t kColLdsMax = 160 * 1024 - 1024;

template <typename T, int NP, bool MIX>
struct KC {
  static constexpr int VU = 16 / (int)sizeof(T);      // elements per 16-byte chunk of T
  // columns of S per lane: as many as registers allow (fewer lanes per row
  // means less per-row work repeated across the lanes of a row); the mixed
  // mode keeps 16 to leave room for its double-precision residual pass
  static constexpr int C = MIX ? (NP < 16 ? NP : 16)
                               : sizeof(T) == 4 ? (NP < 32 ? NP : 32) : (NP < 16 ? NP : 16);
  // element size of the LDS copy of S (BF16 in the mixed mode)
  static constexpr int SE = MIX ? 2 : (int)sizeof(T);
  static constexpr int L = NP / C;                    // lanes per row
  static constexpr int NV = C / VU;                   // chunks per lane and row
  static constexpr int RG = kCB / L;                  // rows per row step
  static constexpr int NPART = kNW * 4;                // Gram partials: one per 16-lane row
  // LDS copy of S, row-step major: chunk v of lane group cl of row i.  The
  // NV chunks a lane reads in one row step lie RG * L chunks apart, at
  // compile-time offsets from one address.
  static __device__ __host__ constexpr size_t lchunk(int i, int v, int cl) {
    return ((size_t)((i / RG) * NV + v) * RG + (i % RG)) * L + cl;
  }
  // fixed LDS: 5 vectors of mp are added at run time; then the S cache
  static constexpr size_t fixed = sizeof(T) * (size_t)NPART * NP      // red
                                  + sizeof(double) * 5 * NP          // Gr Gc Gd Gz Wc
                                  + sizeof(double) * NPART * 4       // red3
                                  + sizeof(double) * 32              // scal, hist
                                  + sizeof(T) * NP;                  // GcT
};

enum PassKind { PK_INIT, PK_WARM1, PK_WARM1D, PK_WARM2, PK_STEP, PK_RELRES, PK_TRUEW, PK_TRUER };
// mixed mode: an inner BF16 solve stops at this fraction of its outer residual
constexpr double kInnerRel = 1e-2;
enum ScalSlot { SC_RHO, SC_A, SC_B, SC_C, SC_ALPHA, SC_BETA, SC_MODE, SC_DN, SC_AD, SC_RHOPREV,
                SC_HIST = 16 };

template <typename T>
struct ColArgs {
  T* Sp;          // S in plane layout, mp x NP
  __bf16* Sh;     // mixed mode: the same layout in BF16 (else null)
  T* Dt;          // D transposed, N x mp
  int mp, RL;     // padded rows, rows of S cached in LDS
  // batched mode (vectors in global memory): z, r, p (N x mp each), diag(R)
  // padded to mp; null otherwise
  T* Vz;
  T* Vr;
  T* Vp;
  T* Rp;
  // split mode: the P workgroups of a member each own ms padded rows from
  // r0; partial sums travel through xb (flag-in-word exchange slots)
  int P, part, ms, r0;
  unsigned long long* xb;
  // single-problem solvers: W published as flag-in-word values (2 N^2 words)
  unsigned long long* wb;
};

// Split mode exchange: NP + 4 doubles per workgroup, each double as two
// 64-bit words (32 data bits, 32 epoch bits).
template <int NP>
struct XC {
  static constexpr int XS = NP + 4;   // Gram column sums, then the 4 scalar sums
  static constexpr int XW = 2 * XS;   // words per workgroup and exchange
};

// Rows [ib, ie) of one problem: HX (double), S = HX - zbar 1^T into the
// plane layout (and its BF16 copy), D = y 1^T + E - HX transposed, and, when
// ca.Rp is set, diag(R) padded with zeros to the padded row count.  SLICED
// instead stores S as consecutive slices of ca.ms rows, each in the LDS
// order of the split solver (KC::lchunk), so a workgroup copies its slice
// as one block.  Lanes take 4 columns of a row; U row steps have their
// loads in flight together (the index loads, then the dependent X_f loads).
template <typename T, int NP, bool MIX, bool SLICED = false>
__device__ void gather_rows(const CGArgs<T>& a, const ColArgs<T>& ca, int ib, int ie) {
  using K = KC<T, NP, MIX>;
  constexpr int CPL = 4;                 // columns per lane
  constexpr int LPR = NP / CPL;          // lanes per row (an aligned group of 4, 8 or 16)
  constexpr int RPS = kCB / LPR;         // rows per step
  constexpr int U = 4;
  const int tid = threadIdx.x, lr = tid % LPR, rw = tid / LPR, c0 = lr * CPL;
  const int N = a.N, m = a.m, mp = ca.mp;
  for (int s0 = ib; s0 < ie; s0 += U * RPS) {
    double h[U][CPL], yv[U];
    T ev[U][CPL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = s0 + u * RPS + rw;
      const bool live = i < ie && i < m;
      yv[u] = live ? (double)a.y[i] : 0.0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        h[u][c] = 0.0;
        ev[u][c] = (live && a.eps && c0 + c < N) ? a.eps[(size_t)i * N + c0 + c] : (T)0;
      }
    }
    for (int t = 0; t < a.k; ++t) {
      int col[U];
      double wt[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = s0 + u * RPS + rw;
        col[u] = 0;
        wt[u] = 0.0;
        if (i < ie && i < m) {
          const int cx = a.idx[(size_t)i * a.k + t];
          if ((unsigned)cx < (unsigned)a.ng) {
            col[u] = cx;
            wt[u] = (double)a.hw[(size_t)i * a.k + t];
          } else {
            atomicOr(a.err, 2);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < CPL; ++c)
          if (c0 + c < N) h[u][c] += wt[u] * (double)a.Xg[(size_t)col[u] * N + c0 + c];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = s0 + u * RPS + rw;
      double sum = 0.0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) sum += h[u][c];
      const double mean = group_sum<LPR>(sum) / N;  // all lanes take part (uniform loop)
      if (i < ie) {
        const double sc = i < m ? precond_row_scale(a, i) : 1.0;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          const int cc = c0 + c;
          const bool live = i < m && cc < N;
          const T sv = live ? (T)((h[u][c] - mean) * sc) : (T)0;
          const int g = cc / K::C, uu = cc % K::C, v = uu / K::VU, w = uu % K::VU;
          const size_t pos =
              SLICED ? (size_t)(i / ca.ms) * ca.ms * NP + K::lchunk(i % ca.ms, v, g) * K::VU + w
                     : (((size_t)v * mp + i) * K::L + g) * K::VU + w;
          ca.Sp[pos] = sv;
          if constexpr (MIX) ca.Sh[pos] = (__bf16)sv;
          if (cc < N)
            ca.Dt[(size_t)cc * mp + i] =
                live ? (T)((yv[u] - h[u][c] + (double)ev[u][c]) * sc) : (T)0;
        }
        if (ca.Rp && lr == 0) ca.Rp[i] = i < m ? effective_r(a, i) : (T)0;
      }
    }
  }
}

// Split mode, after the CG: the member's lead workgroup publishes column j
// of W = S^T Z/(N-1) as flag-in-word values (tag 1) in ws, element (k, j)
// in words 2 (k N + j) and 2 (k N + j) + 1 for T = double; for T = float the
// update only uses (T) W, so the element travels already rounded, as one
// word (k N + j), and the words a poll reads are contiguous.
template <typename T>
__device__ inline void split_publish_w(int N, int j, const double* Wc, double inv,
                                       unsigned long long* ws) {
  const int tid = threadIdx.x;
  if constexpr (sizeof(T) == 4) {
    if (tid < N) {
      const unsigned h = (unsigned)__float_as_int((float)(Wc[tid] * inv));
      __hip_atomic_store(ws + ((size_t)tid * N + j), (unsigned long long)h | (1ull << 32),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (tid < 2 * N) {
    const int k = tid >> 1;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(Wc[k] * inv);
    const unsigned h = (tid & 1) ? (unsigned)(bits >> 32) : (unsigned)bits;
    __hip_atomic_store(ws + 2 * ((size_t)k * N + j) + (tid & 1),
                       (unsigned long long)h | (1ull << 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Split mode: X_a = X_f + (X_f - xbar 1^T) W on this workgroup's share of
// 64-row tiles, once every member has published its column of W (whole
// rows per tile, so X_a is written in full lines).  A wait that runs out
// sets bit 0 of *err.
template <typename T, int NP>
__device__ void split_update_rows(const CGArgs<T>& a, const unsigned long long* ws,
                                  unsigned char* smem_raw) {
  using U = UCfg<T, NP>;
  const int tid = threadIdx.x, N = a.N;
  const int ntiles = (a.n + U::RBX - 1) / U::RBX;
  if ((int)blockIdx.x >= ntiles) return;
  T* As = (T*)smem_raw;
  T* Wt = As + (size_t)U::RBX * U::LD;
  double* mean = (double*)(Wt + (size_t)NP * U::LD);
  // the first tile's rows of X_f (they need no W) load while W is on its way
  update_tile_load<T, NP, kCB>(a.n, N, a.Xf, 0, (int)blockIdx.x * U::RBX, As, mean);
  // each thread's words (E elements, two words each) are polled together,
  // EC elements at a time: one round trip per poll, not one per word
  constexpr int E = (NP * NP + kCB - 1) / kCB, EC = E < 8 ? E : 8;
  constexpr int NH = sizeof(T) == 4 ? 1 : 2;  // words per element
  bool bad = false;
  long spins = 0;
  // first a light wait: thread j < N watches one word of member j's column
  if (tid < N) {
    while ((unsigned)(__hip_atomic_load(ws + NH * ((size_t)(N - 1) * N + tid) + NH - 1,
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) != 1u) {
      __builtin_amdgcn_s_sleep(8);
      if (++spins > kSpinLimit) {
        bad = true;
        break;
      }
    }
  }
  bad = __syncthreads_or(bad);
  for (int q0 = 0; q0 < E && !bad; q0 += EC) {
    unsigned long long x[EC][2];
    for (;;) {
      bool ready = true;
#pragma unroll
      for (int q = 0; q < EC; ++q) {
        const int e = tid + (q0 + q) * kCB, k = e / NP, jj = e % NP;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          if (e < NP * NP && k < N && jj < N) {
            x[q][h] = __hip_atomic_load(ws + NH * ((size_t)k * N + jj) + h, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
            ready = ready && (unsigned)(x[q][h] >> 32) == 1u;
          } else {
            x[q][h] = 1ull << 32;
          }
        }
      }
      if (ready) break;
      __builtin_amdgcn_s_sleep(4);
      if (++spins > kSpinLimit) {
        bad = true;
        break;
      }
    }
#pragma unroll
    for (int q = 0; q < EC; ++q) {
      const int e = tid + (q0 + q) * kCB, k = e / NP, jj = e % NP;
      if (e < NP * NP) {
        if constexpr (sizeof(T) == 4)
          Wt[jj * U::LD + k] = (T)__int_as_float((int)(x[q][0] & 0xffffffffull));
        else
          Wt[jj * U::LD + k] = (T)__longlong_as_double(
              (long long)((x[q][1] << 32) | (x[q][0] & 0xffffffffull)));
      }
    }
  }
  if (__syncthreads_or(bad)) {
    if (tid == 0) atomicOr(a.err, 1);
    return;
  }
  update_tile_apply<T, NP, kCB>(a.n, N, a.Xf, a.Xa, (int)blockIdx.x * U::RBX, As, Wt);
  for (int t = blockIdx.x + gridDim.x; t < ntiles; t += gridDim.x)
    update_tile<T, NP, kCB>(a.n, N, a.Xf, a.Xa, 0, t * U::RBX, As, Wt, mean);
}

// One member's CG (column j) over the gathered S and D, from step 2 of the
// single-problem kernel; writes W_:j, the column's iteration count and
// status, and optionally z and its true residual.  GV keeps z, r, p, d and
// diag(R) in global memory (any m; LDS then holds only reductions and the S
// cache), else in LDS.
// UPD: the launch applies the ensemble update itself (single-problem
// solvers; the batched mode has a launch of its own for it).
template <typename T, int NP, bool MIX, bool GV, bool SPLIT = false, bool UPD = true>
__device__ void column_phase(const CGArgs<T>& a, const ColArgs<T>& ca, int j,
                             unsigned char* smem_raw) {
  static_assert(!(SPLIT && (MIX || GV)), "split mode keeps its rows in LDS, full precision");
  using K = KC<T, NP, MIX>;
  using V = typename Vec4<T>::type;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int N = a.N, m = a.m, mp = ca.mp, RL = ca.RL;
  // rows of this workgroup: all mp, or (split mode) ms rows from global row r0
  const int ms = SPLIT ? ca.ms : mp;
  const int r0 = SPLIT ? ca.r0 : 0;
  const int cl = tid % K::L, g = tid / K::L;
  const double inv = 1.0 / (double)(N - 1);
  const T invT = (T)inv;
  constexpr int DH = (NP + 63) / 64;  // columns per lane of the decide (wave 0)

  // ---------------- LDS (and, with GV, global vectors) ----------------
  T* vz;
  T* vr;
  T* vp;
  const T* vd;
  const T* vrv;
  T* red;
  if constexpr (GV) {
    vz = ca.Vz + (size_t)j * mp;
    vr = ca.Vr + (size_t)j * mp;
    vp = ca.Vp + (size_t)j * mp;
    vd = ca.Dt + (size_t)j * mp;
    vrv = ca.Rp;
    red = (T*)smem_raw;
  } else {
    vz = (T*)smem_raw;
    vr = vz + ms;
    vp = vr + ms;
    vd = vp + ms;
    vrv = vd + ms;
    red = (T*)(vrv + ms);
  }
  double* Gr = (double*)(red + (size_t)K::NPART * NP);
  double* Gc = Gr + NP;
  double* Gd = Gc + NP;
  double* Gz = Gd + NP;
  double* Wc = Gz + NP;
  double* red3 = Wc + NP;                         // [NPART][4] scalar partials
  double* scal = red3 + K::NPART * 4;             // 32
  T* GcT = (T*)(scal + 32);                       // Gc as the row steps use it, in T
  T* Sc = GcT + NP;                               // RL x NP, plane layout
  __bf16* Sc16 = (__bf16*)(GcT + NP);             // mixed mode: the same in BF16
  unsigned* xh = (unsigned*)(Sc + (size_t)RL * NP);  // split mode: received exchange words

  // a plain launch's start-up census: check in now, wait after the S cache
  // fill below (which needs no other workgroup)
  unsigned long long census_count = 0;
  if constexpr (UPD) {
    if (a.census && tid == 0) census_count = census_arrive(a.census);
  }
  const bool warm = a.z0 != nullptr;
  // z itself is needed only for z_out, the true residual and the mixed
  // mode's outer steps: W accumulates alpha_k G_k, so the plain recurrence
  // can leave z alone
  const bool need_z = MIX || a.z_out != nullptr || a.want_relres;
  for (int i = tid; i < ms; i += kCB) {
    const T d = ca.Dt[(size_t)j * mp + r0 + i];
    if constexpr (!GV) {
      const_cast<T*>(vd)[i] = d;
      const_cast<T*>(vrv)[i] = r0 + i < m ? effective_r(a, r0 + i) : (T)0;
    }
    vr[i] = d;
    vp[i] = 0;
    vz[i] = (warm && r0 + i < m) ? precond_z0(a, r0 + i, a.z0[(size_t)(r0 + i) * N + j]) : (T)0;
  }
  // S cache: RL rows of each plane, one 16-byte chunk per copy (split mode:
  // the gather stored this workgroup's slice in LDS order, one block)
  if constexpr (SPLIT) {
    // the slice is contiguous and already in LDS order: LDS DMA, each wave
    // instruction 1 KiB (16 bytes per lane), no registers on the way
    typedef __attribute__((address_space(3))) unsigned char lds_u8;
    const unsigned char* src =
        reinterpret_cast<const unsigned char*>(ca.Sp + (size_t)ca.part * ms * NP);
    lds_u8* dst = (lds_u8*)(void*)Sc;
    const int nk = (int)(((size_t)ms * NP * sizeof(T)) >> 10);
    const int lane = tid & 63, wv = tid >> 6;
    for (int c = wv; c < nk; c += kNW)
      __builtin_amdgcn_global_load_lds(src + ((size_t)c << 10) + lane * 16, dst + (c << 10), 16,
                                       0, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  } else if constexpr (MIX) {
    const int per_plane = RL * K::L;  // chunks per plane
    for (int e = tid; e < K::NV * per_plane; e += kCB) {
      const int v = e / per_plane, r = e - v * per_plane;
      const size_t dst = K::lchunk(r / K::L, v, r % K::L) * K::VU;
      // a chunk of VU BF16 values is 8 bytes
      *reinterpret_cast<uint2*>(Sc16 + dst) =
          *reinterpret_cast<const uint2*>(ca.Sh + ((size_t)v * mp * K::L + r) * K::VU);
    }
  } else {
    // The cache by LDS DMA, 64 chunks (1 KiB) per wave instruction.  RL is a
    // multiple of the row step, so a plane holds whole row steps of kCB
    // chunks, and 64 consecutive chunks of a plane land in 64 consecutive
    // LDS chunks of one row step.
    static_assert(kCB % 64 == 0 && K::VU * (int)sizeof(T) == 16, "one 16-byte chunk per lane");
    typedef __attribute__((address_space(3))) unsigned char lds_u8;
    lds_u8* dst0 = (lds_u8*)(void*)Sc;
    const int per_plane = RL * K::L, nk = K::NV * per_plane / 64;
    const int lane = tid & 63, wv = tid >> 6;
    for (int c = wv; c < nk; c += kNW) {
      const int e0 = c * 64, v = e0 / per_plane, r0 = e0 - v * per_plane;
      const size_t dst = K::lchunk(r0 / K::L, v, r0 % K::L) * 16;
      const T* src = ca.Sp + ((size_t)v * mp * K::L + r0 + lane) * K::VU;
      __builtin_amdgcn_global_load_lds(src, dst0 + dst, 16, 0, 0);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  if (tid < NP) {
    Gc[tid] = 0.0;
    GcT[tid] = 0;
    Wc[tid] = 0.0;
  }
  // every workgroup must be resident before any wait on another one
  if constexpr (UPD) {
    if (a.census && !census_wait(a.census, a.err, a.census_ticks, census_count)) return;
  }
  __syncthreads();

  const int nsteps = ms / K::RG;
  // lane's chunks of row i (row step uniform: RL is a multiple of RG)
  // lane's chunks of row i: from the LDS cache (i < RL) or from global
  // memory.  Two separate functions, so that each load keeps its address
  // space (a merged pointer would become a flat load, which the compiler
  // must then wait for together with every LDS access).
  auto bf16_chunk = [&](const __bf16* p, T (&sv)[K::C], int v) {
    const uint2 x = *reinterpret_cast<const uint2*>(p);
    sv[v * K::VU + 0] = __uint_as_float(x.x << 16);
    sv[v * K::VU + 1] = __uint_as_float(x.x & 0xffff0000u);
    sv[v * K::VU + 2] = __uint_as_float(x.y << 16);
    sv[v * K::VU + 3] = __uint_as_float(x.y & 0xffff0000u);
  };
  auto load_row_lds = [&](int i, T (&sv)[K::C]) {
    if constexpr (MIX) {
      const __bf16* base = Sc16 + K::lchunk(i, 0, cl) * K::VU;
#pragma unroll
      for (int v = 0; v < K::NV; ++v) bf16_chunk(base + (size_t)v * K::RG * K::L * K::VU, sv, v);
    } else {
      T tmp[K::VU];
      const T* base = Sc + K::lchunk(i, 0, cl) * K::VU;
#pragma unroll
      for (int v = 0; v < K::NV; ++v) {
        vload<K::VU>(base + (size_t)v * K::RG * K::L * K::VU, tmp);
#pragma unroll
        for (int w = 0; w < K::VU; ++w) sv[v * K::VU + w] = tmp[w];
      }
    }
  };
  // full-precision rows from global memory (the mixed mode's outer residual)
  auto load_row_f32 = [&](int i, T (&sv)[K::C]) {
    T tmp[K::VU];
    const T* base = ca.Sp + ((size_t)(r0 + i) * K::L + cl) * K::VU;
#pragma unroll
    for (int v = 0; v < K::NV; ++v) {
      vload<K::VU>(base + (size_t)v * mp * K::L * K::VU, tmp);
#pragma unroll
      for (int w = 0; w < K::VU; ++w) sv[v * K::VU + w] = tmp[w];
    }
  };
  auto load_row_glb = [&](int i, T (&sv)[K::C]) {
    if constexpr (MIX) {
      const __bf16* base = ca.Sh + ((size_t)(r0 + i) * K::L + cl) * K::VU;
#pragma unroll
      for (int v = 0; v < K::NV; ++v) bf16_chunk(base + (size_t)v * mp * K::L * K::VU, sv, v);
    } else {
      load_row_f32(i, sv);
    }
  };
  const int nsl = min(RL / K::RG, nsteps);  // row steps served from the LDS cache

  // Split mode: sum the P workgroups' partials of the last pass (vec: its
  // NP Gram sums or null, and scal[SC_RHO..SC_C]) in part order, so every
  // workgroup of the member holds bitwise the same totals.  Each value
  // travels as two 64-bit words that carry the exchange number in their
  // upper halves, written and polled with agent-scope atomics: a word is
  // complete when its number is current, so no fence or cache maintenance
  // is needed.  Slots alternate by exchange parity (a workgroup cannot be
  // two exchanges ahead of a peer).  A wait that runs out sets bit 0 of
  // *err and xfail.
  unsigned xep = 0;
  bool xfail = false;
  auto split_exchange = [&](double* vec) {
    if constexpr (SPLIT) {
      using X = XC<NP>;
      const int P = ca.P;
      ++xep;
      unsigned long long* slot = ca.xb + ((size_t)j * 2 + (xep & 1)) * P * X::XW;
      if (tid < X::XW) {
        const int t = tid >> 1;
        const double v = t < NP ? (vec ? vec[t] : 0.0) : scal[SC_RHO + (t - NP)];
        const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
        const unsigned h = (tid & 1) ? (unsigned)(bits >> 32) : (unsigned)bits;
        __hip_atomic_store(slot + (size_t)ca.part * X::XW + tid,
                           (unsigned long long)h | ((unsigned long long)xep << 32),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      bool bad = false;
      for (int w = tid; w < P * X::XW; w += kCB) {
        long spins = 0;
        unsigned long long x;
        while ((unsigned)((x = __hip_atomic_load(slot + w, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) >> 32) != xep) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) {
            bad = true;
            break;
          }
        }
        xh[w] = (unsigned)x;
      }
      bad = __syncthreads_or(bad);
      if (tid < X::XS) {
        double sum = 0.0;
#pragma unroll 4
        for (int q = 0; q < P; ++q) {
          const unsigned lo = xh[q * X::XW + 2 * tid], hi = xh[q * X::XW + 2 * tid + 1];
          sum += __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
        }
        if (tid < NP) {
          if (vec) vec[tid] = sum;
        } else {
          scal[SC_RHO + (tid - NP)] = sum;
        }
      }
      __syncthreads();
      if (bad) {
        xfail = true;
        if (tid == 0) atomicOr(a.err, 1);
      }
    }
  };

  // One pass over all rows.  Reduces S^T x into Gr (and S^T d into Gd for
  // PK_WARM1, S^T z0 into Gz), and the scalar sums into scal[SC_RHO..SC_C].
  // Each lane loads the next row step's S chunks and row values while it
  // computes the current one; the L lanes of a row combine their partial dot products with DPP exchanges
  // and then hold bitwise-identical row values.
  auto pass = [&](auto kind_tag, T al, T be, int mode) {
    constexpr int kind = decltype(kind_tag)::value;
    constexpr bool kDot = kind == PK_WARM2 || kind == PK_STEP;
    T acc[K::C], gl[K::C], wl[K::C];
    double wd[kind == PK_TRUER ? K::C : 1];
    if constexpr (kind == PK_TRUER)
#pragma unroll
      for (int u = 0; u < K::C; ++u) wd[u] = Wc[cl * K::C + u] * inv;
    // a step's G in T, 16 bytes per load (the decide stores it so)
    if constexpr (kind == PK_STEP) vload<K::C>(GcT + cl * K::C, gl);
#pragma unroll
    for (int u = 0; u < K::C; ++u) {
      acc[u] = 0;
      const int k = cl * K::C + u;
      if constexpr (kind != PK_STEP) gl[u] = (T)(kind == PK_WARM2 ? Gz[k] : Gc[k]);
      wl[u] = (T)(Wc[k] * inv);
    }
    const bool restart = kind == PK_STEP && mode == MODE_RESTART;
    // per-lane scalar sums over its rows in T (a few terms each), combined in
    // double across lanes and waves
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    double r0 = 0, r1 = 0;  // PK_RELRES / PK_TRUER: residual sums, in double throughout
    struct RowV { T r, p, z, d, rv; };
    auto load_vals = [&](int i, RowV& v) {
      v.rv = vrv[i];
      if constexpr (kind == PK_INIT || kind == PK_STEP) v.r = vr[i];
      if constexpr (kind == PK_STEP) v.p = vp[i];
      if constexpr (kind == PK_STEP) {
        v.z = need_z ? vz[i] : (T)0;
      } else if constexpr (kind != PK_INIT && kind != PK_WARM1D) {
        v.z = vz[i];
      }
      if (kind == PK_WARM1 || kind == PK_WARM1D || kind == PK_WARM2 || kind == PK_RELRES ||
          kind == PK_TRUEW || kind == PK_TRUER || restart)
        v.d = vd[i];
    };
    auto row = [&](const T (&cur)[K::C], const RowV& v, int i) {
      if constexpr (kind == PK_TRUEW) {
        // S^T z with the full-precision S; ||d||^2 and sum r d^2 alongside
#pragma unroll
        for (int u = 0; u < K::C; ++u) acc[u] += cur[u] * v.z;
        s0 += v.d * v.d;
        s1 += v.rv * v.d * v.d;
      } else if constexpr (kind == PK_TRUER) {
        // true residual r = d - S W/(N-1) - R z in double (W from the last
        // full-precision S^T z), stored for the next inner solve; S^T r alongside
        double dp[2] = {0.0, 0.0};
#pragma unroll
        for (int u = 0; u < K::C; ++u) dp[u & 1] += (double)cur[u] * wd[u];
        const double dot = group_sum<K::L>(dp[0] + dp[1]);
        const double res = (double)v.d - dot - (double)v.rv * (double)v.z;
        const T x = (T)res;
        if (cl == 0) vr[i] = x;
        r0 += res * res;
        r1 += (double)v.rv * res * res;
#pragma unroll
        for (int u = 0; u < K::C; ++u) acc[u] += cur[u] * x;
      } else if constexpr (kind == PK_RELRES) {
        double dp[2] = {0.0, 0.0};
#pragma unroll
        for (int u = 0; u < K::C; ++u) dp[u & 1] += (double)cur[u] * wl[u];
        const double dot = group_sum<K::L>(dp[0] + dp[1]);
        const double res = (double)v.d - dot - (double)v.rv * (double)v.z;
        r0 += res * res;
      } else if constexpr (kind == PK_WARM1) {
#pragma unroll
        for (int u = 0; u < K::C; ++u) acc[u] += cur[u] * v.z;
        s0 += v.d * v.d;
        s1 += v.rv * v.d * v.d;
      } else if constexpr (kind == PK_WARM1D) {
#pragma unroll
        for (int u = 0; u < K::C; ++u) acc[u] += cur[u] * v.d;
      } else {
        T dot = 0;
        if constexpr (kDot) {
          constexpr int NPt = K::C >= 16 ? 4 : 2;
          T dp[NPt];
#pragma unroll
          for (int t = 0; t < NPt; ++t) dp[t] = 0;
#pragma unroll
          for (int u = 0; u < K::C; ++u) dp[u % NPt] += cur[u] * gl[u];
          dot = NPt == 4 ? (dp[0] + dp[1]) + (dp[2 % NPt] + dp[3 % NPt]) : dp[0] + dp[1];
          dot = group_sum<K::L>(dot);
        }
        T x;
        if constexpr (kind == PK_INIT) {
          x = v.r;
          s0 += x * x;
          s1 += v.rv * x * x;
        } else if constexpr (kind == PK_WARM2) {
          x = v.d - (dot * invT + v.rv * v.z);
          if (cl == 0) vr[i] = x;
          s0 += x * x;
          s1 += v.rv * x * x;
        } else {  // PK_STEP
          T ri = v.r, pi = v.p, zi = v.z;
          if (!restart) {
            pi = ri + be * pi;
          } else {  // MODE_RESTART: r = d, z = 0, p = d
            ri = v.d;
            zi = 0;
            pi = ri;
          }
          const T q = dot * invT + v.rv * pi;
          zi += al * pi;
          ri -= al * q;
          if (cl == 0) {
            vr[i] = ri;
            vp[i] = pi;
            if (need_z) vz[i] = zi;
          }
          x = ri;
          const T rr = v.rv * ri;
          s0 += ri * ri;
          s1 += rr * ri;
          s2 += rr * pi;
          s3 += v.rv * pi * pi;
        }
#pragma unroll
        for (int u = 0; u < K::C; ++u) acc[u] += cur[u] * x;
      }
    };
    // the cached and the streamed row steps run as two loops
    auto steps = [&](auto from_lds, int rb, int re) {
      auto load = [&](int i, T (&sv)[K::C]) {
        if constexpr (decltype(from_lds)::value == 1) load_row_lds(i, sv);
        else if constexpr (decltype(from_lds)::value == 2) load_row_f32(i, sv);
        else load_row_glb(i, sv);
      };
      // two register buffers in turn: step rs + 1 loads while step rs computes
      T bA[K::C], bB[K::C];
      RowV vA, vB;
      if (rb < re) {
        load(rb * K::RG + g, bA);
        load_vals(rb * K::RG + g, vA);
      }
      for (int rs = rb; rs < re; rs += 2) {
        if (rs + 1 < re) {
          load((rs + 1) * K::RG + g, bB);
          load_vals((rs + 1) * K::RG + g, vB);
        }
        row(bA, vA, rs * K::RG + g);
        if (rs + 1 < re) {
          if (rs + 2 < re) {
            load((rs + 2) * K::RG + g, bA);
            load_vals((rs + 2) * K::RG + g, vA);
          }
          row(bB, vB, (rs + 1) * K::RG + g);
        }
      }
    };
    if constexpr (kind == PK_TRUEW || kind == PK_TRUER) {
      steps(std::integral_constant<int, 2>{}, 0, nsteps);
    } else {
      steps(std::integral_constant<int, 1>{}, 0, nsl);
      steps(std::integral_constant<int, 0>{}, nsl, nsteps);
    }
    // ---- reductions (fixed order) ----
    // scalars: one lane per row contributes; the four sums go over each
    // 16-lane row in double with DPP, interleaved, and lane 0 of the row
    // writes a partial (the same 32 partials as the Gram sums)
    {
      const bool own = cl == 0;
      constexpr bool dbl = kind == PK_RELRES || kind == PK_TRUER;
      double v4[4] = {own ? (dbl ? r0 : (double)s0) : 0.0, own ? (dbl ? r1 : (double)s1) : 0.0,
                      own ? (double)s2 : 0.0, own ? (double)s3 : 0.0};
      // only the lanes with cl == 0 hold sums: rotate over those alone
      // (steps of L lanes), so lane 0 of the row ends with their total
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if constexpr (K::L <= 1) v4[f] += dpp<0x121>(v4[f]);  // row_ror:1
        if constexpr (K::L <= 2) v4[f] += dpp<0x122>(v4[f]);  // row_ror:2
        if constexpr (K::L <= 4) v4[f] += dpp<0x124>(v4[f]);  // row_ror:4
        if constexpr (K::L <= 8) v4[f] += dpp<0x128>(v4[f]);  // row_ror:8
      }
      if ((lane & 15) == 0)
#pragma unroll
        for (int f = 0; f < 4; ++f) red3[(wv * 4 + (lane >> 4)) * 4 + f] = v4[f];
    }
    // Gram: rotate-and-add inside each 16-lane row over the lanes holding the
    // same columns (lane % L), then lanes 0..L-1 of every row write a partial
    constexpr bool gram = kind != PK_RELRES;
    const int prow = wv * 4 + (lane >> 4);  // partial index: 16-lane row of the workgroup
    if constexpr (gram) {
#pragma unroll
      for (int u = 0; u < K::C; ++u) {
        T x = acc[u];
        if constexpr (K::L <= 1) x += dpp<0x121>(x);  // row_ror:1
        if constexpr (K::L <= 2) x += dpp<0x122>(x);  // row_ror:2
        if constexpr (K::L <= 4) x += dpp<0x124>(x);  // row_ror:4
        if constexpr (K::L <= 8) x += dpp<0x128>(x);  // row_ror:8
        // keep the last add in front of the writers' branch: inside it the
        // rotation's source lanes would be inactive, so it could not be
        // folded into the add
        asm volatile("" : "+v"(x));
        acc[u] = x;
      }
      if ((lane & 15) < K::L)
#pragma unroll
        for (int u = 0; u < K::C; ++u) red[(size_t)prow * NP + cl * K::C + u] = acc[u];
    }
    __syncthreads();
    // column c's 32 partials: GL consecutive lanes sum 32/GL each in double,
    // then a DPP tree over the GL (a fixed order); the scalars in 4 threads
    // of the last wave
    constexpr int GL = NP * 8 <= kCB - 64 ? 8 : NP * 4 <= kCB - 64 ? 4 : 2, GQ = K::NPART / GL;
    static_assert(NP * GL <= kCB - 64, "one wave left for the scalar sums");
    if (gram && tid < NP * GL) {
      const int c = tid / GL, q0 = (tid % GL) * GQ;
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < GQ; ++q) sum += (double)red[(size_t)(q0 + q) * NP + c];
      sum = group_sum<GL>(sum);
      if (tid % GL == 0)
        (kind == PK_WARM1 || kind == PK_TRUEW ? Gz : kind == PK_WARM1D ? Gd : Gr)[c] = sum;
    }
    if (tid >= kCB - 64 && tid < kCB - 32) {
      // scalar f's 32 partials: 8 lanes sum 4 each, then a DPP tree
      const int f = (tid - (kCB - 64)) >> 3, q0 = (tid & 7) * 4;
      double t = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) t += red3[(q0 + q) * 4 + f];
      t = group_sum<8>(t);
      if ((tid & 7) == 0) scal[SC_RHO + f] = t;
    }
    __syncthreads();
    if constexpr (SPLIT)
      split_exchange(gram ? (kind == PK_WARM1 || kind == PK_TRUEW ? Gz
                             : kind == PK_WARM1D                 ? Gd
                                                                 : Gr)
                          : nullptr);
  };
  using KInit = std::integral_constant<int, PK_INIT>;
  using KWarm1 = std::integral_constant<int, PK_WARM1>;
  using KWarm1d = std::integral_constant<int, PK_WARM1D>;
  using KWarm2 = std::integral_constant<int, PK_WARM2>;
  using KStep = std::integral_constant<int, PK_STEP>;
  using KRel = std::integral_constant<int, PK_RELRES>;
  using KTrueW = std::integral_constant<int, PK_TRUEW>;
  using KTrueR = std::integral_constant<int, PK_TRUER>;

  double dn = 0.0, ad = 0.0, mix_rho = 0.0;
  int status = COL_RUNNING, iters = 0, fell_back = 0;
  if constexpr (!MIX) {
  if (!warm) {
    pass(KInit{}, (T)0, (T)0, 0);
    dn = scal[SC_RHO];
    ad = scal[SC_A];
  } else {
    pass(KWarm1{}, (T)0, (T)0, 0);
    dn = scal[SC_RHO];
    ad = scal[SC_A];
    pass(KWarm1d{}, (T)0, (T)0, 0);
    if (tid < NP) Wc[tid] = Gz[tid];
    __syncthreads();
    pass(KWarm2{}, (T)0, (T)0, 0);
  }
  CGD_TRACE(3);
  // per-column state (wave 0; lane 0 decides)
  int c_warm = warm ? 1 : 0, c_fresh = 1;
  double rhoprev = 0.0;
  for (int kit = 0;; ++kit) {
    if (wv == 0) {
      int mode = MODE_FROZEN;
      double beta = 0.0;
      // this lane's columns of the new Gram sums and the last two G, read
      // while lane 0 decides
      double grl[DH], gcl[DH], gdl[DH];
#pragma unroll
      for (int h = 0; h < DH; ++h) {
        const int c = lane + 64 * h;
        grl[h] = c < NP ? Gr[c] : 0.0;
        gcl[h] = c < NP ? Gc[c] : 0.0;
        gdl[h] = c < NP ? Gd[c] : 0.0;
      }
      if (lane == 0) {
        const double rho = scal[SC_RHO];
        const double nr = sqrt(rho), thr = a.tol * sqrt(dn);
        bool restart = false;
        if (xfail) {
          status = COL_NONFINITE;
          iters = kit;
        } else if (kit == 0 && c_warm && a.fallback && rho > dn) {
          restart = true;
        } else if (nr <= thr) {
          status = COL_CONVERGED;
          iters = kit;
        } else if (kit >= a.maxit) {
          status = COL_MAXIT;
          iters = kit;
        } else if (c_warm && a.fallback && kit >= kStallWindow &&
                   nr > kStallFactor * scal[SC_HIST + kit % kStallWindow]) {
          restart = true;
        } else {
          mode = MODE_STEP;
          beta = c_fresh ? 0.0 : rho / rhoprev;
        }
        if (c_warm) scal[SC_HIST + kit % kStallWindow] = nr;
        if (restart) {
          c_warm = 0;
          fell_back = 1;
          if (dn == 0.0 || a.tol >= 1.0) {
            mode = MODE_ZERO;
            status = COL_CONVERGED;
            iters = kit;
          } else {
            mode = MODE_RESTART;
          }
        }
      }
      mode = readlane(mode, 0);
      beta = readlane(beta, 0);
      // new G = S^T p (rounded as the products use it) and its squared norm;
      // lane l holds columns l, l + 64, ...
      double gk[DH], gsq = 0.0;
#pragma unroll
      for (int h = 0; h < DH; ++h) {
        const int c = lane + 64 * h;
        gk[h] = 0.0;
        if (c < NP && (mode == MODE_STEP || mode == MODE_RESTART)) {
          const double gv = mode == MODE_STEP ? grl[h] + beta * gcl[h] : gdl[h];
          gk[h] = (double)(T)gv;
        }
        gsq += gk[h] * gk[h];
      }
      const double gg = wave_sum(gsq);
      double alpha = 0.0;
      const double rho = scal[SC_RHO];
      if (mode == MODE_STEP)
        alpha = rho / (gg * inv + scal[SC_A] + 2.0 * beta * scal[SC_B] + beta * beta * scal[SC_C]);
      else if (mode == MODE_RESTART)
        alpha = dn / (gg * inv + ad);
      if ((mode == MODE_STEP || mode == MODE_RESTART) && (!isfinite(alpha) || !isfinite(beta))) {
        if (lane == 0) {
          status = COL_NONFINITE;
          iters = kit;
        }
        mode = MODE_FROZEN;
        alpha = 0.0;
      }
#pragma unroll
      for (int h = 0; h < DH; ++h) {
        const int c = lane + 64 * h;
        if (c < NP) {
          if (mode == MODE_STEP || mode == MODE_RESTART) {
            Gc[c] = gk[h];
            GcT[c] = (T)gk[h];
            Wc[c] = (mode == MODE_RESTART ? 0.0 : Wc[c]) + alpha * gk[h];
          } else if (mode == MODE_ZERO) {
            Wc[c] = 0.0;
          }
        }
      }
      if (lane == 0) {
        if (mode == MODE_STEP || mode == MODE_RESTART) {
          rhoprev = mode == MODE_STEP ? rho : dn;
          c_fresh = 0;
        }
        scal[SC_ALPHA] = alpha;
        scal[SC_BETA] = beta;
        scal[SC_MODE] = (double)mode;
      }
    }
    __syncthreads();
    if (kit < 100) CGD_TRACE(4 + 2 * kit);
    const int mode = (int)scal[SC_MODE];
    if (mode == MODE_ZERO) {
      for (int i = tid; i < ms; i += kCB) {
        vz[i] = 0;
        vr[i] = vd[i];
      }
      __syncthreads();
      break;
    }
    if (mode != MODE_STEP && mode != MODE_RESTART) break;
    pass(KStep{}, (T)scal[SC_ALPHA], (T)scal[SC_BETA], mode);
    if (kit < 100) CGD_TRACE(5 + 2 * kit);
  }
  } else {
    // Mixed precision: restarted iterative refinement.  Outer step: W = S^T z
    // and the true residual r = d - Psi z with the FP32 S and double
    // accumulation; stop when ||r|| <= tol ||d||.  Inner solve: CG on the
    // BF16 copy of S for Psi delta = r from delta = 0 (z accumulates delta
    // directly), until its recursive residual drops below kInnerRel ||r||.
    // The iteration count is the total of inner steps; W is the exact S^T z
    // of the final outer step.
    for (int outer = 0;; ++outer) {
      pass(KTrueW{}, (T)0, (T)0, 0);
      if (outer == 0) {
        dn = scal[SC_RHO];
        ad = scal[SC_A];
      }
      if (tid < NP) Wc[tid] = Gz[tid];
      __syncthreads();
      pass(KTrueR{}, (T)0, (T)0, 0);
      mix_rho = scal[SC_RHO];
      if (!isfinite(mix_rho)) {
        status = COL_NONFINITE;
        break;
      }
      if (sqrt(mix_rho) <= a.tol * sqrt(dn)) {
        status = COL_CONVERGED;
        break;
      }
      if (iters >= a.maxit) {
        status = COL_MAXIT;
        break;
      }
      const double inner_thr = fmax(a.tol * sqrt(dn), kInnerRel * sqrt(mix_rho));
      double rhoprev = 0.0;
      for (int kin = 0;; ++kin) {
        if (wv == 0) {
          const double rho = scal[SC_RHO];
          int mode = MODE_STEP;
          if (sqrt(rho) <= inner_thr || iters + kin >= a.maxit ||
              (a.rr_period > 0 && kin >= a.rr_period))
            mode = MODE_FROZEN;
          const double beta = kin == 0 ? 0.0 : rho / rhoprev;
          double gk[DH], gsq = 0.0;
#pragma unroll
          for (int h = 0; h < DH; ++h) {
            const int c = lane + 64 * h;
            gk[h] = (c < NP && mode == MODE_STEP) ? (double)(T)(Gr[c] + beta * Gc[c]) : 0.0;
            gsq += gk[h] * gk[h];
          }
          const double gg = wave_sum(gsq);
          double alpha = 0.0;
          if (mode == MODE_STEP) {
            alpha = rho / (gg * inv + scal[SC_A] + 2.0 * beta * scal[SC_B] +
                           beta * beta * scal[SC_C]);
            if (!isfinite(alpha) || !isfinite(beta)) {
              mode = MODE_FROZEN;
              alpha = 0.0;
            }
          }
#pragma unroll
          for (int h = 0; h < DH; ++h)
            if (lane + 64 * h < NP && mode == MODE_STEP) {
              Gc[lane + 64 * h] = gk[h];
              GcT[lane + 64 * h] = (T)gk[h];
            }
          rhoprev = rho;
          if (lane == 0) {
            scal[SC_ALPHA] = alpha;
            scal[SC_BETA] = beta;
            scal[SC_MODE] = (double)mode;
          }
        }
        __syncthreads();
        if ((int)scal[SC_MODE] != MODE_STEP) {
          iters += kin;
          break;
        }
        pass(KStep{}, (T)scal[SC_ALPHA], (T)scal[SC_BETA], MODE_STEP);
      }
      __syncthreads();
    }
  }
  CGD_TRACE(250);

  // ---------------- finish column j ----------------
  const bool lead = !SPLIT || ca.part == 0;  // writes the member's per-column results
  if (tid == 0 && lead) {
    a.coli[CI_ITERS * N + j] = iters;
    a.coli[CI_STATUS * N + j] = status;
    a.coli[CI_FALLBACK * N + j] = fell_back;
    a.col[CF_DN * N + j] = dn;
    if (a.iters_out) a.iters_out[j] = iters;
  }
  if (tid < N && lead) a.Wd[(size_t)tid * N + j] = Wc[tid] * inv;
  if (a.z_out)
    for (int i = tid; i < ms && r0 + i < m; i += kCB) a.z_out[(size_t)(r0 + i) * N + j] = vz[i];
  if (MIX && a.want_relres) {
    if (tid == 0) {
      const double rr2 = dn > 0 ? sqrt(mix_rho / dn) : 0.0;
      a.relres[j] = rr2;
      if (a.relres_out) a.relres_out[j] = rr2;
    }
  } else if (a.want_relres) {
    pass(KRel{}, (T)0, (T)0, 0);
    if (tid == 0 && lead) {
      const double rr2 = dn > 0 ? sqrt(scal[SC_RHO] / dn) : 0.0;
      a.relres[j] = rr2;
      if (a.relres_out) a.relres_out[j] = rr2;
    }
  }
  // ensemble update (single-problem solvers): publish column j of W, then
  // the workgroups with a 64-row tile of X_a apply it once all columns are in
  if constexpr (UPD) {
    CGD_TRACE(251);
    if (lead) split_publish_w<T>(N, j, Wc, inv, ca.wb);
    __syncthreads();
    split_update_rows<T, NP>(a, ca.wb, smem_raw);
    CGD_TRACE(253);
  }

}

// Workgroup 0 of a per-member solver: the gather's error words into *err.
template <typename T>
__device__ inline void fold_gather_errors(const CGArgs<T>& a) {
  if (blockIdx.x != 0 || !a.gerr) return;
  int f = 0;
  for (int e = threadIdx.x; e < a.ngerr; e += kCB) f |= a.gerr[e];
  if (f) atomicOr(a.err, f);
}

template <typename T, int NP, bool MIX, bool GV>
__global__ __launch_bounds__(kCB) void k_cg_columns(CGArgs<T> a, ColArgs<T> ca) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  CGD_TRACE(0);
  fold_gather_errors(a);
  column_phase<T, NP, MIX, GV>(a, ca, blockIdx.x, smem_raw);
}

// The gather of S, D (and diag(R)) as a launch of its own, one row step per
// workgroup, ahead of the solvers that then read them with no grid-wide wait.
// With a.gerr set, workgroups past the ng gather ones clear the solver's
// exchange words (a.zp) and the error word, and each gather workgroup writes
// its own error word, so no launch has to clear anything beforehand.
template <typename T, int NP, bool MIX, bool SLICED>
__global__ __launch_bounds__(kCB) void k_gather(CGArgs<T> a, ColArgs<T> ca, int ng) {
  constexpr int R = kCB * 2 / NP;  // rows per workgroup: half a step of gather_rows
  if ((int)blockIdx.x >= ng) {
    const long nz = (long)(gridDim.x - ng) * kCB;
    for (long e = (long)(blockIdx.x - ng) * kCB + threadIdx.x; e < a.zn; e += nz) a.zp[e] = 0u;
    if ((int)blockIdx.x == ng && threadIdx.x == 0) *a.err = 0;
    return;
  }
  __shared__ int gerr;
  if (threadIdx.x == 0) gerr = 0;
  __syncthreads();
  CGArgs<T> b = a;
  if (a.gerr) b.err = &gerr;
  const int ib = blockIdx.x * R;
  gather_rows<T, NP, MIX, SLICED>(b, ca, ib, min(ca.mp, ib + R));
  if (a.gerr) {
    __syncthreads();
    if (threadIdx.x == 0) a.gerr[blockIdx.x] = gerr;
  }
}

// Returns the number of gather workgroups (the solver's a.ngerr).
template <typename T, int NP, bool MIX, bool SLICED>
hipError_t launch_gather(const CGArgs<T>& a, const ColArgs<T>& ca, int* ng, hipStream_t s) {
  constexpr int R = kCB * 2 / NP;
  static_assert(R >= 8, "the workspace holds one error word per 8 padded rows");
  *ng = (ca.mp + R - 1) / R;
  const int nz = a.gerr ? 1 + (int)((a.zn + 4L * kCB - 1) / (4L * kCB)) : 0;
  hipLaunchKernelGGL((k_gather<T, NP, MIX, SLICED>), dim3(*ng + nz), dim3(kCB), 0, s, a, ca, *ng);
  return hipGetLastError();
}

// Split solver: P workgroups per member (grid N * P, co-resident), each
// owning ms rows of S in LDS; one flag-in-word exchange of partial sums per
// pass; no grid-wide wait at all.
template <typename T, int NP>
__global__ __launch_bounds__(kCB) void k_cg_split(CGArgs<T> a, ColArgs<T> ca) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x, P = ca.P;
  int j, part;
  if (a.N % 8 == 0) {
    // workgroups go round-robin over the 8 XCDs: keep a member's parts on one
    const int x = b % 8, t = b / 8;
    j = x + 8 * (t / P);
    part = t % P;
  } else {
    j = b / P;
    part = b % P;
  }
  CGD_TRACE(0);
  fold_gather_errors(a);
  ColArgs<T> c = ca;
  c.part = part;
  c.r0 = part * ca.ms;
  column_phase<T, NP, false, false, true>(a, c, j, smem_raw);
}

template <typename T>
constexpr int col_np(int N) {
  return N <= 16 ? 16 : N <= 32 ? 32 : N <= 64 ? 64 : (sizeof(T) == 4 && N <= 128) ? 128 : 0;
}

// Whether the CG vectors of an m-row problem fit in LDS beside the
// reductions (the S cache then takes what is left, possibly nothing); else
// they live in global memory (GV).
template <typename T, int NP, bool MIX>
bool col_lds_vectors(int m) {
  using K = KC<T, NP, MIX>;
  const size_t p = (size_t)(m + K::RG - 1) / K::RG * K::RG;
  return sizeof(T) * 5 * p + K::fixed <= kColLdsMax;
}

template <typename T, int NP, bool MIX, bool GV>
size_t col_lds(int mp, int RL) {
  using K = KC<T, NP, MIX>;
  const size_t cg =
      (GV ? 0 : sizeof(T) * 5 * (size_t)mp) + K::fixed + (size_t)K::SE * RL * NP;
  return cg > UCfg<T, NP>::lds ? cg : UCfg<T, NP>::lds;
}

template <typename T, int NP, bool MIX, bool GV>
void col_shape(int m, int* mp, int* RL) {
  using K = KC<T, NP, MIX>;
  const int p = (m + K::RG - 1) / K::RG * K::RG;
  const size_t base = (GV ? 0 : sizeof(T) * 5 * (size_t)p) + K::fixed;
  long rl = 0;
  if (base < kColLdsMax) rl = (long)((kColLdsMax - base) / ((size_t)K::SE * NP));
  rl = rl / K::RG * K::RG;
  if (rl > p) rl = p;
  *mp = p;
  *RL = (int)rl;
}

template <typename T, int NP, bool MIX, bool GV>
hipError_t launch_np(const CGArgs<T>& a, const ColArgs<T>& vec, hipEvent_t* ev, hipStream_t s) {
  ColArgs<T> ca = vec;
  ca.Dt = a.D;
  col_shape<T, NP, MIX, GV>(a.m, &ca.mp, &ca.RL);
  if (!GV) ca.Rp = nullptr;
  CGArgs<T> a2 = a;
  hipError_t e = launch_gather<T, NP, MIX, false>(a, ca, &a2.ngerr, s);
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;  // the solver launch alone
  const size_t sh = col_lds<T, NP, MIX, GV>(ca.mp, ca.RL);
  auto fn = k_cg_columns<T, NP, MIX, GV>;
  e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  // the workgroups wait for each other's published W before the update:
  // either a cooperative launch (the runtime makes all of them resident or
  // refuses) or a plain one whose start-up census fails fast
  if (!a2.census) {
    void* args[] = {(void*)&a2, (void*)&ca};
    return hipLaunchCooperativeKernel((const void*)fn, dim3(a.N), dim3(kCB), args, (unsigned)sh,
                                      s);
  }
  hipLaunchKernelGGL(fn, dim3(a.N), dim3(kCB), sh, s, a2, ca);
  return hipGetLastError();
}

// Co-resident workgroups of kernel fn (kCB threads, sh bytes of dynamic LDS)
// on the current device, cached per (kernel, device, LDS size) so that the
// per-call solver choice makes no runtime queries after the first.
int kernel_coresident(const void* fn, size_t sh) {
  struct Entry {
    const void* fn;
    int dev;
    size_t sh;
    int value;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry& e : cache)
      if (e.fn == fn && e.dev == dev && e.sh == sh) return e.value;
  }
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess)
    return 0;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kCB, sh) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  std::lock_guard<std::mutex> lock(mu);
  cache.push_back({fn, dev, sh, per_cu * cus});
  return per_cu * cus;
}

template <typename T, int NP, bool MIX>
int coresident_np(int m) {
  int mp, RL;
  size_t sh;
  const void* fn;
  if (col_lds_vectors<T, NP, MIX>(m)) {
    col_shape<T, NP, MIX, false>(m, &mp, &RL);
    sh = col_lds<T, NP, MIX, false>(mp, RL);
    fn = (const void*)k_cg_columns<T, NP, MIX, false>;
  } else {
    col_shape<T, NP, MIX, true>(m, &mp, &RL);
    sh = col_lds<T, NP, MIX, true>(mp, RL);
    fn = (const void*)k_cg_columns<T, NP, MIX, true>;
  }
  if (sh > kColLdsMax) return 0;
  return kernel_coresident(fn, sh);
}

// Padded rows of the column solver for (m, np); *gv: vectors in global memory.
template <typename T, bool MIX>
void shape_mix(int m, int np, int* mp, int* gv) {
  int rl = 0;
  auto one = [&](auto npc) {
    constexpr int NP = decltype(npc)::value;
    *gv = !col_lds_vectors<T, NP, MIX>(m);
    if (*gv) col_shape<T, NP, MIX, true>(m, mp, &rl);
    else col_shape<T, NP, MIX, false>(m, mp, &rl);
  };
  if (np == 16) one(std::integral_constant<int, 16>{});
  else if (np == 32) one(std::integral_constant<int, 32>{});
  else if (np == 64) one(std::integral_constant<int, 64>{});
  else if constexpr (sizeof(T) == 4) one(std::integral_constant<int, 128>{});
}

template <typename T, bool MIX>
int coresident_mix(int m, int np) {
  if (np == 16) return coresident_np<T, 16, MIX>(m);
  if (np == 32) return coresident_np<T, 32, MIX>(m);
  if (np == 64) return coresident_np<T, 64, MIX>(m);
  if constexpr (sizeof(T) == 4)
    if (np == 128) return coresident_np<T, 128, MIX>(m);
  return 0;
}

template <typename T, bool MIX>
hipError_t launch_mix(const CGArgs<T>& a, const ColArgs<T>& vec, hipEvent_t* ev, hipStream_t s) {
  const int np = col_np<T>(a.N);
  const bool gv = vec.Vz != nullptr;
  auto one = [&](auto npc) {
    constexpr int NP = decltype(npc)::value;
    return gv ? launch_np<T, NP, MIX, true>(a, vec, ev, s)
              : launch_np<T, NP, MIX, false>(a, vec, ev, s);
  };
  if (np == 16) return one(std::integral_constant<int, 16>{});
  if (np == 32) return one(std::integral_constant<int, 32>{});
  if (np == 64) return one(std::integral_constant<int, 64>{});
  if constexpr (sizeof(T) == 4)
    if (np == 128) return one(std::integral_constant<int, 128>{});
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Batched mode: many independent problems, each solved as above (the same
// per-member recurrence, stop rule and update), in three launches over work
// tables, so no workgroup ever waits for another:
//   gather  one entry per (problem, block of P.gr padded rows);
//   solve   one entry per (problem, member), all members of a problem on one
//           XCD (entries w with w % 8 equal, padding entries -1), problems in
//           decreasing order of work so the longest start first, CG vectors
//           in global memory;
//   update  one entry per (problem, block of P.ur state rows).
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline CGArgs<T> batch_args(const BProb<T>& P, int* err) {
  CGArgs<T> a = {};
  a.n = P.n;
  a.m = P.m;
  a.N = P.N;
  a.k = P.k;
  a.Xf = P.Xf;
  a.Xa = P.Xa;
  a.Xg = P.Xf;
  a.ng = P.n;
  a.idx = P.idx;
  a.hw = P.hw;
  a.y = P.y;
  a.rdiag = P.rdiag;
  a.eps = P.eps;
  a.err = err;
  a.Wd = P.Wd;
  a.col = P.col;
  a.coli = P.coli;
  a.iters_out = P.iters_out;
  return a;
}

template <typename T>
__device__ inline ColArgs<T> batch_cols(const BProb<T>& P) {
  ColArgs<T> ca = {};
  ca.Sp = P.Sp;
  ca.Dt = P.Dt;
  ca.mp = P.mp;
  ca.RL = P.RL;
  ca.Vz = P.Vz;
  ca.Vr = P.Vr;
  ca.Vp = P.Vp;
  ca.Rp = P.Rp;
  return ca;
}

template <typename T>
__global__ __launch_bounds__(kCB) void k_bcol_gather(const BProb<T>* probs, const int2* tab,
                                                     int* err, int precond) {
  const int2 ent = tab[blockIdx.x];
  const BProb<T> P = probs[ent.x];
  CGArgs<T> a = batch_args(P, err);
  a.precond = precond;
  const ColArgs<T> ca = batch_cols(P);
  const int ie = min(P.mp, ent.y + P.gr);
  switch (P.NP) {
    case 16: gather_rows<T, 16, false>(a, ca, ent.y, ie); break;
    case 32: gather_rows<T, 32, false>(a, ca, ent.y, ie); break;
    default: gather_rows<T, 64, false>(a, ca, ent.y, ie); break;
  }
}

template <typename T>
__global__ __launch_bounds__(kCB) void k_bcol_solve(const BProb<T>* probs, const int2* tab,
                                                    double tol, int maxit, int* err,
                                                    int precond) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int2 ent = tab[blockIdx.x];
  if (ent.x < 0) return;  // padding of an XCD queue
  const BProb<T> P = probs[ent.x];
  CGArgs<T> a = batch_args(P, err);
  a.tol = tol;
  a.maxit = maxit;
  a.precond = precond;
  const ColArgs<T> ca = batch_cols(P);
  switch (P.NP) {
    case 16: column_phase<T, 16, false, true, false, false>(a, ca, ent.y, smem_raw); break;
    case 32: column_phase<T, 32, false, true, false, false>(a, ca, ent.y, smem_raw); break;
    default: column_phase<T, 64, false, true, false, false>(a, ca, ent.y, smem_raw); break;
  }
}

template <typename T, int NP>
__device__ void batch_update_rows(const BProb<T>& P, int i0, unsigned char* smem_raw) {
  using U = UCfg<T, NP>;
  T* As = (T*)smem_raw;
  T* Wt = As + (size_t)U::RBX * U::LD;
  double* mean = (double*)(Wt + (size_t)NP * U::LD);
  update_load_w<T, NP, kCB>(P.N, P.Wd, 0, Wt);
  const int ie = min(P.n, i0 + P.ur);
  for (int r0 = i0; r0 < ie; r0 += U::RBX)
    update_tile<T, NP, kCB>(P.n, P.N, P.Xf, P.Xa, 0, r0, As, Wt, mean);
}

template <typename T>
__global__ __launch_bounds__(kCB) void k_bcol_update(const BProb<T>* probs, const int2* tab) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int2 ent = tab[blockIdx.x];
  const BProb<T> P = probs[ent.x];
  switch (P.NP) {
    case 16: batch_update_rows<T, 16>(P, ent.y, smem_raw); break;
    case 32: batch_update_rows<T, 32>(P, ent.y, smem_raw); break;
    default: batch_update_rows<T, 64>(P, ent.y, smem_raw); break;
  }
}

template <typename T, int NP>
void batch_shape_np(int m, int* mp, int* RL) {
  using K = KC<T, NP, false>;
  const int p = (m + K::RG - 1) / K::RG * K::RG;
  long rl = (long)((kColLdsMax - K::fixed) / ((size_t)K::SE * NP));
  rl = rl / K::RG * K::RG;
  if (rl > p) rl = p;
  *mp = p;
  *RL = (int)rl;
}

template <typename T, int NP>
size_t split_lds(int ms, int P) {
  using K = KC<T, NP, false>;
  const size_t cg = sizeof(T) * 5 * (size_t)ms + K::fixed + sizeof(T) * (size_t)ms * NP +
                    sizeof(unsigned) * (size_t)P * XC<NP>::XW;
  return cg > UCfg<T, NP>::lds ? cg : UCfg<T, NP>::lds;
}

// Smallest P >= 2 whose row slices (ms rows, a multiple of the row step)
// fit the LDS with the slice of S; 0 if none up to kMaxSplitParts.
template <typename T, int NP>
int split_shape_np(int m, int* P, int* ms) {
  using K = KC<T, NP, false>;
  for (int p = 2; p <= kMaxSplitParts; ++p) {
    const int rows = (m + p - 1) / p;
    const int s = (rows + K::RG - 1) / K::RG * K::RG;
    if (split_lds<T, NP>(s, p) <= kColLdsMax) {
      *P = p;
      *ms = s;
      return 1;
    }
  }
  return 0;
}

template <typename T, int NP>
int split_coresident_np(int ms, int P) {
  return kernel_coresident((const void*)k_cg_split<T, NP>, split_lds<T, NP>(ms, P));
}

template <typename T, int NP>
hipError_t launch_split_np(const CGArgs<T>& a, int P, int ms, T* Sg, T* Dg,
                           unsigned long long* xb, unsigned long long* wb, hipEvent_t* ev,
                           hipStream_t s) {
  ColArgs<T> ca = {};
  ca.Sp = Sg;
  ca.Dt = Dg;
  ca.mp = P * ms;
  ca.RL = ms;
  ca.P = P;
  ca.ms = ms;
  ca.xb = xb;
  ca.wb = wb;
  CGArgs<T> a2 = a;
  hipError_t e = launch_gather<T, NP, false, true>(a, ca, &a2.ngerr, s);
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;  // the solver launch alone
  const size_t sh = split_lds<T, NP>(ms, P);
  auto fn = k_cg_split<T, NP>;
  e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  // a member's workgroups exchange partial sums every pass: either a
  // cooperative launch (the runtime makes all N * P resident or refuses) or
  // a plain one whose start-up census fails fast
  if (!a2.census) {
    void* args[] = {(void*)&a2, (void*)&ca};
    return hipLaunchCooperativeKernel((const void*)fn, dim3(a.N * P), dim3(kCB), args,
                                      (unsigned)sh, s);
  }
  hipLaunchKernelGGL(fn, dim3(a.N * P), dim3(kCB), sh, s, a2, ca);
  return hipGetLastError();
}

}  // namespace

// Column solver geometry for the workspace: padded rows and padded N, or 0
// when the column solver does not apply to (m, N, prec).  mix selects the
// mixed-precision variant (FP32 data, BF16 copy of S).
template <typename T>
int columns_shape(int m, int N, int mix, int* mp, int* NPc, int* gv) {
  const int np = col_np<T>(N);
  if (np == 0 || m > kColumnsMaxRows) return 0;
  if constexpr (sizeof(T) == 4) {
    if (mix) shape_mix<T, true>(m, np, mp, gv);
    else shape_mix<T, false>(m, np, mp, gv);
  } else {
    if (mix) return 0;  // the mixed mode takes FP32 data
    shape_mix<T, false>(m, np, mp, gv);
  }
  *NPc = np;
  return 1;
}

template <typename T>
int columns_coresident(int m, int N, int mix) {
  const int np = col_np<T>(N);
  if constexpr (sizeof(T) == 4)
    return mix ? coresident_mix<T, true>(m, np) : coresident_mix<T, false>(m, np);
  else
    return mix ? 0 : coresident_mix<T, false>(m, np);
}


template <typename T>
hipError_t launch_cg_columns(const CGArgs<T>& a, T* Sp, __bf16* Sh, unsigned long long* wb,
                             T* Vz, T* Vr, T* Vp, T* Rp, hipEvent_t* ev, hipStream_t s) {
  ColArgs<T> vec = {};  // unused fields must be null
  vec.Sp = Sp;
  vec.Sh = Sh;
  vec.wb = wb;
  vec.Vz = Vz;
  vec.Vr = Vr;
  vec.Vp = Vp;
  vec.Rp = Rp;
  if (Sh) {
    if constexpr (sizeof(T) == 4) return launch_mix<T, true>(a, vec, ev, s);
    return hipErrorInvalidValue;
  }
  return launch_mix<T, false>(a, vec, ev, s);
}

template <typename T>
int batched_shape(int m, int N, int* NP, int* mp, int* RL) {
  const int np = col_np<T>(N);
  if (N < 2 || np == 0) return 0;
  *NP = np;
  if (np == 16) batch_shape_np<T, 16>(m, mp, RL);
  else if (np == 32) batch_shape_np<T, 32>(m, mp, RL);
  else batch_shape_np<T, 64>(m, mp, RL);
  return 1;
}

template <typename T>
hipError_t launch_batched(const BProb<T>* probs, const int2* gtab, int ngather,
                          const int2* stab, int nsolve, const int2* utab, int nupdate,
                          double tol, int maxit, int precond, int* err, hipEvent_t* ev,
                          hipStream_t s) {
  hipError_t e;
  hipLaunchKernelGGL(k_bcol_gather<T>, dim3(ngather), dim3(kCB), 0, s, probs, gtab, err,
                     precond);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // profiling events bracket the CG launch alone
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
  const size_t sh = kColLdsMax;
  if ((e = hipFuncSetAttribute((const void*)k_bcol_solve<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_bcol_solve<T>, dim3(nsolve), dim3(kCB), sh, s, probs, stab, tol, maxit,
                     err, precond);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  const size_t shu = UCfg<T, 64>::lds;
  hipLaunchKernelGGL(k_bcol_update<T>, dim3(nupdate), dim3(kCB), shu, s, probs, utab);
  return hipGetLastError();
}

template <typename T>
int split_shape(int m, int N, int* P, int* ms) {
  const int np = col_np<T>(N);
  if (N < 2) return 0;
  if (np == 16) return split_shape_np<T, 16>(m, P, ms);
  if (np == 32) return split_shape_np<T, 32>(m, P, ms);
  if (np == 64) return split_shape_np<T, 64>(m, P, ms);
  return 0;
}

template <typename T>
int split_coresident(int N, int P, int ms) {
  const int np = col_np<T>(N);
  if (np == 16) return split_coresident_np<T, 16>(ms, P);
  if (np == 32) return split_coresident_np<T, 32>(ms, P);
  if (np == 64) return split_coresident_np<T, 64>(ms, P);
  return 0;
}

size_t split_exchange_words(int N, int P) {
  const int xw = N <= 16 ? XC<16>::XW : N <= 32 ? XC<32>::XW : XC<64>::XW;
  return (size_t)N * 2 * P * xw;
}

template <typename T>
hipError_t launch_cg_split(const CGArgs<T>& a, int P, int ms, T* Sg, T* Dg,
                           unsigned long long* xb, unsigned long long* wb, hipEvent_t* ev,
                           hipStream_t s) {
  const int np = col_np<T>(a.N);
  if (np == 16) return launch_split_np<T, 16>(a, P, ms, Sg, Dg, xb, wb, ev, s);
  if (np == 32) return launch_split_np<T, 32>(a, P, ms, Sg, Dg, xb, wb, ev, s);
  return launch_split_np<T, 64>(a, P, ms, Sg, Dg, xb, wb, ev, s);
}

template <typename T>
size_t columns_streamed_bytes(int m, int N) {
  int mp = 0, RL = 0;
  auto one = [&](auto npc) {
    constexpr int NP = decltype(npc)::value;
    if (col_lds_vectors<T, NP, false>(m)) col_shape<T, NP, false, false>(m, &mp, &RL);
    else col_shape<T, NP, false, true>(m, &mp, &RL);
  };
  const int np = col_np<T>(N);
  if (np == 16) one(std::integral_constant<int, 16>{});
  else if (np == 32) one(std::integral_constant<int, 32>{});
  else if (np == 64) one(std::integral_constant<int, 64>{});
  else return 0;
  return sizeof(T) * (size_t)(mp - RL) * np;
}

template int split_shape<float>(int, int, int*, int*);
template int split_shape<double>(int, int, int*, int*);
template int split_coresident<float>(int, int, int);
template int split_coresident<double>(int, int, int);
template hipError_t launch_cg_split<float>(const CGArgs<float>&, int, int, float*, float*,
                                           unsigned long long*, unsigned long long*, hipEvent_t*,
                                           hipStream_t);
template hipError_t launch_cg_split<double>(const CGArgs<double>&, int, int, double*, double*,
                                            unsigned long long*, unsigned long long*, hipEvent_t*,
                                            hipStream_t);
template size_t columns_streamed_bytes<float>(int, int);
template size_t columns_streamed_bytes<double>(int, int);

template int columns_shape<float>(int, int, int, int*, int*, int*);
template int columns_shape<double>(int, int, int, int*, int*, int*);
template int columns_coresident<float>(int, int, int);
template int columns_coresident<double>(int, int, int);
template hipError_t launch_cg_columns<float>(const CGArgs<float>&, float*, __bf16*,
                                             unsigned long long*, float*, float*, float*, float*,
                                             hipEvent_t*, hipStream_t);
template int batched_shape<float>(int, int, int*, int*, int*);
template int batched_shape<double>(int, int, int*, int*, int*);
template hipError_t launch_batched<float>(const BProb<float>*, const int2*, int, const int2*, int,
                                          const int2*, int, double, int, int, int*, hipEvent_t*,
                                          hipStream_t);
template hipError_t launch_batched<double>(const BProb<double>*, const int2*, int, const int2*,
                                           int, const int2*, int, double, int, int, int*,
                                           hipEvent_t*, hipStream_t);
template hipError_t launch_cg_columns<double>(const CGArgs<double>&, double*, __bf16*,
                                              unsigned long long*, double*, double*, double*,
                                              double*, hipEvent_t*, hipStream_t);

}  // namespace cgd
