// Row-block x member-group CG solver of the CGD-EnKF analysis (gfx950, FP32
// storage, products on MFMA).
//
// The N recurrences of the per-member CG (Algorithm 1) are independent; they
// share only the products with S of Section 3.3, Psi p = S (S^T p)/(N-1) + R p.
// This solver splits the members into groups of 32 and the observation rows
// into blocks of RB rows.  Workgroup (c, b) holds, for the whole solve:
//
//  * rows [b RB, b RB + RB) of S for all N members, in LDS (a gather
//    launch ahead of the solver forms S, D and the rows' diag(R) once);
//  * z, r and p of group c's 32 members on those rows, in registers, laid
//    out as the accumulators of the 16x16x4 MFMA that forms S_b G.
//
// Four waves: wave w takes the 16 members 16 (w & 1) .. of the group on the
// half (w >> 1) of the rows.  Both contractions run on v_mfma_f32_16x16x4f32.
// The summation index of each product is permuted so that every operand
// comes from a contiguous LDS read or straight from the lane's registers:
//
//  * Q = S_b G takes S rows as the A operand (16-byte reads) and G from
//    registers, where every lane keeps the rows of G that it supplies;
//  * the partial S_b^T r takes S columns as A and the lane's own r as B.
//
// An iteration needs one sum over the row blocks of a group: S^T r (NP x 32)
// and four scalar sums per member.  Those are r^T r, r^T R r, r^T R p and
// p^T R p, the single-reduction form of the recurrence that the other
// solvers use.  The sum is a reduce-scatter followed by an all-gather,
// through exchange words that carry their exchange number in the upper 32
// bits ("flag in the word"), so it needs no fence or cache maintenance:
//
//  1. each workgroup publishes its partial;
//  2. it sums its 1/nblk slice of all the group's partials, in a fixed
//     order, and publishes that slice;
//  3. it gathers the whole sum.
//
// The scalar sums are formed in double and travel as pairs of float words
// (hi + lo, about 48 bits), summed in double.  Every workgroup of a group
// then takes the same decisions (alpha, beta, convergence) from bitwise the
// same sums. No other state is shared, and
// groups never wait for each other.  Every wait is bounded (1 s): one that
// runs out sets bit 0 of *err.
//
// After the loop, W = S^T Z/(N-1) is formed from FP64 products (widened
// operands, v_mfma_f64_16x16x4f64) and summed the same way (float pairs).  With
// statistics, the true residual d - Psi z of every member follows, in
// double.
#include <type_traits>

#include "exchange.h"
#include "internal.h"
#include "mfma_util.h"

namespace cgd {

namespace {

constexpr int kTW = 32;  // members per group

template <int NP, int RB>
struct TC {
  static_assert(NP % 64 == 0 && RB % 32 == 0, "tile shape");
  static constexpr int LDS = NP + 4;          // S row stride in floats (16-byte rows, skewed banks)
  static constexpr int RT = RB / 32;          // 16-row tiles per wave
  static constexpr int KT = NP / 16;          // 16-row tiles of S^T r = 16-wide chunks of S G
  static constexpr int EG = NP * kTW;         // float words of an exchange (S^T r)
  static constexpr int ND = 4 * kTW;          // doubles of an exchange (four per member)
  static constexpr int E = EG + 2 * ND;       // words of an exchange
  static constexpr int EW = 2 * NP * kTW;     // S^T Z in double, two words per value
  static constexpr int SLOT = (2 * E > EW) ? 2 * E : EW;  // words per workgroup
  static constexpr int SLOTR = 2 * E + EW;                // reduced words per group
  static constexpr int CPC = NP / 16;         // members per thread in the gather
};

template <int NP, int RB>
struct __align__(16) TLds {
  using C = TC<NP, RB>;
  float S[RB * C::LDS];
  // lane rows padded by 16 bytes so that lanes 16 apart in a 16-byte access
  // fall on different banks
  union {
    float xg[2][2][64][C::KT * 2 + 4];  // halves of S^T r swapped by the two waves of a tile
    double xw[64][C::KT * 4 + 2];       // the same for S^T Z, one member tile at a time
  };
  float rv[RB];                   // diag(R) of the rows (1 when preconditioned)
  double xs[2][16][4];            // scalar sums of the second wave of each member tile
  double own[kBlock];             // owner step: sums per thread row
  double dnl[kTW];                // ||d_j||^2 of the group's members
};

// The solver's own arguments (a compact copy of the fields of CGArgs it
// uses: fewer scalar registers than the whole struct).
struct TileArgs {
  int N, m, NG, nblk, maxit, want_relres;
  double tol;
  unsigned long long* txp;   // partial exchange words, NG * nblk * SLOT
  unsigned long long* txr;   // reduced exchange words, NG * SLOTR
  const float* S;            // m x NP from the gather launch
  const float* rv;           // m
  const float* D;            // m x N
  float* z_out;
  int* iters_out;
  double* relres_out;
  double* relres;
  int* coli;
  double* col;
  double* Wd;
  int* err;
  unsigned long long* census;
  unsigned long long census_ticks;
  unsigned long long* trace;
};

__device__ inline unsigned long long ld64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st64(unsigned long long* p, unsigned v, unsigned ep) {
  __hip_atomic_store(p, (unsigned long long)v | ((unsigned long long)ep << 32), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
// A wait for an exchange word gives up after this many ticks of the 100 MHz
// real-time counter (1 s; a healthy wait is a few microseconds, or the
// slowest workgroup's gather at the start).
constexpr unsigned long long kTileWaitTicks = 100000000ull;

// Re-reads *p until its exchange number is ep (w: the first read); a wait
// that runs out sets bad, and once bad is set no wait starts.
__device__ inline unsigned long long poll64(const unsigned long long* p, unsigned ep,
                                            unsigned long long w, bool& bad) {
  if ((unsigned)(w >> 32) == ep || bad) return w;
  const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    w = ld64(p);
    if ((unsigned)(w >> 32) == ep) break;
    if (__builtin_amdgcn_s_memrealtime() - t0 > kTileWaitTicks) {
      bad = true;
      break;
    }
  }
  return w;
}
// Waits until every word w[u], u < n (first reads of at(u)), carries exchange
// number ep, re-reading all stale words together in each round: one memory
// round trip per round, however many words are late.  A wait that runs out
// sets bad, and once bad is set no wait starts.
template <int NMAX, typename At>
__device__ __attribute__((always_inline)) void poll_all(unsigned long long (&w)[NMAX], int n, At at,
                                                        unsigned ep, bool& bad) {
  unsigned long long t0 = 0;
  for (;;) {
    bool stale = false;
#pragma unroll
    for (int u = 0; u < NMAX; ++u) stale |= u < n && (unsigned)(w[u] >> 32) != ep;
    if (!stale || bad) return;
    const unsigned long long now = __builtin_amdgcn_s_memrealtime();
    if (t0 == 0) {
      t0 = now;
    } else if (now - t0 > kTileWaitTicks) {
      bad = true;
      return;
    }
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int u = 0; u < NMAX; ++u)
      if (u < n && (unsigned)(w[u] >> 32) != ep) w[u] = ld64(at(u));
  }
}

// A double travels as two float words (hi = float(v), lo = float(v - hi)),
// each a number, so partial sums add word by word; v is carried to about
// 2^-48 relative.
__device__ inline double pair2(unsigned long long hi, unsigned long long lo) {
  return (double)__uint_as_float((unsigned)hi) + (double)__uint_as_float((unsigned)lo);
}
__device__ inline void st_pair(unsigned long long* p, double v, unsigned ep) {
  const float hi = (float)v;
  const float lo = (float)(v - (double)hi);
  st64(p, __float_as_uint(hi), ep);
  st64(p + 1, __float_as_uint(lo), ep);
}

// Owner step of a reduce-scatter: sums this workgroup's slice over the nblk
// partials of its group (partial q at base + q * stride): float items
// [glo, glo + Lg) and float-pair items (doubles) [dlo, dlo + Ld) at word
// doff + 2 d.  Every word of a chunk gets kBlock / (words) threads, each
// summing a fixed range of the partials (up to kBatch loads in flight);
// the ranges are then added in order, so the result does not depend on
// timing.  emitf(x, total) and emitd(d, total) run in one thread per item,
// with x and d the item's index in the whole exchange (glo + ..., dlo + ...).
// Returns false when a wait ran out.
constexpr int kBatch = 24;

template <typename EmitF, typename EmitD>
__device__ __attribute__((always_inline)) bool owner_sum(const unsigned long long* base, size_t stride, int nblk, unsigned ep,
                          int glo, int Lg, int doff, int dlo, int Ld, double* own, EmitF emitf,
                          EmitD emitd) {
  const int tid = threadIdx.x;
  bool bad = false;
  // first wait for one word of each partial (the slice's first), one thread
  // per partial, so that the bulk loads below rarely meet a stale word and
  // few loads poll the memory system meanwhile
  {
    const unsigned long long* p0 = Lg > 0 ? base + glo : base + doff + 2 * dlo;
    for (int q = tid; q < nblk && Lg + Ld > 0; q += kBlock)
      poll64(p0 + (size_t)q * stride, ep, ld64(p0 + (size_t)q * stride), bad);
    if (__syncthreads_or(bad)) return false;
  }
  int f0 = 0, d0 = 0;
  while (f0 < Lg || d0 < Ld) {
    // this chunk: nf float items and nd pairs, nf + 2 nd <= kBlock words
    const int nf = min(Lg - f0, kBlock);
    const int nd = min(Ld - d0, (kBlock - nf) / 2);
    // consecutive threads take consecutive words (coalesced), thread row
    // sub the sub-th range of the partials
    const int W = nf + 2 * nd, R = kBlock / W;
    const int sub = tid / W, x = tid - sub * W;
    double s = 0.0;
    if (sub < R) {
      const unsigned long long* p =
          x < nf ? base + glo + f0 + x : base + doff + 2 * (dlo + d0) + (x - nf);
      const int q0 = sub * nblk / R, q1 = (sub + 1) * nblk / R;
      for (int q = q0; q < q1; q += kBatch) {
        unsigned long long w[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
          if (q + u < q1) w[u] = ld64(p + (size_t)(q + u) * stride);
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
          if (q + u < q1) {
            w[u] = poll64(p + (size_t)(q + u) * stride, ep, w[u], bad);
            s += (double)__uint_as_float((unsigned)w[u]);
          }
      }
    }
    own[tid] = s;
    if (__syncthreads_or(bad)) return false;
    if (tid < nf) {
      double tot = 0.0;
      for (int k = 0; k < R; ++k) tot += own[k * W + tid];
      emitf(glo + f0 + tid, tot);
    } else if (tid < nf + nd) {
      const int d = tid - nf, wh = nf + 2 * d;
      double th = 0.0, tl = 0.0;
      for (int k = 0; k < R; ++k) th += own[k * W + wh];
      for (int k = 0; k < R; ++k) tl += own[k * W + wh + 1];
      emitd(dlo + d0 + d, th + tl);
    }
    __syncthreads();
    f0 += nf;
    d0 += nd;
  }
  return true;
}

// TR: the diagnostic variant that stores phase timestamps to a.trace (the
// plain variant has no trace code, which keeps it free of register spills).
// TR: the diagnostic variant.  Thread 0 of every workgroup keeps 256
// timestamps of the 100 MHz counter in LDS; workgroup 0 copies them to
// a.trace when it leaves.  The plain variant has no trace code at all.
template <bool TR>
__device__ inline unsigned long long* tile_trace_buf() {
  if constexpr (TR) {
    __shared__ unsigned long long buf[256];
    return buf;
  } else {
    return nullptr;
  }
}
#define TTRACE(slot)                                                        \
  do {                                                                      \
    if constexpr (TR)                                                       \
      if (threadIdx.x == 0) trb[(slot)&255] = __builtin_amdgcn_s_memrealtime(); \
  } while (0)

template <int NP, int RB, bool TR>
__global__ __launch_bounds__(kBlock) void k_cg_tile(TileArgs a) {
  // the arguments as plain locals (the lambdas below capture these, not a)
  const float* const ta_D = a.D;
  int const ta_N = a.N;
  int const ta_NG = a.NG;
  const float* const ta_S = a.S;
  double* const ta_Wd = a.Wd;
  unsigned long long* const ta_census = a.census;
  unsigned long long const ta_census_ticks = a.census_ticks;
  double* const ta_col = a.col;
  int* const ta_coli = a.coli;
  int* const ta_err = a.err;
  int* const ta_iters_out = a.iters_out;
  int const ta_m = a.m;
  int const ta_maxit = a.maxit;
  int const ta_nblk = a.nblk;
  double* const ta_relres = a.relres;
  double* const ta_relres_out = a.relres_out;
  const float* const ta_rv = a.rv;
  double const ta_tol = a.tol;
  unsigned long long* const ta_trace = a.trace;
  unsigned long long* const ta_txp = a.txp;
  unsigned long long* const ta_txr = a.txr;
  int const ta_want_relres = a.want_relres;
  float* const ta_z_out = a.z_out;
  using C = TC<NP, RB>;
  using LdsT = TLds<NP, RB>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LdsT& L = *reinterpret_cast<LdsT*>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int cw = wv & 1, h = wv >> 1;
  const int NG = ta_NG, nblk = ta_nblk;
  const int c = blockIdx.x % NG, b = blockIdx.x / NG;
  const int N = ta_N, m = ta_m;
  const int i0 = b * RB;
  const int n = cw * 16 + lr;  // this lane's member within the group ...
  const int j = c * kTW + n;   // ... and in the ensemble
  const bool jv = j < N;
  const int hb = h * (RB / 2);  // first row of this wave's half of the block
  const float inv = (float)(1.0 / (double)(N - 1));
  unsigned long long* mypart = ta_txp + (size_t)(c * nblk + b) * C::SLOT;
  const unsigned long long* gpart = ta_txp + (size_t)c * nblk * C::SLOT;
  unsigned long long* red = ta_txr + (size_t)c * C::SLOTR;
  // this workgroup's slice of the exchanges: float words and doubles
  const int glo = b * C::EG / nblk, Lg = (b + 1) * C::EG / nblk - glo;
  const int dlo = b * C::ND / nblk, Ld = (b + 1) * C::ND / nblk - dlo;
  // a plain launch's start-up census: check in now, wait before the first
  // exchange (the gather needs no other workgroup)
  unsigned long long census_count = 0;
  if (ta_census && tid == 0) census_count = census_arrive(ta_census);
  unsigned long long* const trb = tile_trace_buf<TR>();
  if constexpr (TR) {
    for (int e = tid; e < 256; e += kBlock) trb[e] = 0ull;
    __syncthreads();
  }
  TTRACE(0);
  // leaves the kernel (every exit is uniform across the workgroup)
  auto finish = [&]() __attribute__((always_inline)) {
    if constexpr (TR) {
      __syncthreads();
      if (b == 0 && c == 0 && ta_trace)
        for (int e = tid; e < 256; e += kBlock)
          if (trb[e]) ta_trace[e] = trb[e];
    }
  };

  // ---------------- S block and the rows' diag(R), from the gather launch ----------------
  for (int e = tid; e < RB * NP / 4; e += kBlock) {
    const int i = e / (NP / 4), c4 = (e - i * (NP / 4)) * 4, gi = i0 + i;
    v4f x = v4f{0.f, 0.f, 0.f, 0.f};
    if (gi < m) x = *reinterpret_cast<const v4f*>(ta_S + (size_t)gi * NP + c4);
    *reinterpret_cast<v4f*>(&L.S[i * C::LDS + c4]) = x;
  }
  for (int i = tid; i < RB; i += kBlock) L.rv[i] = (i0 + i < m) ? ta_rv[i0 + i] : 0.f;
  __syncthreads();

  // ---------------- column state: r = d, z = p = 0 ----------------
  float z[C::RT][4], r[C::RT][4], p[C::RT][4];
#pragma unroll
  for (int t = 0; t < C::RT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int gi = i0 + hb + t * 16 + 4 * lg + i;
      r[t][i] = (gi < m && jv) ? ta_D[(size_t)gi * N + j] : 0.f;
      z[t][i] = 0.f;
      p[t][i] = 0.f;
    }

  // partial S_b^T r over this wave's rows (B operand: the lane's own r)
  // Output tile 4 kq + e holds the Gram rows 64 kq + 4 m + e (m = 0..15), so
  // that one 16-byte read of S row "row" at columns 64 kq + 4 lr .. feeds
  // the four tiles of kq: accumulator i of tile 4 kq + e in lane group lg is
  // Gram row gram_row(kq, e, lg, i) below.
  auto gram_partial = [&](v4f (&g)[C::KT]) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < C::KT; ++k) g[k] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < C::RT; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float* srow = &L.S[(hb + t * 16 + 4 * lg + u) * C::LDS + 4 * lr];
        const float bv = r[t][u];
#pragma unroll
        for (int kq = 0; kq < C::KT / 4; ++kq) {
          const v4f av = *reinterpret_cast<const v4f*>(srow + 64 * kq);
#pragma unroll
          for (int e = 0; e < 4; ++e) g[4 * kq + e] = mfma4(av[e], bv, g[4 * kq + e]);
        }
      }
  };
  auto gram_row = [](int k, int lgi, int i) { return 64 * (k >> 2) + 16 * lgi + 4 * i + (k & 3); };
  // Sums over the member tile's rows: the four lane groups, then the two
  // waves (result in the waves with h == 0).
  auto tile_sums = [&](double (&v)[4]) __attribute__((always_inline)) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      v[f] += __shfl_xor(v[f], 16);
      v[f] += __shfl_xor(v[f], 32);
    }
    if (h == 1 && lg == 0)
#pragma unroll
      for (int f = 0; f < 4; ++f) L.xs[cw][lr][f] = v[f];
  };
  // The partial of exchange ep: the two waves of a member tile swap halves
  // through LDS, each publishes the sum of its half (rows 16 k.. for k in
  // [h KH, h KH + KH)), the waves with h == 0 the member sums, then every
  // workgroup runs its owner step.
  // (the half is a compile-time constant in each branch: register arrays
  // indexed by a run-time value would compile to select chains)
  auto swap_publish = [&](auto hc, unsigned ep, v4f (&g)[C::KT]) __attribute__((always_inline)) {
    constexpr int H = decltype(hc)::value, KH = C::KT / 2;
#pragma unroll
    for (int kk = 0; kk < KH; ++kk)
#pragma unroll
      for (int i = 0; i < 4; ++i) L.xg[cw][H][lane][kk * 4 + i] = g[(1 - H) * KH + kk][i];
    __syncthreads();
    unsigned long long* pp = mypart + (ep & 1) * C::E;
#pragma unroll
    for (int kk = 0; kk < KH; ++kk)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        constexpr int k0 = H * KH;
        const float x = g[k0 + kk][i] + L.xg[cw][1 - H][lane][kk * 4 + i];
        st64(pp + gram_row(k0 + kk, lg, i) * kTW + n, __float_as_uint(x), ep);
      }
  };
  auto exchange = [&](unsigned ep, v4f (&g)[C::KT], double (&v)[4], int slot) __attribute__((always_inline)) -> bool {
    if (h == 0)
      swap_publish(std::integral_constant<int, 0>{}, ep, g);
    else
      swap_publish(std::integral_constant<int, 1>{}, ep, g);
    unsigned long long* pp = mypart + (ep & 1) * C::E;
    if (h == 0 && lg == 0)
#pragma unroll
      for (int f = 0; f < 4; ++f)
        st_pair(pp + C::EG + 2 * (n * 4 + f), v[f] + L.xs[cw][lr][f], ep);
    TTRACE(slot);
    unsigned long long* rp = red + (ep & 1) * C::E;
    return owner_sum(
        gpart + (ep & 1) * C::E, C::SLOT, nblk, ep, glo, Lg, C::EG, dlo, Ld, L.own,
        [&](int x, double tot) { st64(rp + x, __float_as_uint((float)tot), ep); },
        [&](int d, double tot) { st_pair(rp + C::EG + 2 * d, tot, ep); });
  };

  // ---------------- exchange 1: S^T d, ||d||^2, d^T R d ----------------
  unsigned ep = 1;
  bool bad = false;
  {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < C::RT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double rr = r[t][i], rvv = L.rv[hb + t * 16 + 4 * lg + i];
        v[0] += rr * rr;
        v[1] += rvv * rr * rr;
      }
    tile_sums(v);
    v4f g[C::KT];
    gram_partial(g);
    if (ta_census && !census_wait(ta_census, ta_err, ta_census_ticks, census_count)) {
      finish();
      return;
    }
    bad = !exchange(ep, g, v, 255);
  }
  TTRACE(1);

  // ---------------- CG iterations ----------------
  float G[C::KT][4];  // S^T p of the previous step, rows 16k + 4 lg + u of member n
#pragma unroll
  for (int k = 0; k < C::KT; ++k)
#pragma unroll
    for (int u = 0; u < 4; ++u) G[k][u] = 0.f;
  const double tol2 = ta_tol * ta_tol;
  bool active = jv, fresh = true;
  int iters = 0, status = COL_RUNNING;
  double dn = 0.0, rhoprev = 0.0;
  for (int kit = 0; !bad; ++kit) {
    // all-gather of exchange ep: every word once per workgroup.  The two
    // waves of a member tile load half of its rows of S^T r each and swap
    // them through LDS; the lanes of lane group 0 load the member's sums and
    // pass them on to the other lane groups.
    // Every thread loads its words at once and polls them together (the
    // owners finish within about a microsecond of each other; on the
    // two-dimensional workload this beats first waiting for one word per
    // owner, which costs one more memory round trip, while the owner step
    // keeps that first wait: there, bulk polling of the slower partials
    // floods the memory system).
    const unsigned long long* rp = red + (ep & 1) * C::E;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    auto gather_half = [&](auto hc) __attribute__((always_inline)) {
      constexpr int H = decltype(hc)::value, KH = C::KT / 2, NGW = KH * 4;
      // words 0 .. NGW-1: rows 16 (H KH + kk) + 4 lg + u; then the member's 8
      // sum words (lane group 0 only)
      unsigned long long w[NGW + 8];
      auto at = [&](int u) {
        return u < NGW ? rp + (16 * (H * KH + u / 4) + 4 * lg + u % 4) * kTW + n
                       : rp + C::EG + 8 * n + (u - NGW);
      };
      const int nw = lg == 0 ? NGW + 8 : NGW;
#pragma unroll
      for (int u = 0; u < NGW + 8; ++u)
        if (u < nw) w[u] = ld64(at(u));
      poll_all(w, nw, at, ep, bad);
#pragma unroll
      for (int u = 0; u < NGW; ++u) L.xg[cw][H][lane][u] = __uint_as_float((unsigned)w[u]);
      if (lg == 0)
#pragma unroll
        for (int f = 0; f < 4; ++f) sums[f] = pair2(w[NGW + 2 * f], w[NGW + 2 * f + 1]);
    };
    if (h == 0)
      gather_half(std::integral_constant<int, 0>{});
    else
      gather_half(std::integral_constant<int, 1>{});
    if (__syncthreads_or(bad)) {
      bad = true;
      break;
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) sums[f] = __shfl(sums[f], lr);
    if (kit < 10) TTRACE(128 + 12 * kit + 0);
    const double rho = sums[0], ar = sums[1], arp = sums[2], ap = sums[3];
    if (kit == 0) dn = rho;
    // decide: converged, out of steps, or one more step with beta
    int mode = MODE_FROZEN;
    double beta = 0.0;
    if (active) {
      if (rho <= tol2 * dn) {  // ||r|| <= tol ||d||
        active = false;
        status = COL_CONVERGED;
        iters = kit;
      } else if (kit >= ta_maxit) {
        active = false;
        status = COL_MAXIT;
        iters = kit;
      } else {
        mode = MODE_STEP;
        beta = fresh ? 0.0 : rho / rhoprev;
      }
    }
    // G = S^T p for p = r + beta p (the recurrence on the sums), and p^T S S^T p.
    // Rows 16 k + 4 lg + u of S^T r come from the half its wave gathered: one
    // 16-byte read per k, outside any branch, so that all reads are in flight
    // together; frozen members take G = 0 by a select.
    // (G in FP32 FMAs, its squared norm in four FP32 partial sums: fewer
    // conversions on the step's serial path than FP64 arithmetic)
    const bool step = mode == MODE_STEP;
    const float bf = (float)beta;
    float ggp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < C::KT; ++k) {
      const v4f x = *reinterpret_cast<const v4f*>(&L.xg[cw][k / (C::KT / 2)][lane][(k % (C::KT / 2)) * 4]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float gd = beta != 0.0 ? fmaf(bf, G[k][u], x[u]) : x[u];
        const float gv = step ? gd : 0.f;
        G[k][u] = gv;
        ggp[u] = fmaf(gv, gv, ggp[u]);
      }
    }
    double gg = ((double)ggp[0] + (double)ggp[1]) + ((double)ggp[2] + (double)ggp[3]);
    gg += __shfl_xor(gg, 16);
    gg += __shfl_xor(gg, 32);
    double alpha = 0.0;
    if (mode == MODE_STEP) {
      alpha = rho / (gg / (double)(N - 1) + ar + 2.0 * beta * arp + beta * beta * ap);
      rhoprev = rho;
      fresh = false;
      if (!isfinite(alpha) || !isfinite(beta)) {
        active = false;
        status = COL_NONFINITE;
        iters = kit;
        mode = MODE_FROZEN;
        alpha = 0.0;
#pragma unroll
        for (int k = 0; k < C::KT; ++k)
#pragma unroll
          for (int u = 0; u < 4; ++u) G[k][u] = 0.f;
      }
    }
    if (!__syncthreads_or(mode == MODE_STEP)) break;  // every member of the group is done
    if (kit < 10) TTRACE(128 + 12 * kit + 1);

    // Q = S_b G over this wave's rows (A: 16-byte S reads, B: the lane's G);
    // p = r + beta p on the vector ALUs meanwhile (frozen members keep z and
    // r, with p = 0)
    const float be = (float)beta, al = (float)alpha;
    v4f qacc[C::RT];
#pragma unroll
    for (int t = 0; t < C::RT; ++t) qacc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < C::KT; ++k) {
      v4f av[C::RT];
#pragma unroll
      for (int t = 0; t < C::RT; ++t)
        av[t] = *reinterpret_cast<const v4f*>(&L.S[(hb + t * 16 + lr) * C::LDS + 16 * k + 4 * lg]);
      // consecutive MFMAs write different accumulators
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < C::RT; ++t) qacc[t] = mfma4(av[t][u], G[k][u], qacc[t]);
    }
#pragma unroll
    for (int t = 0; t < C::RT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) p[t][i] = (mode == MODE_STEP) ? r[t][i] + be * p[t][i] : 0.f;
    if (kit < 10) TTRACE(128 + 12 * kit + 2);
    // per row tile: q = Q/(N-1) + R p; z += alpha p; r -= alpha q; the next
    // sums; then the tile's part of the S^T r partial (its MFMAs overlap the
    // next tile's vector work)
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    v4f g[C::KT];
#pragma unroll
    for (int k = 0; k < C::KT; ++k) g[k] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < C::RT; ++t) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float rvv = L.rv[hb + t * 16 + 4 * lg + i];
        if (mode == MODE_STEP) {
          const float q = qacc[t][i] * inv + rvv * p[t][i];
          z[t][i] += al * p[t][i];
          r[t][i] -= al * q;
        }
        const double rr = r[t][i], pp = p[t][i];
        v[0] += rr * rr;
        v[1] += (double)rvv * rr * rr;
        v[2] += (double)rvv * rr * pp;
        v[3] += (double)rvv * pp * pp;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float* srow = &L.S[(hb + t * 16 + 4 * lg + u) * C::LDS + 4 * lr];
        const float bv = r[t][u];
#pragma unroll
        for (int kq = 0; kq < C::KT / 4; ++kq) {
          const v4f sv = *reinterpret_cast<const v4f*>(srow + 64 * kq);
#pragma unroll
          for (int e = 0; e < 4; ++e) g[4 * kq + e] = mfma4(sv[e], bv, g[4 * kq + e]);
        }
      }
    }
    tile_sums(v);
    if (kit < 10) TTRACE(128 + 12 * kit + 3);
    ++ep;
    bad = !exchange(ep, g, v, kit < 10 ? 128 + 12 * kit + 5 : 255);
    if (kit < 10) TTRACE(128 + 12 * kit + 4);
  }
  TTRACE(250);
  if (bad) {
    if (tid == 0) atomicOr(ta_err, 1);
    finish();
    return;
  }

  // ---------------- per-member results ----------------
  if (b == 0 && h == 0 && lg == 0 && jv) {
    ta_coli[CI_ITERS * N + j] = iters;
    ta_coli[CI_STATUS * N + j] = status;
    ta_coli[CI_FALLBACK * N + j] = 0;
    ta_col[CF_DN * N + j] = dn;
    if (ta_iters_out) ta_iters_out[j] = iters;
  }
  if (h == 0 && lg == 0) L.dnl[n] = dn;
  if (ta_z_out && jv)
#pragma unroll
    for (int t = 0; t < C::RT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gi = i0 + hb + t * 16 + 4 * lg + i;
        if (gi < m) ta_z_out[(size_t)gi * N + j] = z[t][i];
      }

  // ---------------- W = S^T Z/(N-1): FP64 products, summed like the iterations ----------------
  const unsigned ew = ep + 1;
  {
    v4d wacc[C::KT];
#pragma unroll
    for (int k = 0; k < C::KT; ++k) wacc[k] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < C::RT; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float* srow = &L.S[(hb + t * 16 + 4 * lg + u) * C::LDS + lr];
        const double bz = (double)z[t][u];
#pragma unroll
        for (int k = 0; k < C::KT; ++k) wacc[k] = mfma4((double)srow[16 * k], bz, wacc[k]);
      }
    for (int ct = 0; ct < 2; ++ct) {
      if (cw == ct && h == 1)
#pragma unroll
        for (int k = 0; k < C::KT; ++k)
#pragma unroll
          for (int i = 0; i < 4; ++i) L.xw[lane][k * 4 + i] = wacc[k][i];
      __syncthreads();
      if (cw == ct && h == 0)
#pragma unroll
        for (int k = 0; k < C::KT; ++k)
#pragma unroll
          for (int i = 0; i < 4; ++i) wacc[k][i] += L.xw[lane][k * 4 + i];
      __syncthreads();
    }
    // f64 accumulator rows are lg + 4 i
    if (h == 0)
#pragma unroll
      for (int k = 0; k < C::KT; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          st_pair(mypart + 2 * ((16 * k + frag_row<double>(lg, i)) * kTW + n), wacc[k][i], ew);
  }
  const int NW = NP * kTW;
  const int wlo = b * NW / nblk, wl = (b + 1) * NW / nblk - wlo;
  const double invd = 1.0 / (double)(N - 1);
  const bool keep = ta_want_relres != 0;
  if (!owner_sum(
          gpart, C::SLOT, nblk, ew, 0, 0, 0, wlo, wl, L.own, [](int, double) {},
          [&](int d, double tot) {
            const int kk = d / kTW, jj = c * kTW + (d - kk * kTW);
            if (kk < N && jj < N) ta_Wd[(size_t)kk * N + jj] = tot * invd;
            if (keep) st_pair(red + 2 * C::E + 2 * d, tot, ew);
          })) {
    if (tid == 0) atomicOr(ta_err, 1);
    finish();
    return;
  }
  TTRACE(251);
  if (!keep) {
    finish();
    return;
  }

  // ---------------- true residual d - S (S^T z)/(N-1) - R z, in double ----------------
  double wv2[C::KT][4];
  {
    // one 16-row chunk of W at a time (eight words in flight per lane)
    const unsigned long long* rw = red + 2 * C::E;
#pragma unroll
    for (int k = 0; k < C::KT; ++k) {
      unsigned long long w0[4], w1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const unsigned long long* q = rw + 2 * ((16 * k + 4 * lg + u) * kTW + n);
        w0[u] = ld64(q);
        w1[u] = ld64(q + 1);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const unsigned long long* q = rw + 2 * ((16 * k + 4 * lg + u) * kTW + n);
        w0[u] = poll64(q, ew, w0[u], bad);
        w1[u] = poll64(q + 1, ew, w1[u], bad);
        wv2[k][u] = pair2(w0[u], w1[u]);
      }
    }
    if (__syncthreads_or(bad)) {
      if (tid == 0) atomicOr(ta_err, 1);
      finish();
      return;
    }
  }
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  {
    // the A rows are permuted (row 4 (m % 4) + m / 4 of the tile as row m) so
    // that the f64 accumulators land on the rows this lane holds
    const int pr = 4 * (lr & 3) + (lr >> 2);
#pragma unroll
    for (int t = 0; t < C::RT; ++t) {
      v4d racc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < C::KT; ++k) {
        const v4f av = *reinterpret_cast<const v4f*>(
            &L.S[(hb + t * 16 + pr) * C::LDS + 16 * k + 4 * lg]);
#pragma unroll
        for (int u = 0; u < 4; ++u) racc = mfma4((double)av[u], wv2[k][u], racc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = hb + t * 16 + 4 * lg + i, gi = i0 + row;
        if (gi < m && jv) {
          const double d = (double)ta_D[(size_t)gi * N + j];
          const double res = d - racc[i] * invd - (double)L.rv[row] * (double)z[t][i];
          v[0] += res * res;
        }
      }
    }
  }
  tile_sums(v);
  __syncthreads();
  const unsigned er = ew + 1;
  if (h == 0 && lg == 0) st_pair(mypart + 2 * n, v[0] + L.xs[cw][lr][0], er);
  const int rlo = b * kTW / nblk, rl = (b + 1) * kTW / nblk - rlo;
  if (!owner_sum(
          gpart, C::SLOT, nblk, er, 0, 0, 0, rlo, rl, L.own, [](int, double) {},
          [&](int nn, double tot) {
            const int jj = c * kTW + nn;
            if (jj < N) {
              const double dnj = L.dnl[nn];
              const double rr2 = dnj > 0 ? sqrt(tot / dnj) : 0.0;
              ta_relres[jj] = rr2;
              if (ta_relres_out) ta_relres_out[jj] = rr2;
            }
          })) {
    if (tid == 0) atomicOr(ta_err, 1);
  }
  finish();
}

// ---------------------------------------------------------------------------
// The mixed-precision mode on the same decomposition: restarted iterative
// refinement (the column solver's method, with the S-products on the MFMA).
//
//  * Outer step: W = S^T z and the true residual r = d - Psi z, both from the
//    FP32 S of the gather launch (read from memory) with FP64 MFMA products
//    and FP64 sums; a member stops when ||r|| <= tol ||d||.
//  * Inner solve: CG for Psi delta = r from delta = 0 on the BF16 copy of S
//    kept in LDS (v_mfma_f32_16x16x32_bf16, FP32 accumulation; z accumulates
//    delta), until the member's recursive residual is below 1e-2 of its outer
//    residual or tol ||d||, at least one step per inner solve.
//
// The reported iteration count is the total of inner steps; W is the exact
// S^T z of the final outer step.
//
// SPLIT: the split-BF16 mode on the same code (the split products of Henry,
// Tang and Heinecke, 2019).  S is kept in LDS as two BF16 parts (s1 = bf16(s),
// s2 = bf16(s - s1): about 16 bits, 2^-18 relative), the vector operand is
// split into three the same way, and every S-product is five BF16 MFMA
// products, s2 v2 + s1 v3 + s2 v1 + s1 v2 + s1 v1 (small terms first): their
// bf16x3 set plus the two bf16x6 terms that need no third part of S.  FP32
// accumulation.  The solve is plain CG, stopped on the recursive residual as
// in the FP32 mode; then one final step computes the exact W and the true
// residual in FP64 from the FP32 S, and the member's status is that of its
// CG (no restart).  The gathered W then takes the LDS room of S, which is no
// longer needed.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
__device__ inline v4f mfma_bf16(bf16x8 a, bf16x8 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
constexpr double kTileInnerRel = 1e-2;

template <int NP, int RB, bool SPLIT>
struct __align__(16) TLdsMx {
  using C = TC<NP, RB>;
  // BF16 row stride (16-byte rows, skewed banks); SPLIT rows hold s1, then s2
  static constexpr int LDB = SPLIT ? 2 * NP + 8 : NP + 8;
  static constexpr int WGS = C::KT * 4 + 2;  // gathered-W row stride (doubles)
  __bf16 Sb[RB * LDB];
  union {
    float xg[2][2][64][C::KT * 2 + 4];
    double xw[64][18];
    // gathered W, rows 16 k + 4 lg + u of member n (SPLIT: in the room of Sb)
    double wg[SPLIT ? 1 : 2][64][SPLIT ? 2 : WGS];
  };
  float rv[RB];
  double xs[2][16][4];
  double own[kBlock];
};

template <int NP, int RB, bool TR, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_cg_tilemx(TileArgs a) {
  const float* const ta_D = a.D;
  int const ta_N = a.N;
  int const ta_NG = a.NG;
  const float* const ta_S = a.S;
  double* const ta_Wd = a.Wd;
  unsigned long long* const ta_census = a.census;
  unsigned long long const ta_census_ticks = a.census_ticks;
  double* const ta_col = a.col;
  int* const ta_coli = a.coli;
  int* const ta_err = a.err;
  int* const ta_iters_out = a.iters_out;
  int const ta_m = a.m;
  int const ta_maxit = a.maxit;
  int const ta_nblk = a.nblk;
  double* const ta_relres = a.relres;
  double* const ta_relres_out = a.relres_out;
  const float* const ta_rv = a.rv;
  double const ta_tol = a.tol;
  unsigned long long* const ta_trace = a.trace;
  unsigned long long* const ta_txp = a.txp;
  unsigned long long* const ta_txr = a.txr;
  float* const ta_z_out = a.z_out;
  using C = TC<NP, RB>;
  using LdsT = TLdsMx<NP, RB, SPLIT>;
  constexpr int LDB = LdsT::LDB, WGS = LdsT::WGS;
  constexpr int K32 = NP / 32;  // 32-wide K chunks of Q = S G
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LdsT& L = *reinterpret_cast<LdsT*>(smem_raw);
  static_assert(!SPLIT || 2 * 64 * WGS * sizeof(double) <= sizeof(L.Sb), "W fits in the room of S");
  double* const wgb = SPLIT ? reinterpret_cast<double*>(L.Sb) : &L.wg[0][0][0];
  auto WG = [&](int cw_, int ln, int x) -> double* { return wgb + (cw_ * 64 + ln) * WGS + x; };
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int cw = wv & 1, h = wv >> 1;
  const int NG = ta_NG, nblk = ta_nblk;
  const int c = blockIdx.x % NG, b = blockIdx.x / NG;
  const int N = ta_N, m = ta_m;
  const int i0 = b * RB;
  const int n = cw * 16 + lr;
  const int j = c * kTW + n;
  const bool jv = j < N;
  const int hb = h * (RB / 2);
  const float inv = (float)(1.0 / (double)(N - 1));
  const double invd = 1.0 / (double)(N - 1);
  unsigned long long* mypart = ta_txp + (size_t)(c * nblk + b) * C::SLOT;
  const unsigned long long* gpart = ta_txp + (size_t)c * nblk * C::SLOT;
  unsigned long long* red = ta_txr + (size_t)c * C::SLOTR;
  const int glo = b * C::EG / nblk, Lg = (b + 1) * C::EG / nblk - glo;
  const int dlo = b * C::ND / nblk, Ld = (b + 1) * C::ND / nblk - dlo;
  const int NW = NP * kTW;
  const int wlo = b * NW / nblk, wl = (b + 1) * NW / nblk - wlo;
  unsigned long long census_count = 0;
  if (ta_census && tid == 0) census_count = census_arrive(ta_census);
  unsigned long long* const trb = tile_trace_buf<TR>();
  if constexpr (TR) {
    for (int e = tid; e < 256; e += kBlock) trb[e] = 0ull;
    __syncthreads();
  }
  TTRACE(0);
  auto finish = [&]() __attribute__((always_inline)) {
    if constexpr (TR) {
      __syncthreads();
      if (b == 0 && c == 0 && ta_trace)
        for (int e = tid; e < 256; e += kBlock)
          if (trb[e]) ta_trace[e] = trb[e];
    }
  };

  // ---------------- S block in BF16 and the rows' diag(R) ----------------
  for (int e = tid; e < RB * NP / 4; e += kBlock) {
    const int i = e / (NP / 4), c4 = (e - i * (NP / 4)) * 4, gi = i0 + i;
    v4f x = v4f{0.f, 0.f, 0.f, 0.f};
    if (gi < m) x = *reinterpret_cast<const v4f*>(ta_S + (size_t)gi * NP + c4);
    bf16x4 y, yl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      y[q] = (__bf16)x[q];
      yl[q] = (__bf16)(x[q] - (float)y[q]);
    }
    *reinterpret_cast<bf16x4*>(&L.Sb[i * LDB + c4]) = y;
    if constexpr (SPLIT) *reinterpret_cast<bf16x4*>(&L.Sb[i * LDB + NP + c4]) = yl;
  }
  for (int i = tid; i < RB; i += kBlock) L.rv[i] = (i0 + i < m) ? ta_rv[i0 + i] : 0.f;
  __syncthreads();

  // ---------------- column state: z = p = 0, r = d ----------------
  float z[C::RT][4], r[C::RT][4], p[C::RT][4];
#pragma unroll
  for (int t = 0; t < C::RT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int gi = i0 + hb + t * 16 + 4 * lg + i;
      r[t][i] = (gi < m && jv) ? ta_D[(size_t)gi * N + j] : 0.f;
      z[t][i] = 0.f;
      p[t][i] = 0.f;
    }

  auto gram_row = [](int k, int lgi, int i) { return 64 * (k >> 2) + 16 * lgi + 4 * i + (k & 3); };
  // Partial S_b^T r on the BF16 MFMA over this wave's rows: a 32-row K step
  // takes the row tiles 2s and 2s+1; lane group lg supplies their rows
  // 4 lg + i (its own r, as BF16), and output tile 4 kq + e the Gram rows
  // 64 kq + 4 m + e (gram_row), so that one 8-byte read of S feeds 4 tiles.
  // (SPLIT: five products per tile, small terms first)
  auto gram_bf = [&](v4f (&g)[C::KT]) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < C::KT; ++k) g[k] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < C::RT / 2; ++s) {
      bf16x8 bv, bl, b3;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float x = r[2 * s + q / 4][q % 4];
        bv[q] = (__bf16)x;
        const float x2 = x - (float)bv[q];
        bl[q] = (__bf16)x2;
        b3[q] = (__bf16)(x2 - (float)bl[q]);
      }
#pragma unroll
      for (int kq = 0; kq < C::KT / 4; ++kq) {
        bf16x8 av[4], al[4];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int row = hb + (2 * s + q / 4) * 16 + 4 * lg + (q % 4);
          const bf16x4 x = *reinterpret_cast<const bf16x4*>(&L.Sb[row * LDB + 64 * kq + 4 * lr]);
#pragma unroll
          for (int e = 0; e < 4; ++e) av[e][q] = x[e];
          if constexpr (SPLIT) {
            const bf16x4 xl =
                *reinterpret_cast<const bf16x4*>(&L.Sb[row * LDB + NP + 64 * kq + 4 * lr]);
#pragma unroll
            for (int e = 0; e < 4; ++e) al[e][q] = xl[e];
          }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if constexpr (SPLIT) {
            g[4 * kq + e] = mfma_bf16(al[e], bl, g[4 * kq + e]);
            g[4 * kq + e] = mfma_bf16(av[e], b3, g[4 * kq + e]);
            g[4 * kq + e] = mfma_bf16(al[e], bv, g[4 * kq + e]);
            g[4 * kq + e] = mfma_bf16(av[e], bl, g[4 * kq + e]);
          }
          g[4 * kq + e] = mfma_bf16(av[e], bv, g[4 * kq + e]);
        }
      }
    }
  };
  auto tile_sums = [&](double (&v)[4]) __attribute__((always_inline)) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      v[f] += __shfl_xor(v[f], 16);
      v[f] += __shfl_xor(v[f], 32);
    }
    if (h == 1 && lg == 0)
#pragma unroll
      for (int f = 0; f < 4; ++f) L.xs[cw][lr][f] = v[f];
  };
  auto swap_publish = [&](auto hc, unsigned ep, v4f (&g)[C::KT]) __attribute__((always_inline)) {
    constexpr int H = decltype(hc)::value, KH = C::KT / 2;
#pragma unroll
    for (int kk = 0; kk < KH; ++kk)
#pragma unroll
      for (int i = 0; i < 4; ++i) L.xg[cw][H][lane][kk * 4 + i] = g[(1 - H) * KH + kk][i];
    __syncthreads();
    unsigned long long* pp = mypart + (ep & 1) * C::E;
#pragma unroll
    for (int kk = 0; kk < KH; ++kk)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        constexpr int k0 = H * KH;
        const float x = g[k0 + kk][i] + L.xg[cw][1 - H][lane][kk * 4 + i];
        st64(pp + gram_row(k0 + kk, lg, i) * kTW + n, __float_as_uint(x), ep);
      }
  };
  auto exchange = [&](unsigned ep, v4f (&g)[C::KT], double (&v)[4], int slot) __attribute__((always_inline)) -> bool {
    if (h == 0)
      swap_publish(std::integral_constant<int, 0>{}, ep, g);
    else
      swap_publish(std::integral_constant<int, 1>{}, ep, g);
    unsigned long long* pp = mypart + (ep & 1) * C::E;
    if (h == 0 && lg == 0)
#pragma unroll
      for (int f = 0; f < 4; ++f)
        st_pair(pp + C::EG + 2 * (n * 4 + f), v[f] + L.xs[cw][lr][f], ep);
    TTRACE(slot);
    unsigned long long* rp = red + (ep & 1) * C::E;
    return owner_sum(
        gpart + (ep & 1) * C::E, C::SLOT, nblk, ep, glo, Lg, C::EG, dlo, Ld, L.own,
        [&](int x, double tot) { st64(rp + x, __float_as_uint((float)tot), ep); },
        [&](int d, double tot) { st_pair(rp + C::EG + 2 * d, tot, ep); });
  };
  // the sums of an exchange's start: r r, r R r (float r) and the true
  // residual's r r in double (third slot, trr)
  auto start_sums = [&](double (&v)[4], double trr) __attribute__((always_inline)) {
    v[0] = v[1] = v[3] = 0.0;
    v[2] = trr;
#pragma unroll
    for (int t = 0; t < C::RT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double rr = r[t][i], rvv = L.rv[hb + t * 16 + 4 * lg + i];
        v[0] += rr * rr;
        v[1] += rvv * rr * rr;
      }
  };

  // ---------------- first outer step: z = 0, so r = d ----------------
  unsigned ep = 0;
  bool bad = false;
  {
    double trr = 0.0;
#pragma unroll
    for (int t = 0; t < C::RT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) trr += (double)r[t][i] * (double)r[t][i];
    double v[4];
    start_sums(v, trr);
    tile_sums(v);
    v4f g[C::KT];
    gram_bf(g);
    if (ta_census && !census_wait(ta_census, ta_err, ta_census_ticks, census_count)) {
      finish();
      return;
    }
    bad = !exchange(++ep, g, v, 2);
  }
  TTRACE(1);

  float G[K32][8];  // S^T p of the previous step, rows 32 k + 8 lg + u of member n
#pragma unroll
  for (int k = 0; k < K32; ++k)
#pragma unroll
    for (int u = 0; u < 8; ++u) G[k][u] = 0.f;
  const double tol2 = ta_tol * ta_tol;
  bool active = jv, inner = false, fresh = true;
  bool outer_x = true, first = true;  // the exchange gathered next starts an inner solve
  int iters = 0, status = COL_RUNNING;
  bool wdone = false;  // W of the current z published
  int split_status = COL_RUNNING;  // SPLIT: how the member's CG stopped
  int nout = 0;        // outer steps taken (trace slots 20 + 8 nout: start,
                       // W gathered (+3), exchange done (+6), step index (+7))
  double dn = 0.0, rhoprev = 0.0, thr2 = 0.0, rho_true = 0.0;
  for (int kit = 0; !bad; ++kit) {
    // ---- all-gather of exchange ep (each word once per workgroup) ----
    // (each thread polls its words together, as in the FP32 solver)
    const unsigned long long* rp = red + (ep & 1) * C::E;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    auto gather_half = [&](auto hc) __attribute__((always_inline)) {
      constexpr int H = decltype(hc)::value, KH = K32 / 2, NGW = KH * 8;
      // words 0 .. NGW-1: rows 32 (H KH + kk) + 8 lg + u; then the member's 8
      // sum words (lane group 0 only)
      unsigned long long w[NGW + 8];
      auto at = [&](int u) {
        return u < NGW ? rp + (32 * (H * KH + u / 8) + 8 * lg + u % 8) * kTW + n
                       : rp + C::EG + 8 * n + (u - NGW);
      };
      const int nw = lg == 0 ? NGW + 8 : NGW;
#pragma unroll
      for (int u = 0; u < NGW + 8; ++u)
        if (u < nw) w[u] = ld64(at(u));
      poll_all(w, nw, at, ep, bad);
#pragma unroll
      for (int u = 0; u < NGW; ++u) L.xg[cw][H][lane][u] = __uint_as_float((unsigned)w[u]);
      if (lg == 0)
#pragma unroll
        for (int f = 0; f < 4; ++f) sums[f] = pair2(w[NGW + 2 * f], w[NGW + 2 * f + 1]);
    };
    if (h == 0)
      gather_half(std::integral_constant<int, 0>{});
    else
      gather_half(std::integral_constant<int, 1>{});
    if (__syncthreads_or(bad)) {
      bad = true;
      break;
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) sums[f] = __shfl(sums[f], lr);
    if (kit < 10) TTRACE(128 + 12 * kit + 0);
    const double rho = sums[0], ar = sums[1];
    // at the start of an inner solve the third slot is the true residual's
    // r r and the step's p is zero; later it is r R p, the fourth p R p
    const double arp = outer_x ? 0.0 : sums[2], ap = outer_x ? 0.0 : sums[3];
    if (outer_x) {
      rho_true = sums[2];
      if (first) dn = rho_true;
      if (active) {
        if (SPLIT && !first) {
          active = false;  // SPLIT: the final step after the CG
          status = split_status;
        } else if (rho_true <= tol2 * dn) {
          active = false;
          status = COL_CONVERGED;
        } else if (iters >= ta_maxit) {
          active = false;
          status = COL_MAXIT;
        } else {
          inner = true;
          fresh = true;
          thr2 = SPLIT ? tol2 * dn : fmax(tol2 * dn, kTileInnerRel * kTileInnerRel * rho_true);
        }
      }
    }
    // ---- decide the inner step ----
    int mode = MODE_FROZEN;
    double beta = 0.0;
    if (inner) {
      if ((!fresh && rho <= thr2) || iters >= ta_maxit) {
        inner = false;  // this inner solve is done for the member
        split_status = (!fresh && rho <= thr2) ? COL_CONVERGED : COL_MAXIT;
      } else {
        mode = MODE_STEP;
        beta = fresh ? 0.0 : rho / rhoprev;
      }
    }
    // (16-byte LDS reads outside any branch; frozen members take G = 0 by a
    // select)
    // (G in FP32 FMAs, its squared norm in four FP32 partial sums)
    const bool step = mode == MODE_STEP;
    const float bf = (float)beta;
    float ggp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < K32; ++k)
#pragma unroll
      for (int c4 = 0; c4 < 2; ++c4) {
        const v4f x = *reinterpret_cast<const v4f*>(&L.xg[cw][k / (K32 / 2)][lane][(k % (K32 / 2)) * 8 + 4 * c4]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = 4 * c4 + q;
          const float gd = beta != 0.0 ? fmaf(bf, G[k][u], x[q]) : x[q];
          const float gv = step ? gd : 0.f;
          G[k][u] = gv;
          ggp[q] = fmaf(gv, gv, ggp[q]);
        }
      }
    double gg = ((double)ggp[0] + (double)ggp[1]) + ((double)ggp[2] + (double)ggp[3]);
    gg += __shfl_xor(gg, 16);
    gg += __shfl_xor(gg, 32);
    double alpha = 0.0;
    if (mode == MODE_STEP) {
      alpha = rho / (gg * invd + ar + 2.0 * beta * arp + beta * beta * ap);
      rhoprev = rho;
      fresh = false;
      ++iters;
      if (!isfinite(alpha) || !isfinite(beta)) {
        active = false;
        inner = false;
        status = COL_NONFINITE;
        mode = MODE_FROZEN;
        alpha = 0.0;
#pragma unroll
        for (int k = 0; k < K32; ++k)
#pragma unroll
          for (int u = 0; u < 8; ++u) G[k][u] = 0.f;
      }
    }
    outer_x = false;
    first = false;
    if (__syncthreads_or(mode == MODE_STEP)) {
      // ---------------- one inner step on the BF16 operator ----------------
      if (kit < 10) TTRACE(128 + 12 * kit + 1);
      const float be = (float)beta, al = (float)alpha;
      bf16x8 gb[K32], gl[K32], g3[K32];
#pragma unroll
      for (int k = 0; k < K32; ++k)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          gb[k][u] = (__bf16)G[k][u];
          const float x2 = G[k][u] - (float)gb[k][u];
          gl[k][u] = (__bf16)x2;
          g3[k][u] = (__bf16)(x2 - (float)gl[k][u]);
        }
      v4f qacc[C::RT];
#pragma unroll
      for (int t = 0; t < C::RT; ++t) qacc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < K32; ++k)
#pragma unroll
        for (int t = 0; t < C::RT; ++t) {
          const __bf16* srow = &L.Sb[(hb + t * 16 + lr) * LDB + 32 * k + 8 * lg];
          const bf16x8 av = *reinterpret_cast<const bf16x8*>(srow);
          if constexpr (SPLIT) {
            const bf16x8 al = *reinterpret_cast<const bf16x8*>(srow + NP);
            qacc[t] = mfma_bf16(al, gl[k], qacc[t]);
            qacc[t] = mfma_bf16(av, g3[k], qacc[t]);
            qacc[t] = mfma_bf16(al, gb[k], qacc[t]);
            qacc[t] = mfma_bf16(av, gl[k], qacc[t]);
          }
          qacc[t] = mfma_bf16(av, gb[k], qacc[t]);
        }
#pragma unroll
      for (int t = 0; t < C::RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) p[t][i] = (mode == MODE_STEP) ? r[t][i] + be * p[t][i] : 0.f;
      double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < C::RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float rvv = L.rv[hb + t * 16 + 4 * lg + i];
          if (mode == MODE_STEP) {
            const float q = qacc[t][i] * inv + rvv * p[t][i];
            z[t][i] += al * p[t][i];
            r[t][i] -= al * q;
          }
          const double rr = r[t][i], pp = p[t][i];
          v[0] += rr * rr;
          v[1] += (double)rvv * rr * rr;
          v[2] += (double)rvv * rr * pp;
          v[3] += (double)rvv * pp * pp;
        }
      tile_sums(v);
      if (kit < 10) TTRACE(128 + 12 * kit + 2);
      v4f g[C::KT];
      gram_bf(g);
      if (kit < 10) TTRACE(128 + 12 * kit + 3);
      bad = !exchange(++ep, g, v, kit < 10 ? 128 + 12 * kit + 5 : 255);
      if (kit < 10) TTRACE(128 + 12 * kit + 4);
      continue;
    }
    if (!__syncthreads_or(active)) break;  // every member of the group is done

    if (kit < 10) TTRACE(128 + 12 * kit + 6);
    const int os = nout < 12 ? 20 + 8 * nout : 255;
    if constexpr (TR)
      if (tid == 0 && nout < 12) trb[os + 7] = (unsigned long long)kit;
    ++nout;
    TTRACE(os);
    // ---------------- outer step: W = S^T z and r = d - Psi z, FP64 ----------------
    // W partial on the FP64 MFMA, S from memory (16-byte loads feeding four
    // interleaved output tiles, rows 64 kq + 4 m + e), FP64 accumulator rows
    // are lg + 4 i
    // The step after this one restarts (beta = 0): G is not needed until then,
    // and zeroing it frees its registers here.
#pragma unroll
    for (int k = 0; k < K32; ++k)
#pragma unroll
      for (int u = 0; u < 8; ++u) G[k][u] = 0.f;
    // (one 64-row chunk kq of W at a time).  Rows past m read row m - 1:
    // z is exactly zero there.  The empty asm keeps the row addresses from
    // being computed ahead of the loop (they would stay live all along).
    ++ep;
    int orow = i0 + hb + 4 * lg;
    asm volatile("" : "+v"(orow));
#pragma unroll 1
    for (int kq = 0; kq < C::KT / 4; ++kq) {
      v4d wacc[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) wacc[e] = v4d{0.0, 0.0, 0.0, 0.0};
      // two row tiles (eight 16-byte loads) per batch; the next batch is in
      // flight while this one feeds the MFMA (the trace variant loads each
      // batch just before its use)
      constexpr int NW2 = TR ? 1 : 2;
      v4f sb[NW2][8];
      auto load_pair = [&](int tp, v4f (&bb)[8]) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int gi = min(orow + (2 * tp + q / 4) * 16 + q % 4, m - 1);
          bb[q] = *reinterpret_cast<const v4f*>(ta_S + (size_t)gi * NP + 64 * kq + 4 * lr);
        }
      };
      if constexpr (NW2 == 2) load_pair(0, sb[0]);
#pragma unroll
      for (int tp = 0; tp < C::RT / 2; ++tp) {
        if constexpr (NW2 == 1)
          load_pair(tp, sb[0]);
        else if (tp + 1 < C::RT / 2)
          load_pair(tp + 1, sb[(tp + 1) % NW2]);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double bz = (double)z[2 * tp + q / 4][q % 4];
#pragma unroll
          for (int e = 0; e < 4; ++e) wacc[e] = mfma4((double)sb[tp % NW2][q][e], bz, wacc[e]);
        }
      }
      for (int ct = 0; ct < 2; ++ct) {
        if (cw == ct && h == 1)
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int i = 0; i < 4; ++i) L.xw[lane][e * 4 + i] = wacc[e][i];
        __syncthreads();
        if (cw == ct && h == 0)
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int i = 0; i < 4; ++i) wacc[e][i] += L.xw[lane][e * 4 + i];
        __syncthreads();
      }
      if (h == 0)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = 64 * kq + 4 * frag_row<double>(lg, i) + e;
            st_pair(mypart + 2 * (row * kTW + n), wacc[e][i], ep);
          }
    }
    if (!owner_sum(
            gpart, C::SLOT, nblk, ep, 0, 0, 0, wlo, wl, L.own, [](int, double) {},
            [&](int d, double tot) {
              const int kk = d / kTW, jj = c * kTW + (d - kk * kTW);
              if (kk < N && jj < N) ta_Wd[(size_t)kk * N + jj] = tot * invd;
              st_pair(red + 2 * C::E + 2 * d, tot, ep);
            })) {
      bad = true;
      break;
    }
    if (kit < 10) TTRACE(128 + 12 * kit + 7);
    wdone = true;
    // gather W into LDS (rows 16 k + 4 lg + u of member n; the two wave
    // halves take half of the 16-row chunks each), then
    // r = d - S W/(N-1) - R z
    {
      const unsigned long long* rw = red + 2 * C::E;
#pragma unroll 1
      for (int kk = 0; kk < C::KT / 2; ++kk) {
        const int k = h * (C::KT / 2) + kk;
        unsigned long long w0[4], w1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned long long* q = rw + 2 * ((16 * k + 4 * lg + u) * kTW + n);
          w0[u] = ld64(q);
          w1[u] = ld64(q + 1);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned long long* q = rw + 2 * ((16 * k + 4 * lg + u) * kTW + n);
          w0[u] = poll64(q, ep, w0[u], bad);
          w1[u] = poll64(q + 1, ep, w1[u], bad);
          *WG(cw, lane, k * 4 + u) = pair2(w0[u], w1[u]);
        }
      }
      if (__syncthreads_or(bad)) {
        bad = true;
        break;
      }
    }
    TTRACE(os + 3);
    double trr = 0.0;
    {
      // the A rows are permuted (row 4 (m % 4) + m / 4 as row m) so that the
      // FP64 accumulators land on the rows this lane holds
      // (rows past m read row m - 1; their results are not used)
      // (the next row tile's S and D loads are in flight during this one's
      // MFMAs)
      int opr = i0 + hb + 4 * (lr & 3) + (lr >> 2);
      asm volatile("" : "+v"(opr));
      // d goes into p's registers (p restarts from zero below); unconditional
      // loads from a clamped row and member, since a branch around a load
      // would drain the S loads in flight.  (A fresh opaque row base: the
      // W partial's row indices are not kept live until here.)
      // The trace variant loads d per row tile instead.
      int drow = orow;
      asm volatile("" : "+v"(drow));
      auto load_d = [&](int t, int i) __attribute__((always_inline)) {
        return ta_D[(size_t)min(drow + t * 16 + i, m - 1) * N + min(j, N - 1)];
      };
      if constexpr (!TR)
#pragma unroll
        for (int t = 0; t < C::RT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) p[t][i] = load_d(t, i);
      // (the trace variant loads each tile just before its use: its
      // timestamps take the registers of the second buffer)
      constexpr int NB = TR ? 1 : 2;
      v4f ab[NB][C::KT];
      auto load_tile = [&](int t, v4f (&aa)[C::KT]) __attribute__((always_inline)) {
        const float* arow = ta_S + (size_t)min(opr + t * 16, m - 1) * NP + 4 * lg;
#pragma unroll
        for (int k = 0; k < C::KT; ++k) aa[k] = *reinterpret_cast<const v4f*>(arow + 16 * k);
      };
      if constexpr (NB == 2) load_tile(0, ab[0]);
#pragma unroll
      for (int t = 0; t < C::RT; ++t) {
        if constexpr (NB == 1)
          load_tile(t, ab[0]);
        else if (t + 1 < C::RT)
          load_tile(t + 1, ab[(t + 1) % NB]);
        float dv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) dv[i] = TR ? load_d(t, i) : p[t][i];
        v4d racc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < C::KT; ++k) {
          const v4f av = ab[t % NB][k];
          const v2d w01 = *reinterpret_cast<const v2d*>(WG(cw, lane, k * 4));
          const v2d w23 = *reinterpret_cast<const v2d*>(WG(cw, lane, k * 4 + 2));
          racc = mfma4((double)av[0], w01[0], racc);
          racc = mfma4((double)av[1], w01[1], racc);
          racc = mfma4((double)av[2], w23[0], racc);
          racc = mfma4((double)av[3], w23[1], racc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = hb + t * 16 + 4 * lg + i, gi = drow + t * 16 + i;
          const double rvv = L.rv[row];
          const double res0 = (double)dv[i] - racc[i] * invd - rvv * (double)z[t][i];
          const double res = (gi < m && jv) ? res0 : 0.0;
          trr += res * res;
          // members that are done keep r (their inner solves no longer run)
          if (active) r[t][i] = (float)res;
          p[t][i] = 0.f;
        }
      }
    }
    // every wave has read W (wg) before the exchange below writes xg over it
    __syncthreads();
    if (kit < 10) TTRACE(128 + 12 * kit + 8);
    {
      double v[4];
      start_sums(v, trr);
      tile_sums(v);
      v4f g[C::KT];
      // (SPLIT: no CG step follows, and W has taken the room of S)
      if constexpr (SPLIT) {
#pragma unroll
        for (int k = 0; k < C::KT; ++k) g[k] = v4f{0.f, 0.f, 0.f, 0.f};
      } else {
        gram_bf(g);
      }
      if (kit < 10) TTRACE(128 + 12 * kit + 3);
      bad = !exchange(++ep, g, v, kit < 10 ? 128 + 12 * kit + 5 : 255);
      if (kit < 10) TTRACE(128 + 12 * kit + 4);
      TTRACE(os + 6);
      outer_x = true;
    }
  }
  TTRACE(250);
  if (bad) {
    if (tid == 0) atomicOr(ta_err, 1);
    finish();
    return;
  }
  // no member took a step: z = 0 and W = 0 (this workgroup's share)
  if (!wdone)
    for (int d = wlo + tid; d < wlo + wl; d += kBlock) {
      const int kk = d / kTW, jj = c * kTW + (d - kk * kTW);
      if (kk < N && jj < N) ta_Wd[(size_t)kk * N + jj] = 0.0;
    }
  // ---------------- per-member results ----------------
  if (b == 0 && h == 0 && lg == 0 && jv) {
    ta_coli[CI_ITERS * N + j] = iters;
    ta_coli[CI_STATUS * N + j] = status;
    ta_coli[CI_FALLBACK * N + j] = 0;
    ta_col[CF_DN * N + j] = dn;
    if (ta_iters_out) ta_iters_out[j] = iters;
    const double rr2 = dn > 0 ? sqrt(rho_true / dn) : 0.0;
    ta_relres[j] = rr2;
    if (ta_relres_out) ta_relres_out[j] = rr2;
  }
  if (ta_z_out && jv)
#pragma unroll
    for (int t = 0; t < C::RT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gi = i0 + hb + t * 16 + 4 * lg + i;
        if (gi < m) ta_z_out[(size_t)gi * N + j] = z[t][i];
      }
  finish();
}

// Gather ahead of the solver: for 16 observation rows per workgroup (16
// lanes per row, NP / 16 members per lane), HX, the row mean and
// S = HX - zbar in double, rounded once, into S (m x NP, row-major, zero past
// N); D = y + eps - HX (m x N); the rows' diag(R) (1 when preconditioned,
// with S and D scaled by 1/sqrt(r)).
template <int NP>
__global__ __launch_bounds__(kBlock) void k_tile_gather(CGArgs<float> a) {
  constexpr int CPC = NP / 16;
  const int tid = threadIdx.x, N = a.N;
  const int gi = blockIdx.x * 16 + (tid >> 4), cc = (tid & 15) * CPC;
  if (gi >= a.m) return;  // all 16 lanes of the row together
  double hx[CPC];
#pragma unroll
  for (int u = 0; u < CPC; ++u) hx[u] = 0.0;
  const bool vec = (N & 3) == 0;
  for (int t = 0; t < a.k; ++t) {
    const int src = a.idx[(size_t)gi * a.k + t];
    const double wt = (double)a.hw[(size_t)gi * a.k + t];
    if ((unsigned)src >= (unsigned)a.ng) {
      if ((tid & 15) == 0) atomicOr(a.err, 2);
      continue;
    }
    const float* xr = a.Xg + (size_t)src * N + cc;
    if (vec) {
#pragma unroll
      for (int u = 0; u < CPC; u += 4)
        if (cc + u < N) {
          const v4f x = *reinterpret_cast<const v4f*>(xr + u);
#pragma unroll
          for (int q = 0; q < 4; ++q) hx[u + q] += wt * (double)x[q];
        }
    } else {
#pragma unroll
      for (int u = 0; u < CPC; ++u)
        if (cc + u < N) hx[u] += wt * (double)xr[u];
    }
  }
  double sum = 0.0;
#pragma unroll
  for (int u = 0; u < CPC; ++u) sum += hx[u];
  sum = group_sum<16>(sum);
  const double mean = sum / (double)N;
  const double sc = precond_row_scale(a, gi);
  const double yv = (double)a.y[gi];
#pragma unroll
  for (int u = 0; u < CPC; ++u) {
    const int col = cc + u;
    a.tS[(size_t)gi * NP + col] = col < N ? (float)((hx[u] - mean) * sc) : 0.f;
    if (col < N) {
      double dd = yv - hx[u];
      if (a.eps) dd += (double)a.eps[(size_t)gi * N + col];
      a.D[(size_t)gi * N + col] = (float)(dd * sc);
    }
  }
  if ((tid & 15) == 0) a.tR[gi] = effective_r(a, gi);
}

__global__ void k_zero_words(unsigned long long* p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

// The solver variants: 0 FP32 (k_cg_tile), 1 the mixed mode, 2 the split-BF16
// mode (both k_cg_tilemx).
template <int NP, int RB, int V, bool TR>
const void* tile_fn() {
  if constexpr (V == 0)
    return (const void*)k_cg_tile<NP, RB, TR>;
  else
    return (const void*)k_cg_tilemx<NP, RB, TR, V == 2>;
}
template <int NP, int RB, int V>
constexpr size_t tile_lds() {
  if constexpr (V == 0)
    return sizeof(TLds<NP, RB>);
  else
    return sizeof(TLdsMx<NP, RB, V == 2>);
}

template <int NP, int RB, int V>
int tile_coresident_one() {
  int dev = 0, cus = 0, per = 0, per_tr = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t sh = tile_lds<NP, RB, V>();
  const void* f0 = tile_fn<NP, RB, V, false>();
  const void* f1 = tile_fn<NP, RB, V, true>();
  if (hipFuncSetAttribute(f0, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess ||
      hipFuncSetAttribute(f1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f0, kBlock, sh) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_tr, f1, kBlock, sh) != hipSuccess)
    return 0;
  return (per < per_tr ? per : per_tr) * cus;
}

template <int NP, int RB, int V>
hipError_t launch_tile_one(const CGArgs<float>& a, hipStream_t s) {
  const size_t words = tile_words(NP, a.tNG, a.tnblk);
  hipLaunchKernelGGL(k_zero_words, dim3(1024), dim3(kBlock), 0, s, a.txp, words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_gather<NP>, dim3((a.m + 15) / 16), dim3(kBlock), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const void* fn = a.trace ? tile_fn<NP, RB, V, true>() : tile_fn<NP, RB, V, false>();
  const size_t sh = tile_lds<NP, RB, V>();
  if ((e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh)) !=
      hipSuccess)
    return e;
  TileArgs t;
  t.N = a.N;
  t.m = a.m;
  t.NG = a.tNG;
  t.nblk = a.tnblk;
  t.maxit = a.maxit;
  t.want_relres = a.want_relres;
  t.tol = a.tol;
  t.txp = a.txp;
  t.txr = a.txr;
  t.S = a.tS;
  t.rv = a.tR;
  t.D = a.D;
  t.z_out = a.z_out;
  t.iters_out = a.iters_out;
  t.relres_out = a.relres_out;
  t.relres = a.relres;
  t.coli = a.coli;
  t.col = a.col;
  t.Wd = a.Wd;
  t.err = a.err;
  t.census = a.census;
  t.census_ticks = a.census_ticks;
  t.trace = a.trace;
  const dim3 grid(a.tNG * a.tnblk);
  void* args[] = {&t};
  if (!t.census) return hipLaunchCooperativeKernel(fn, grid, dim3(kBlock), args, sh, s);
  return hipLaunchKernel(fn, grid, dim3(kBlock), args, sh, s);
}

template <int NP>
size_t words_np(int NG, int nblk) {
  using C = TC<NP, 128>;
  return (size_t)NG * nblk * C::SLOT + (size_t)NG * C::SLOTR + 1;
}

}  // namespace

int tile_shape(int m, int N, int* NP, int* RB, int* NG, int* nblk) {
  if (N < 2 || N > 128 || m < 1) return 0;
  const int np = N <= 64 ? 64 : 128;
  const int ng = (N + kTW - 1) / kTW;
  // 128-row blocks while they fill at most 256 workgroups, else 256-row blocks
  int rb = 128;
  long nb = ((long)m + rb - 1) / rb;
  if ((long)ng * nb > 256) {
    rb = 256;
    nb = ((long)m + rb - 1) / rb;
  }
  if ((long)ng * nb > kMaxResidentGrid) return 0;
  *NP = np;
  *RB = rb;
  *NG = ng;
  *nblk = (int)nb;
  return 1;
}

template <int V>
int tile_coresident_v(int NP, int RB) {
  if (NP == 64 && RB == 128) return tile_coresident_one<64, 128, V>();
  if (NP == 64 && RB == 256) return tile_coresident_one<64, 256, V>();
  if (NP == 128 && RB == 128) return tile_coresident_one<128, 128, V>();
  if (NP == 128 && RB == 256) return tile_coresident_one<128, 256, V>();
  return 0;
}

int tile_coresident(int NP, int RB, int variant) {
  if (variant == 1) return tile_coresident_v<1>(NP, RB);
  if (variant == 2) return tile_coresident_v<2>(NP, RB);
  return tile_coresident_v<0>(NP, RB);
}

size_t tile_part_words(int NP, int NG, int nblk) {
  return NP == 64 ? (size_t)NG * nblk * TC<64, 128>::SLOT
                  : (size_t)NG * nblk * TC<128, 128>::SLOT;
}

size_t tile_words(int NP, int NG, int nblk) {
  return NP == 64 ? words_np<64>(NG, nblk) : words_np<128>(NG, nblk);
}

template <int V>
hipError_t launch_tile_v(const CGArgs<float>& a, int NP, int RB, hipStream_t s) {
  if (NP == 64 && RB == 128) return launch_tile_one<64, 128, V>(a, s);
  if (NP == 64 && RB == 256) return launch_tile_one<64, 256, V>(a, s);
  if (NP == 128 && RB == 128) return launch_tile_one<128, 128, V>(a, s);
  if (NP == 128 && RB == 256) return launch_tile_one<128, 256, V>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_cg_tile(const CGArgs<float>& a, int NP, int RB, int variant, hipStream_t s) {
  if (variant == 1) return launch_tile_v<1>(a, NP, RB, s);
  if (variant == 2) return launch_tile_v<2>(a, NP, RB, s);
  return launch_tile_v<0>(a, NP, RB, s);
}

}  // namespace cgd
