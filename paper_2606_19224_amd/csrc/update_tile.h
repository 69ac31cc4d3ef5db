// Ensemble update tile on the 16x16x4 MFMA (gfx950), shared by the update
// kernel and the solvers that apply the update themselves.
//
// X_a = X_f + A' W' with
//   mode 0: A' = X_f - xbar 1^T, W' = W         (Algorithm 1, W = S^T Z/(N-1))
//   mode 1: A' = X_f,            W' = W - I     (Algorithm 2: X_f W = X_f + X_f (W - I))
// so that the product carries only the increment.  A tile is RB whole rows
// (64 unless a launch wants more, smaller tiles): A' (RB x NP) and W'^T
// (NP x NP) sit in LDS, each wave computes 16x16 output tiles with the
// summation index split into contiguous runs per lane group (a permutation
// of the sum), then adds X_f, which the same thread re-reads (before its
// products) for exactly the elements it writes, so X_a may alias X_f.
#pragma once

#include "mfma_util.h"

namespace cgd {
namespace {

template <typename T, int NP, int RB = 64>
struct UCfg {
  static_assert(RB % 16 == 0, "RB");
  static constexpr int RBX = RB;
  static constexpr int PAD = 16 / (int)sizeof(T);
  static constexpr int LD = NP + PAD;
  static constexpr int TJ = NP / 16, TI = RBX / 16, NT = TI * TJ;
  static constexpr int KQ = NP / 4;
  // As [RBX][LD], Wt [NP][LD], mean [RBX]
  static constexpr size_t lds = sizeof(T) * (size_t)(RBX + NP) * LD + sizeof(double) * RBX;
  // the streaming form in mode 0 adds the exact copy Xr [RBX][LD]
  static constexpr size_t lds_xr = lds + sizeof(T) * (size_t)RBX * LD;
};

// Wt[j][k] = W'[k][j] for k, j < NP (zero outside N x N).  Each thread
// issues up to U loads before its first store, so the loads' latency is paid
// a few times per workgroup rather than once per element.
template <typename T, int NP, int BS>
__device__ inline void update_load_w(int N, const double* Wd, int mode, T* Wt) {
  using C = UCfg<T, NP>;
  constexpr int U = 16;
  for (int e0 = 0; e0 < NP * NP; e0 += BS * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * BS + (int)threadIdx.x;
      const int kk = e / NP, j = e - kk * NP;
      v[u] = (e < NP * NP && kk < N && j < N) ? Wd[(size_t)kk * N + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * BS + (int)threadIdx.x;
      const int kk = e / NP, j = e - kk * NP;
      if (e < NP * NP) {
        double x = v[u];
        if (mode == 1 && kk == j && j < N) x -= 1.0;
        Wt[j * C::LD + kk] = (T)x;
      }
    }
  }
}

// First half of a tile: rows i0 .. i0+RB-1 of A' into As (fewer at the end),
// which needs no W, so a caller may run it while W is still on its way.
// Ends with a barrier.
template <typename T, int NP, int BS, int RB = 64>
__device__ inline void update_tile_load(int n, int N, const T* Xf, int mode, int i0, T* As,
                                        double* mean) {
  using C = UCfg<T, NP, RB>;
  using V = typename Vec4<T>::type;
  constexpr int NW = BS / 64, TPW = (C::NT + NW - 1) / NW;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int rows = min(C::RBX, n - i0);
  // up to 16 loads in flight per thread before the first store
  constexpr int U = 16;
  for (int e0 = 0; e0 < C::RBX * NP; e0 += BS * U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * BS + tid, i = e / NP, j = e - i * NP;
      v[u] = (e < C::RBX * NP && i < rows && j < N) ? Xf[(size_t)(i0 + i) * N + j] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * BS + tid, i = e / NP, j = e - i * NP;
      if (e < C::RBX * NP) As[i * C::LD + j] = v[u];
    }
  }
  __syncthreads();
  if (mode == 0) {
    // row means: 8 lanes per row, each a strided part, then a DPP tree
    for (int i0 = 0; i0 < C::RBX; i0 += BS / 8) {
      const int i = i0 + tid / 8, q = tid % 8;
      double sum = 0.0;
      if (i < C::RBX)
        for (int j = q; j < N; j += 8) sum += (double)As[i * C::LD + j];
      sum = group_sum<8>(sum);
      if (q == 0 && i < C::RBX) mean[i] = sum / N;
    }
    __syncthreads();
    for (int e = tid; e < C::RBX * NP; e += BS) {
      const int i = e / NP, j = e - i * NP;
      if (i < rows && j < N) As[i * C::LD + j] = (T)((double)As[i * C::LD + j] - mean[i]);
    }
    __syncthreads();
  }
}

// Second half: X_a rows i0 .. i0+RB-1 = X_f + A' W' from As and Wt.  Wt must
// be complete and ordered by a barrier since it was written.  Ends with a
// barrier, so the LDS may be reused for the next tile.
template <typename T, int NP, int BS, int RB = 64>
__device__ inline void update_tile_apply(int n, int N, const T* Xf, T* Xa, int i0, const T* As,
                                         const T* Wt) {
  using C = UCfg<T, NP, RB>;
  using V = typename Vec4<T>::type;
  constexpr int NW = BS / 64, TPW = (C::NT + NW - 1) / NW;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int rows = min(C::RBX, n - i0);
  // this thread's elements of X_f for all of its tiles, requested before the
  // first product so that their latency overlaps all of them; every element
  // is read before any is written, so X_a may still alias X_f
  T xf[TPW][4];
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    const int t = wv + NW * s;
    const int ti = t / C::TJ, tj = t - ti * C::TJ, col = tj * 16 + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = ti * 16 + frag_row<T>(lk, i);
      xf[s][i] = (t < C::NT && row < rows && col < N) ? Xf[(size_t)(i0 + row) * N + col] : (T)0;
    }
  }
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    const int t = wv + NW * s;
    if (t < C::NT) {
      const int ti = t / C::TJ, tj = t - ti * C::TJ;
      const int col = tj * 16 + lr;
      T av[C::KQ], bv[C::KQ];
      vload<C::KQ>(As + (ti * 16 + lr) * C::LD + lk * C::KQ, av);
      vload<C::KQ>(Wt + (tj * 16 + lr) * C::LD + lk * C::KQ, bv);
      // four independent accumulation chains, added at the end, so that
      // consecutive MFMAs do not wait on each other
      constexpr int CH = C::KQ >= 4 ? 4 : 1;
      V part[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) part[q] = V{0, 0, 0, 0};
#pragma unroll
      for (int u = 0; u < C::KQ; ++u) part[u % CH] = mfma4(av[u], bv[u], part[u % CH]);
      V acc = part[0];
#pragma unroll
      for (int q = 1; q < CH; ++q) acc += part[q];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = ti * 16 + frag_row<T>(lk, i);
        if (row < rows && col < N)
          Xa[(size_t)(i0 + row) * N + col] = (T)((double)xf[s][i] + (double)acc[i]);
      }
    }
  }
  __syncthreads();
}

// Streaming form for a persistent workgroup that owns every gridDim.x-th tile
// (the single-analysis updates): the next tile's rows of X_f are requested
// into registers before the current tile's products, so that their latency
// overlaps the MFMA work, and go into As once the products are done (the
// apply ends with a barrier).  Wt must be written before the call; the first
// barrier here orders it.  X_a may alias X_f: a workgroup reads each of its
// tiles' rows (into As) before it writes them, and no other workgroup
// touches them.
template <typename T, int NP, int BS, int RB>
__device__ __attribute__((always_inline)) inline void update_tile_fetch(int n, int N, const T* Xf, int i0,
                                         T (&al)[RB * NP / BS]) {
  const int tid = threadIdx.x, rows = min(RB, n - i0);
#pragma unroll
  for (int u = 0; u < RB * NP / BS; ++u) {
    const int e = u * BS + tid, i = e / NP, c = e - i * NP;
    al[u] = (i < rows && c < N) ? Xf[(size_t)(i0 + i) * N + c] : (T)0;
  }
}

// Mode 0: subtract the tile's row means (in double) from As.  Starts after a
// barrier that ordered As; ends with a barrier.
template <typename T, int NP, int BS, int RB>
__device__ __attribute__((always_inline)) inline void update_tile_center(int N, int rows, T* As, double* mean) {
  using C = UCfg<T, NP, RB>;
  const int tid = threadIdx.x;
  for (int r0 = 0; r0 < C::RBX; r0 += BS / 8) {
    const int i = r0 + tid / 8, q = tid % 8;
    double sum = 0.0;
    if (i < C::RBX)
      for (int j = q; j < N; j += 8) sum += (double)As[i * C::LD + j];
    sum = group_sum<8>(sum);
    if (q == 0 && i < C::RBX) mean[i] = sum / N;
  }
  __syncthreads();
  for (int e = tid; e < C::RBX * NP; e += BS) {
    const int i = e / NP, j = e - i * NP;
    if (i < rows && j < N) As[i * C::LD + j] = (T)((double)As[i * C::LD + j] - mean[i]);
  }
  __syncthreads();
}

// The apply step of the streaming form: the X_f term of X_a = X_f + A' W'
// comes from the tile's exact copy Xr in LDS (As itself in mode 1, where
// A' = X_f), which keeps the registers free for the next tile's rows.  Ends
// with a barrier.
template <typename T, int NP, int BS, int RB>
__device__ __attribute__((always_inline)) inline void update_tile_apply_lds(int n, int N, T* Xa, int i0, const T* As,
                                             const T* Xr, const T* Wt) {
  using C = UCfg<T, NP, RB>;
  using V = typename Vec4<T>::type;
  constexpr int NW = BS / 64, TPW = (C::NT + NW - 1) / NW;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int rows = min(C::RBX, n - i0);
  // (one output tile at a time: its 32 MFMAs cover its own LDS loads, and the
  // registers stay free for the next tile's rows in flight)
#pragma unroll 1
  for (int s = 0; s < TPW; ++s) {
    const int t = wv + NW * s;
    if (t < C::NT) {
      const int ti = t / C::TJ, tj = t - ti * C::TJ;
      const int col = tj * 16 + lr;
      T av[C::KQ], bv[C::KQ];
      vload<C::KQ>(As + (ti * 16 + lr) * C::LD + lk * C::KQ, av);
      vload<C::KQ>(Wt + (tj * 16 + lr) * C::LD + lk * C::KQ, bv);
      constexpr int CH = C::KQ >= 4 ? 4 : 1;
      V part[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) part[q] = V{0, 0, 0, 0};
#pragma unroll
      for (int u = 0; u < C::KQ; ++u) part[u % CH] = mfma4(av[u], bv[u], part[u % CH]);
      V acc = part[0];
#pragma unroll
      for (int q = 1; q < CH; ++q) acc += part[q];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = ti * 16 + frag_row<T>(lk, i);
        if (row < rows && col < N)
          Xa[(size_t)(i0 + row) * N + col] = (T)((double)Xr[row * C::LD + col] + (double)acc[i]);
      }
    }
  }
  __syncthreads();
}

// Xr: RB x LD for the exact X_f rows in mode 0 (may be As in mode 1).
template <typename T, int NP, int BS, int RB>
__device__ __attribute__((always_inline)) inline void update_tiles_stream(int n, int N, const T* Xf, T* Xa, int mode, T* As,
                                           T* Xr, const T* Wt, double* mean) {
  using C = UCfg<T, NP, RB>;
  constexpr int NAL = RB * NP / BS;
  static_assert(NAL * BS == RB * NP, "tile loads");
  const int tiles = (n + RB - 1) / RB, tid = threadIdx.x;
  int t = blockIdx.x;
  if (t >= tiles) return;
  T al[NAL];
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < NAL; ++u) {
      const int e = u * BS + tid, i = e / NP, c = e - i * NP;
      As[i * C::LD + c] = al[u];
      if (Xr != As) Xr[i * C::LD + c] = al[u];
    }
  };
  update_tile_fetch<T, NP, BS, RB>(n, N, Xf, t * RB, al);
  store();
  __syncthreads();
  if (mode == 0) update_tile_center<T, NP, BS, RB>(N, min(RB, n - t * RB), As, mean);
  for (; t < tiles; t += gridDim.x) {
    const int tn = t + gridDim.x;
    if (tn < tiles) update_tile_fetch<T, NP, BS, RB>(n, N, Xf, tn * RB, al);
    update_tile_apply_lds<T, NP, BS, RB>(n, N, Xa, t * RB, As, Xr, Wt);
    if (tn < tiles) {
      store();
      __syncthreads();
      if (mode == 0) update_tile_center<T, NP, BS, RB>(N, min(RB, n - tn * RB), As, mean);
    }
  }
}

// Rows i0 .. i0+RB-1 of X_a (fewer at the end).  Wt must be complete (the
// first barrier of the load orders it).  Ends with a barrier, so the LDS may
// be reused for the next tile.
template <typename T, int NP, int BS, int RB = 64>
__device__ inline void update_tile(int n, int N, const T* Xf, T* Xa, int mode, int i0, T* As,
                                   const T* Wt, double* mean) {
  update_tile_load<T, NP, BS, RB>(n, N, Xf, mode, i0, As, mean);
  update_tile_apply<T, NP, BS, RB>(n, N, Xf, Xa, i0, As, Wt);
}

}  // namespace
}  // namespace cgd
