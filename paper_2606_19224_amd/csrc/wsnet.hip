// Learned warm start for the CG (gfx950): a 4-layer circular conv1d network
// over the observation chain, BF16 operands on the 16x16x32 MFMA with FP32
// accumulation, trained by the kernels below (forward, backward, Adam with
// FP32 master weights).
//
// Every convolution is an implicit GEMM: for a tile of 64 observation
// positions, out[i][o] = sum over k = (t, c) of x[i + t - 2][c] * W[o][t][c]
// (circular in i).  A workgroup stages the input rows of its tile (with the
// 2+2 halo) and the whole weight tensor in LDS; each wave computes 16x16
// output tiles, each lane feeding 8 consecutive k values of the same tap per
// MFMA (any bijection of k onto lanes gives the same sum, as long as both
// operands use it).  The backward pass over the data is the same kernel with
// the weights transposed and their taps reversed; the weight gradient is a
// GEMM over positions with per-workgroup partials summed in a fixed order.
//
// Layouts: activations [B][M][C] in BF16 (channels innermost, C padded to 16
// or 64); master parameters FP32 in the oracle's order (per layer W[o][c][t]
// then b[o]); packed BF16 weights [C_out][TP][C_in] with TP taps (5, or 6
// when C_in = 16 so that TP*C_in is a multiple of 32; the extra tap is zero).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "mfma_util.h"
#include "wsnet_internal.h"

namespace cgd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;     // positions per conv workgroup
constexpr int kWP = 128;      // positions per weight-gradient workgroup

__device__ inline f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int CIN>
constexpr int taps_pad() { return CIN == 16 ? 6 : 5; }

// ---------------------------------------------------------------------------
// conv: MODE 0 forward + bias + ReLU (BF16 out), MODE 1 forward + bias, FP32
// output of channel 0 only (last layer), MODE 2 backward over the data:
// no bias, output multiplied by [mask > 0] (ReLU derivative of the layer
// input), BF16 out.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(int M, const __bf16* __restrict__ in,
                                              const __bf16* __restrict__ W,
                                              const float* __restrict__ bias,
                                              const __bf16* __restrict__ mask, void* out) {
  constexpr int TP = taps_pad<CIN>();
  constexpr int K = TP * CIN;              // multiple of 32
  constexpr int ROWS = kTile + TP - 1;     // staged input rows
  constexpr int LDX = CIN + 8;             // padded row strides (16-byte aligned)
  constexpr int LDW = K + 8;
  constexpr int TO = COUT / 16, NT = 4 * TO, TPW = NT / 4;
  __shared__ __align__(16) __bf16 xs[ROWS * LDX];
  __shared__ __align__(16) __bf16 ws[COUT * LDW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15, lg = lane >> 4;
  const int b = blockIdx.y, i0 = blockIdx.x * kTile;
  const __bf16* inb = in + (size_t)b * M * CIN;
  // stage input rows i0-2 .. i0+kTile+TP-4 (circular), 8 channels per copy
  for (int e = tid; e < ROWS * (CIN / 8); e += 256) {
    const int r = e / (CIN / 8), c8 = e - r * (CIN / 8);
    int pos = i0 - 2 + r;
    pos %= M;
    if (pos < 0) pos += M;
    *reinterpret_cast<bf16x8*>(xs + r * LDX + c8 * 8) =
        *reinterpret_cast<const bf16x8*>(inb + (size_t)pos * CIN + c8 * 8);
  }
  for (int e = tid; e < COUT * (K / 8); e += 256) {
    const int o = e / (K / 8), k8 = e - o * (K / 8);
    *reinterpret_cast<bf16x8*>(ws + o * LDW + k8 * 8) =
        *reinterpret_cast<const bf16x8*>(W + (size_t)o * K + k8 * 8);
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    const int tile = wv + 4 * s;
    const int ti = tile / TO, to = tile - ti * TO;
    f32x4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < K / 32; ++ks) {
      const int k0 = ks * 32 + 8 * lg;
      const int t = k0 / CIN, c = k0 - t * CIN;
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(xs + (ti * 16 + lr + t) * LDX + c);
      const bf16x8 w = *reinterpret_cast<const bf16x8*>(ws + (to * 16 + lr) * LDW + k0);
      acc = mfma_bf16(a, w, acc);
    }
    const int ch = to * 16 + lr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int pos = i0 + ti * 16 + 4 * lg + q;
      if (pos >= M) continue;
      float v = acc[q];
      if constexpr (MODE == 0) {
        v += bias[ch];
        v = v > 0.f ? v : 0.f;
        ((__bf16*)out)[((size_t)b * M + pos) * COUT + ch] = (__bf16)v;
      } else if constexpr (MODE == 1) {
        if (ch == 0) ((float*)out)[(size_t)b * M + pos] = v + bias[0];
      } else {
        const float mk = (float)mask[((size_t)b * M + pos) * COUT + ch];
        ((__bf16*)out)[((size_t)b * M + pos) * COUT + ch] = (__bf16)(mk > 0.f ? v : 0.f);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient partials: part[wg][o][t][c] = sum over the workgroup's
// positions p of g[p][o] * x[p + t - 2][c];  bpart[wg][o] = sum_p g[p][o].
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(int M, const __bf16* __restrict__ x,
                                               const __bf16* __restrict__ g,
                                               float* __restrict__ part,
                                               float* __restrict__ bpart) {
  constexpr int TP = taps_pad<CIN>();
  constexpr int LDG = kWP + 8;
  constexpr int LDI = kWP + 8 + 8;            // kWP + TP - 1 staged positions, padded
  constexpr int TO = COUT / 16, TC = TP * CIN / 16, NT = TO * TC;
  __shared__ __align__(16) __bf16 gT[COUT * LDG];
  __shared__ __align__(16) __bf16 xT[CIN * LDI];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15, lg = lane >> 4;
  const int b = blockIdx.y, p0 = blockIdx.x * kWP;
  const int wg = blockIdx.y * gridDim.x + blockIdx.x;
  const int np = min(kWP, M - p0);
  const __bf16* gb = g + (size_t)b * M * COUT;
  const __bf16* xb = x + (size_t)b * M * CIN;
  for (int e = tid; e < kWP * COUT; e += 256) {
    const int p = e / COUT, o = e - p * COUT;
    gT[o * LDG + p] = p < np ? gb[(size_t)(p0 + p) * COUT + o] : (__bf16)0.f;
  }
  for (int e = tid; e < (kWP + TP - 1) * CIN; e += 256) {
    const int j = e / CIN, c = e - j * CIN;
    int pos = p0 - 2 + j;
    pos %= M;
    if (pos < 0) pos += M;
    xT[c * LDI + j] = xb[(size_t)pos * CIN + c];
  }
  __syncthreads();
  float* pw = part + (size_t)wg * COUT * TP * CIN;
  for (int tile = wv; tile < NT; tile += 4) {
    const int to = tile / TC, tc = tile - to * TC;
    const int t = (tc * 16) / CIN, c0 = (tc * 16) - t * CIN;
    f32x4 acc = {0, 0, 0, 0};
#pragma unroll 2
    for (int ks = 0; ks < kWP / 32; ++ks) {
      const int pk = ks * 32 + 8 * lg;
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(gT + (to * 16 + lr) * LDG + pk);
      bf16x8 bb;
      const __bf16* src = xT + (c0 + lr) * LDI + pk + t;
#pragma unroll
      for (int q = 0; q < 8; ++q) bb[q] = src[q];
      acc = mfma_bf16(a, bb, acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = to * 16 + 4 * lg + q;
      pw[((size_t)o * TP + t) * CIN + c0 + lr] = acc[q];
    }
  }
  if (tid < COUT) {
    float s = 0.f;
    for (int p = 0; p < kWP; ++p) s += (float)gT[tid * LDG + p];
    bpart[(size_t)wg * COUT + tid] = s;
  }
}

// Sum of the partials in a fixed order into the FP32 gradient (oracle layout:
// W[o][c][t] for the true sizes, then b[o]).
template <int CIN, int COUT>
__global__ void k_wgrad_reduce(int nwg, int cin, int cout, const float* part, const float* bpart,
                               float* grad) {
  constexpr int TP = taps_pad<CIN>();
  const int nw = cout * cin * 5;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nw) {
    const int o = e / (cin * 5), r = e - o * cin * 5, c = r / 5, t = r - c * 5;
    double s = 0.0;
    for (int w = 0; w < nwg; ++w) s += part[(((size_t)w * COUT + o) * TP + t) * CIN + c];
    grad[e] = (float)s;
  } else if (e < nw + cout) {
    const int o = e - nw;
    double s = 0.0;
    for (int w = 0; w < nwg; ++w) s += bpart[(size_t)w * COUT + o];
    grad[e] = (float)s;
  }
}

// ---------------------------------------------------------------------------
// features, loss, Adam, packing
// ---------------------------------------------------------------------------
// [B][M][4] FP32 features -> [B][M][16] BF16 (channels 3..15 zero)
__global__ void k_feat_to_act(int BM, const float* feat, __bf16* a0) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= BM * 16) return;
  const int p = e >> 4, c = e & 15;
  a0[e] = (__bf16)(c < 3 ? feat[(size_t)p * 4 + c] : 0.f);
}

// g4[b][i][0] = 2 (out - target)/(B M), other channels 0; per-sample squared
// error sums into lpart[b] (double).
__global__ void k_loss(int M, float scale, const float* out, const float* target, __bf16* g4,
                       double* lpart) {
  __shared__ double red[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < M; i += 256) {
    const size_t e = (size_t)b * M + i;
    const float d = out[e] - target[e];
    s += (double)d * d;
    __bf16* gp = g4 + e * 16;
    gp[0] = (__bf16)(2.f * d * scale);
#pragma unroll
    for (int c = 1; c < 16; ++c) gp[c] = (__bf16)0.f;
  }
  red[tid] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) red[tid] += red[tid + k];
    __syncthreads();
  }
  if (tid == 0) lpart[b] = red[0];
}

__global__ void k_loss_final(int B, double count, const double* lpart, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += lpart[b];
    *loss = (float)(s / count);
  }
}

__global__ void k_adam(int n, float* p, float* m, float* v, const float* g, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Packed BF16 weights of one layer: forward Wf[o][t][c] (COUTP x TPF x CINP)
// and backward-data Wb[c][t'][o] = W[o][c][4 - t'] (CINP x TPB x COUTP); FP32
// bias padded to COUTP.
__global__ void k_pack(int cin, int cout, int CINP, int COUTP, int TPF, int TPB, const float* w,
                       const float* bias, __bf16* Wf, __bf16* Wb, float* biasp) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nf = COUTP * TPF * CINP, nb = CINP * TPB * COUTP;
  if (e < nf) {
    const int o = e / (TPF * CINP), r = e - o * TPF * CINP, t = r / CINP, c = r - t * CINP;
    const float v = (o < cout && c < cin && t < 5) ? w[((size_t)o * cin + c) * 5 + t] : 0.f;
    Wf[e] = (__bf16)v;
  } else if (e < nf + nb) {
    const int f = e - nf;
    const int c = f / (TPB * COUTP), r = f - c * TPB * COUTP, t = r / COUTP, o = r - t * COUTP;
    const float v = (o < cout && c < cin && t < 5) ? w[((size_t)o * cin + c) * 5 + (4 - t)] : 0.f;
    Wb[f] = (__bf16)v;
  } else if (e < nf + nb + COUTP) {
    const int o = e - nf - nb;
    biasp[o] = o < cout ? bias[o] : 0.f;
  }
}

// Features from the analysis inputs.  Rows pass: D[i][j] (FP32, row-major m x
// N), var[i] = sum_j S_ij^2/(N-1) with HX in double, and per-block column
// sums of D^2 (double).
__global__ void k_feat_rows(int n, int m, int N, int k, const float* Xf, const int32_t* idx,
                            const float* hw, const float* y, const float* eps, float* D,
                            float* var, double* cpart, int rows_per_block, int* err) {
  extern __shared__ double fsh[];  // rows_per_block * N HX values, then N column sums
  const int tid = threadIdx.x, i0 = blockIdx.x * rows_per_block;
  const int rows = min(rows_per_block, m - i0);
  double* hx = fsh;
  for (int e = tid; e < rows * N; e += blockDim.x) {
    const int i = i0 + e / N, j = e % N;
    double h = 0.0;
    for (int t = 0; t < k; ++t) {
      const int c = idx[(size_t)i * k + t];
      if ((unsigned)c < (unsigned)n)
        h += (double)hw[(size_t)i * k + t] * (double)Xf[(size_t)c * N + j];
      else
        atomicOr(err, 2);
    }
    hx[e] = h;
    double d = (double)y[i] - h;
    if (eps) d += (double)eps[(size_t)i * N + j];
    D[(size_t)i * N + j] = (float)d;
  }
  __syncthreads();
  for (int r = tid; r < rows; r += blockDim.x) {
    double mu = 0.0;
    for (int j = 0; j < N; ++j) mu += hx[r * N + j];
    mu /= N;
    double s2 = 0.0;
    for (int j = 0; j < N; ++j) {
      const double sv = hx[r * N + j] - mu;
      s2 += sv * sv;
    }
    var[i0 + r] = (float)(s2 / (N - 1));
  }
  for (int j = tid; j < N; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) {
      const double d = (double)D[(size_t)(i0 + r) * N + j];
      s += d * d;
    }
    cpart[(size_t)blockIdx.x * N + j] = s;
  }
}

// s_j = RMS of d_j over the m observations from the block partials of
// sum_i d_ij^2: lane l adds blocks l, l + 64, ... in order, then a fixed lane
// tree; called by one whole wavefront, every lane gets the same value (1 if
// the column is zero).  The feature pass and the fused inference share it.
__device__ inline float member_rms(const double* cpart, int nblk, int N, int j, int m) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += cpart[(size_t)b * N + j];
  s = group_sum<16>(s);
  s = (__shfl(s, 0) + __shfl(s, 16)) + (__shfl(s, 32) + __shfl(s, 48));
  double rms = sqrt(s / m);
  if (!(rms > 0.0)) rms = 1.0;
  return (float)rms;
}

// Column pass: s_j = RMS of d_j, then feat[j][i] = (d_ij / s_j, var_i, r_i, 0).
__global__ void k_feat_cols(int m, int N, int nblk, const float* D, const float* var,
                            const float* rdiag, const double* cpart, float* feat, float* scale) {
  __shared__ float s_sh;
  const int j = blockIdx.x, tid = threadIdx.x;
  if (tid < 64) {
    const float rms = member_rms(cpart, nblk, N, j, m);
    if (tid == 0) {
      s_sh = rms;
      scale[j] = rms;
    }
  }
  __syncthreads();
  const float inv = 1.f / s_sh;
  for (int i = tid; i < m; i += blockDim.x) {
    float* f = feat + ((size_t)j * m + i) * 4;
    f[0] = D[(size_t)i * N + j] * inv;
    f[1] = var[i];
    f[2] = rdiag[i];
    f[3] = 0.f;
  }
}

// Training target of member j at observation i: Z[i][j] / s_j, laid out
// [N][m] like the network output.
__global__ void k_target(int m, int N, const float* Z, const float* scale, float* target) {
  const long total = (long)m * N;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / m), i = (int)(e - (long)j * m);
    target[e] = Z[(size_t)i * N + j] / scale[j];
  }
}

// Jacobi start z0[i][j] = d_ij / Psi_ii from the features: d_ij = s_j f0 and
// Psi_ii = (S S^T)_ii/(N-1) + r_i = f1 + f2.
__global__ void k_jacobi_z0(int m, int N, const float* feat, const float* scale, float* z0) {
  const long total = (long)m * N;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e - (long)i * N);
    const float* f = feat + ((size_t)j * m + i) * 4;
    z0[e] = scale[j] * f[0] / (f[1] + f[2]);
  }
}

// ---------------------------------------------------------------------------
// Inference in two launches: the rows pass below (which also converts the
// forward weights), then k_infer, which runs all four layers of a tile of
// positions of one member on chip.
// ---------------------------------------------------------------------------

// Forward weights and biases of the four layers to convert in the rows launch
// (Wf[o][t][c], COUTP x TPF x CINP BF16, and the bias padded to COUTP).
struct FwdPack {
  const float* params;
  __bf16* Wf[4];
  float* bias[4];
  int off[4], cin[4], cout[4], cinp[4], coutp[4], tpf[4];
  int start[5];  // running element counts (weights, then bias) per layer
};

__device__ inline void pack_forward(const FwdPack& P, int e) {
  int l = 0;
  while (l < 3 && e >= P.start[l + 1]) ++l;
  e -= P.start[l];
  const int nf = P.coutp[l] * P.tpf[l] * P.cinp[l];
  const float* w = P.params + P.off[l];
  if (e < nf) {
    const int o = e / (P.tpf[l] * P.cinp[l]), r = e - o * P.tpf[l] * P.cinp[l];
    const int t = r / P.cinp[l], c = r - t * P.cinp[l];
    const float v = (o < P.cout[l] && c < P.cin[l] && t < 5) ? w[((size_t)o * P.cin[l] + c) * 5 + t]
                                                           : 0.f;
    P.Wf[l][e] = (__bf16)v;
  } else {
    const int o = e - nf;
    P.bias[l][o] = o < P.cout[l] ? w[(size_t)P.cout[l] * P.cin[l] * 5 + o] : 0.f;
  }
}

// Rows pass for N <= 128 (NP = 32, 64 or 128): NP/4 lanes per observation
// row, four members each.  D[i][j] = y_i + eps_ij - HX_ij (FP32), var_i =
// sum_j (HX_ij - mean_i)^2/(N-1) with HX in double, and per-workgroup column
// sums of D^2 (double, of the FP32-rounded D) in cpart[blockIdx][j].
// Workgroups past the nrb row workgroups convert the forward weights.
template <int NP>
__global__ __launch_bounds__(256) void k_feat_rows2(int n, int m, int N, int k, const float* Xf,
                                                    const int32_t* idx, const float* hw,
                                                    const float* y, const float* eps, float* D,
                                                    float* var, double* cpart, int* err, int nrb,
                                                    FwdPack pk) {
  constexpr int LPR = NP / 4, RPB = 256 / LPR;
  __shared__ double colsq[RPB][NP];
  const int tid = threadIdx.x;
  if ((int)blockIdx.x >= nrb) {
    const int e = ((int)blockIdx.x - nrb) * 256 + tid;
    if (e < pk.start[4]) pack_forward(pk, e);
    return;
  }
  const int q = tid % LPR, rr = tid / LPR, i = blockIdx.x * RPB + rr;
  const bool live = i < m;
  double yv = 0.0, ev[4] = {0.0, 0.0, 0.0, 0.0}, h[4] = {0.0, 0.0, 0.0, 0.0};
  if (live) {
    yv = (double)y[i];
    if (eps) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * q + u < N) ev[u] = (double)eps[(size_t)i * N + 4 * q + u];
    }
    for (int t = 0; t < k; ++t) {
      const int c = idx[(size_t)i * k + t];
      if ((unsigned)c >= (unsigned)n) {
        if (q == 0) atomicOr(err, 2);
        continue;
      }
      const double wt = (double)hw[(size_t)i * k + t];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * q + u < N) h[u] += wt * (double)Xf[(size_t)c * N + 4 * q + u];
    }
  }
  const double mu = group_sum<LPR>((h[0] + h[1]) + (h[2] + h[3])) / N;
  double s2 = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (4 * q + u < N) s2 += (h[u] - mu) * (h[u] - mu);
  s2 = group_sum<LPR>(s2);
  if (live && q == 0) var[i] = (float)(s2 / (N - 1));
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = 4 * q + u;
    double dsq = 0.0;
    if (live && j < N) {
      const float d = (float)(yv - h[u] + ev[u]);
      D[(size_t)i * N + j] = d;
      dsq = (double)d * (double)d;
    }
    colsq[rr][j] = dsq;
  }
  __syncthreads();
  if (tid < N) {
    double sum = 0.0;
    for (int r = 0; r < RPB; ++r) sum += colsq[r][tid];
    cpart[(size_t)blockIdx.x * N + tid] = sum;
  }
}

// Fused inference of the warm-start network: z0[i][j] = s_j * net(features)_i
// for every member j and observation i, in one persistent launch.  A work item
// is T consecutive positions of one member; workgroup g takes a contiguous
// range of items (so mostly one member, whose scale it computes once).
// Activations stay in LDS as BF16 rows of 16 (features) or 64 channels; a
// layer's output rows reach 2 positions further out per remaining layer, so
// an item's input carries 8 positions of circular halo per side:
//   features  rows r <-> position i0 - 8 + r   (buffer Y)
//   layer 0   rows r <-> position i0 - 6 + r   (X)
//   layer 1   rows r <-> position i0 - 4 + r   (Y)
//   layer 2   rows r <-> position i0 - 2 + r   (X)
//   layer 3   row  r <-> position i0 + r       (z0)
// Each product is the same sequence of 16x16x32 MFMAs as the per-layer
// convolution (same operands, same order), so the result is bitwise that of
// features -> forward -> scale.  All four layers' weights are staged in LDS
// once per workgroup; each wave keeps the fragments of its two 16-channel
// output tiles of the two 64-channel layers in registers for the whole launch
// (the small first and last layers take theirs from LDS per item) and walks
// row tiles, so the products read only the activations from LDS.
constexpr int kInfTile = 128;  // positions per inference work item

template <int T>
struct InfCfg {
  static constexpr int RT = (T + 12 + 15) / 16;   // row tiles of layers 0-2
  static constexpr int ROWS = RT * 16 + 16;       // staged rows (zero beyond the data)
  static constexpr int LD16 = 16 + 8, LD64 = 64 + 8;
  static constexpr int K0 = 6 * 16, K1 = 5 * 64;  // packed widths (layers 1-3 share K1)
  static constexpr int LW0 = K0 + 8, LW1 = K1 + 8;
  static constexpr size_t act = 2 * (size_t)ROWS * LD64;  // X and Y, BF16 elements
  static constexpr size_t wts = 64 * (size_t)LW0 + 2 * 64 * (size_t)LW1 + 16 * (size_t)LW1;
  static constexpr size_t lds = sizeof(__bf16) * (act + wts);
};

template <int CIN, int COUT>
struct LayerW {
  static constexpr int TP = taps_pad<CIN>(), K = TP * CIN, KS = K / 32, TO = COUT / 16;
  static constexpr int CPW = TO >= 2 ? 2 : 1;     // output tiles per wave
  static constexpr int RG = 8 / (TO / CPW);       // row groups
  bf16x8 f[CPW][KS];
  // this wave's fragments of W[o][k] (rows of stride ldw)
  __device__ inline void load(const __bf16* W, int ldw, int wv, int lane) {
    const int lr = lane & 15, lg = lane >> 4, cp = wv % (TO / CPW);
#pragma unroll
    for (int x = 0; x < CPW; ++x)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        f[x][ks] = *reinterpret_cast<const bf16x8*>(
            W + (size_t)((cp * CPW + x) * 16 + lr) * ldw + ks * 32 + 8 * lg);
  }
};

// One layer from LDS rows xin (stride LDI) to LDS rows xout (stride LDO), bias
// and ReLU, over RT row tiles.
template <int CIN, int COUT, int LDI, int LDO, int RT>
__device__ inline void infer_layer(const LayerW<CIN, COUT>& W, const __bf16* xin, __bf16* xout,
                                   const float* bias, int wv, int lane) {
  using L = LayerW<CIN, COUT>;
  const int lr = lane & 15, lg = lane >> 4, cp = wv % (L::TO / L::CPW), rg = wv / (L::TO / L::CPW);
  float bv[L::CPW];
#pragma unroll
  for (int x = 0; x < L::CPW; ++x) bv[x] = bias[(cp * L::CPW + x) * 16 + lr];
  for (int ti = rg; ti < RT; ti += L::RG) {
    f32x4 acc[L::CPW];
#pragma unroll
    for (int x = 0; x < L::CPW; ++x) acc[x] = f32x4{0, 0, 0, 0};
    // every A fragment of the row tile in flight before the first product
    bf16x8 av[L::KS];
#pragma unroll
    for (int ks = 0; ks < L::KS; ++ks) {
      const int k0 = ks * 32 + 8 * lg, t = k0 / CIN, c = k0 - t * CIN;
      av[ks] = *reinterpret_cast<const bf16x8*>(xin + (ti * 16 + lr + t) * LDI + c);
    }
#pragma unroll
    for (int ks = 0; ks < L::KS; ++ks)
#pragma unroll
      for (int x = 0; x < L::CPW; ++x) acc[x] = mfma_bf16(av[ks], W.f[x][ks], acc[x]);
    // keep the loads ahead of the products (LDS reads, then MFMAs)
    __builtin_amdgcn_sched_group_barrier(0x100, L::KS, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, L::KS * L::CPW, 0);
#pragma unroll
    for (int x = 0; x < L::CPW; ++x) {
      const int ch = (cp * L::CPW + x) * 16 + lr;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        float v = acc[x][qq] + bv[x];
        v = v > 0.f ? v : 0.f;
        xout[(ti * 16 + 4 * lg + qq) * LDO + ch] = (__bf16)v;
      }
    }
  }
}

struct InferArgs {
  int m, N, nblk, tiles, per;  // tiles per member, items per workgroup
  const float* D;
  const float* var;
  const float* rdiag;
  const double* cpart;
  const __bf16* W[4];
  const float* bias[4];
  float* z0;
};

template <int T>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_infer(InferArgs a) {
  using C = InfCfg<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* X = (__bf16*)smem_raw;                 // ROWS x LD64
  __bf16* Y = X + (size_t)C::ROWS * C::LD64;     // ROWS x LD64; the features (LD16) first
  __bf16* W0s = X + C::act;                      // 64 x LW0
  __bf16* W1s = W0s + 64 * C::LW0;               // 64 x LW1
  __bf16* W2s = W1s + 64 * C::LW1;               // 64 x LW1
  __bf16* W3s = W2s + 64 * C::LW1;               // 16 x LW1
  __shared__ float s_sh;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = a.m, N = a.N;
  const int it0 = blockIdx.x * a.per, it1 = min(it0 + a.per, a.tiles * N);
  if (it0 >= it1) return;
  {
    const __bf16* src[4] = {a.W[0], a.W[1], a.W[2], a.W[3]};
    __bf16* dst[4] = {W0s, W1s, W2s, W3s};
    const int rows[4] = {64, 64, 64, 16}, kk[4] = {C::K0, C::K1, C::K1, C::K1};
    const int ld[4] = {C::LW0, C::LW1, C::LW1, C::LW1};
#pragma unroll
    for (int l = 0; l < 4; ++l)
      for (int e = tid; e < rows[l] * (kk[l] / 8); e += 512) {
        const int o = e / (kk[l] / 8), k8 = e - o * (kk[l] / 8);
        *reinterpret_cast<bf16x8*>(dst[l] + o * ld[l] + k8 * 8) =
            *reinterpret_cast<const bf16x8*>(src[l] + (size_t)o * kk[l] + k8 * 8);
      }
  }
  // rows of X and Y past the computed tiles stay zero (the taps of the rows
  // past the halo read them); the features use Y's first ROWS x LD16 only
  for (int e = tid; e < 16 * C::LD64 / 8; e += 512) {
    *reinterpret_cast<bf16x8*>(X + (size_t)C::RT * 16 * C::LD64 + e * 8) = bf16x8{};
    *reinterpret_cast<bf16x8*>(Y + (size_t)C::RT * 16 * C::LD64 + e * 8) = bf16x8{};
  }
  __syncthreads();
  // the two 64-channel layers' fragments stay in registers for every item
  LayerW<64, 64> w1, w2;
  w1.load(W1s, C::LW1, wv, lane);
  w2.load(W2s, C::LW1, wv, lane);
  const float b30 = a.bias[3][0];
  static_assert(C::ROWS <= 512, "one staged row per thread");
  // an item's raw feature inputs (thread r holds row r), loaded one item ahead
  auto fetch = [&](int item, float& dv, float& vv, float& rv) {
    dv = vv = rv = 0.f;
    const int j = item / a.tiles, i0 = (item - j * a.tiles) * T;
    if (tid < T + 16) {
      int pos = (i0 - 8 + tid) % m;
      if (pos < 0) pos += m;
      dv = a.D[(size_t)pos * N + j];
      vv = a.var[pos];
      rv = a.rdiag[pos];
    }
  };
  float dv, vv, rv;
  fetch(it0, dv, vv, rv);
  int jprev = -1;
  for (int item = it0; item < it1; ++item) {
    const int j = item / a.tiles, i0 = (item - j * a.tiles) * T;
    if (j != jprev) {
      if (wv == 0) {
        const float rms = member_rms(a.cpart, a.nblk, N, j, m);
        if (lane == 0) s_sh = rms;
      }
      jprev = j;
    }
    __syncthreads();  // s_sh, and the previous item is done with X and Y
    const float sj = s_sh, inv = 1.f / sj;
    // features (d/s, var, r, 0 ...), rows past T + 16 zero
    if (tid < C::ROWS) {
      bf16x8 lo = {}, hi = {};
      if (tid < T + 16) {
        lo[0] = (__bf16)(dv * inv);
        lo[1] = (__bf16)vv;
        lo[2] = (__bf16)rv;
      }
      *reinterpret_cast<bf16x8*>(Y + tid * C::LD16) = lo;
      *reinterpret_cast<bf16x8*>(Y + tid * C::LD16 + 8) = hi;
    }
    if (item + 1 < it1) fetch(item + 1, dv, vv, rv);
    __syncthreads();
    {
      LayerW<16, 64> w0;
      w0.load(W0s, C::LW0, wv, lane);
      infer_layer<16, 64, C::LD16, C::LD64, C::RT>(w0, Y, X, a.bias[0], wv, lane);
    }
    __syncthreads();
    infer_layer<64, 64, C::LD64, C::LD64, C::RT>(w1, X, Y, a.bias[1], wv, lane);
    __syncthreads();
    infer_layer<64, 64, C::LD64, C::LD64, C::RT>(w2, Y, X, a.bias[2], wv, lane);
    __syncthreads();
    // last layer: channel 0 only, no ReLU, z0 = (out + b) * s
    {
      using L = LayerW<64, 16>;
      L w3;
      w3.load(W3s, C::LW1, wv, lane);
      const int lr = lane & 15, lg = lane >> 4;
      for (int ti = wv; ti < T / 16; ti += 8) {
        f32x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < L::KS; ++ks) {
          const int k0 = ks * 32 + 8 * lg, t = k0 / 64, c = k0 - t * 64;
          const bf16x8 av =
              *reinterpret_cast<const bf16x8*>(X + (ti * 16 + lr + t) * C::LD64 + c);
          acc = mfma_bf16(av, w3.f[0][ks], acc);
        }
        if (lr == 0)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int pos = i0 + ti * 16 + 4 * lg + qq;
            if (pos < m) a.z0[(size_t)pos * N + j] = (acc[qq] + b30) * sj;
          }
      }
    }
  }
}

// z0[i][j] = out[j][i] * s_j
__global__ void k_z0(int m, int N, const float* out, const float* scale, float* z0) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * N) return;
  const int i = e / N, j = e - i * N;
  z0[e] = out[(size_t)j * m + i] * scale[j];
}

template <int CIN, int COUT, int MODE>
hipError_t conv(int B, int M, const __bf16* in, const __bf16* W, const float* bias,
                const __bf16* mask, void* out, hipStream_t s) {
  hipLaunchKernelGGL((k_conv<CIN, COUT, MODE>), dim3((M + kTile - 1) / kTile, B), dim3(256), 0,
                     s, M, in, W, bias, mask, out);
  return hipGetLastError();
}

template <int CIN, int COUT>
hipError_t wgrad(int B, int M, const __bf16* x, const __bf16* g, float* part, float* bpart,
                 int cin, int cout, float* grad, hipStream_t s) {
  const int nx = (M + kWP - 1) / kWP;
  hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(nx, B), dim3(256), 0, s, M, x, g, part, bpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int tot = cout * cin * 5 + cout;
  hipLaunchKernelGGL((k_wgrad_reduce<CIN, COUT>), dim3((tot + 255) / 256), dim3(256), 0, s,
                     nx * B, cin, cout, part, bpart, grad);
  return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static const int kCin[4] = {3, 64, 64, 64}, kCout[4] = {64, 64, 64, 1};
static const int kCinP[4] = {16, 64, 64, 64}, kCoutP[4] = {64, 64, 64, 16};

size_t wsnet_param_offset(int layer) {
  size_t o = 0;
  for (int l = 0; l < layer; ++l) o += (size_t)kCout[l] * kCin[l] * 5 + kCout[l];
  return o;
}

size_t wsnet_param_count() { return wsnet_param_offset(4); }

static int tpf(int l) { return kCinP[l] == 16 ? 6 : 5; }
static int tpb(int l) { return kCoutP[l] == 16 ? 6 : 5; }

WsLayout wsnet_layout(int B, int M, int training) {
  WsLayout L;
  memset(&L, 0, sizeof(L));
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (bytes + 255) & ~size_t(255);
    return at;
  };
  for (int l = 0; l < 4; ++l) {
    L.Wf[l] = take(2 * (size_t)kCoutP[l] * tpf(l) * kCinP[l]);
    L.Wb[l] = take(2 * (size_t)kCinP[l] * tpb(l) * kCoutP[l]);
    L.bias[l] = take(4 * (size_t)kCoutP[l]);
  }
  const size_t BM = (size_t)B * M;
  L.act[0] = take(2 * BM * 16);
  for (int l = 1; l < 4; ++l) L.act[l] = take(2 * BM * 64);
  L.out = take(4 * BM);
  if (training) {
    L.g4 = take(2 * BM * 16);
    L.ga = take(2 * BM * 64);
    L.gb = take(2 * BM * 64);
    const size_t nwg = (size_t)B * ((M + kWP - 1) / kWP);
    L.nwg = (int)nwg;
    L.part = take(4 * nwg * 64 * 6 * 64);
    L.bpart = take(4 * nwg * 64);
    L.grad = take(4 * wsnet_param_count());
    L.lpart = take(8 * (size_t)B);
  }
  L.total = o;
  return L;
}

hipError_t wsnet_pack(const float* params, unsigned char* ws, const WsLayout& L, hipStream_t s) {
  for (int l = 0; l < 4; ++l) {
    const float* w = params + wsnet_param_offset(l);
    const float* b = w + (size_t)kCout[l] * kCin[l] * 5;
    const int tot = kCoutP[l] * tpf(l) * kCinP[l] + kCinP[l] * tpb(l) * kCoutP[l] + kCoutP[l];
    hipLaunchKernelGGL(k_pack, dim3((tot + 255) / 256), dim3(256), 0, s, kCin[l], kCout[l],
                       kCinP[l], kCoutP[l], tpf(l), tpb(l), w, b, (__bf16*)(ws + L.Wf[l]),
                       (__bf16*)(ws + L.Wb[l]), (float*)(ws + L.bias[l]));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Forward over packed weights: features [B][M][4] FP32 -> out [B][M] FP32.
hipError_t wsnet_forward(int B, int M, const float* feat, unsigned char* ws, const WsLayout& L,
                         float* out, hipStream_t s) {
  const int BM = B * M;
  hipLaunchKernelGGL(k_feat_to_act, dim3((BM * 16 + 255) / 256), dim3(256), 0, s, BM, feat,
                     (__bf16*)(ws + L.act[0]));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  auto A = [&](int l) { return (__bf16*)(ws + L.act[l]); };
  auto Wf = [&](int l) { return (const __bf16*)(ws + L.Wf[l]); };
  auto Bs = [&](int l) { return (const float*)(ws + L.bias[l]); };
  if ((e = conv<16, 64, 0>(B, M, A(0), Wf(0), Bs(0), nullptr, A(1), s)) != hipSuccess) return e;
  if ((e = conv<64, 64, 0>(B, M, A(1), Wf(1), Bs(1), nullptr, A(2), s)) != hipSuccess) return e;
  if ((e = conv<64, 64, 0>(B, M, A(2), Wf(2), Bs(2), nullptr, A(3), s)) != hipSuccess) return e;
  return conv<64, 16, 1>(B, M, A(3), Wf(3), Bs(3), nullptr, out, s);
}

hipError_t wsnet_loss_grad(int B, int M, const float* params, const float* feat,
                           const float* target, float* loss, float* grad, unsigned char* ws,
                           const WsLayout& L, hipStream_t s) {
  hipError_t e = wsnet_pack(params, ws, L, s);
  if (e != hipSuccess) return e;
  float* out = (float*)(ws + L.out);
  if ((e = wsnet_forward(B, M, feat, ws, L, out, s)) != hipSuccess) return e;
  __bf16* g4 = (__bf16*)(ws + L.g4);
  double* lpart = (double*)(ws + L.lpart);
  hipLaunchKernelGGL(k_loss, dim3(B), dim3(256), 0, s, M, (float)(1.0 / ((double)B * M)), out,
                     target, g4, lpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, B, (double)B * M, lpart, loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  auto A = [&](int l) { return (const __bf16*)(ws + L.act[l]); };
  auto Wb = [&](int l) { return (const __bf16*)(ws + L.Wb[l]); };
  float* part = (float*)(ws + L.part);
  float* bpart = (float*)(ws + L.bpart);
  __bf16* ga = (__bf16*)(ws + L.ga);
  __bf16* gb = (__bf16*)(ws + L.gb);
  auto G = [&](int l) { return grad + wsnet_param_offset(l); };
  // layer 3: input act3, output gradient g4
  if ((e = wgrad<64, 16>(B, M, A(3), g4, part, bpart, 64, 1, G(3), s)) != hipSuccess) return e;
  if ((e = conv<16, 64, 2>(B, M, g4, Wb(3), nullptr, A(3), ga, s)) != hipSuccess) return e;
  // layer 2
  if ((e = wgrad<64, 64>(B, M, A(2), ga, part, bpart, 64, 64, G(2), s)) != hipSuccess) return e;
  if ((e = conv<64, 64, 2>(B, M, ga, Wb(2), nullptr, A(2), gb, s)) != hipSuccess) return e;
  // layer 1
  if ((e = wgrad<64, 64>(B, M, A(1), gb, part, bpart, 64, 64, G(1), s)) != hipSuccess) return e;
  if ((e = conv<64, 64, 2>(B, M, gb, Wb(1), nullptr, A(1), ga, s)) != hipSuccess) return e;
  // layer 0 (no gradient for the input features)
  if ((e = wgrad<16, 64>(B, M, A(0), ga, part, bpart, 3, 64, G(0), s)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t wsnet_train_step(int B, int M, float* params, float* adam_m, float* adam_v, int step,
                            float lr, const float* feat, const float* target, float* loss,
                            unsigned char* ws, const WsLayout& L, hipStream_t s) {
  float* grad = (float*)(ws + L.grad);
  hipError_t e = wsnet_loss_grad(B, M, params, feat, target, loss, grad, ws, L, s);
  if (e != hipSuccess) return e;
  const int np = (int)wsnet_param_count();
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, s, np, params, adam_m, adam_v,
                     grad, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

namespace {

// The rows pass; for N <= 128 with the forward weights converted in the same
// launch when pk.params is set.  Returns the number of row blocks in *nblk.
hipError_t feature_rows(int n, int m, int N, int k, const float* Xf, const int32_t* idx,
                        const float* hw, const float* y, const float* eps, float* Dtmp,
                        float* var, double* cpart, int* err, const FwdPack& pk, int* nblk,
                        hipStream_t s) {
  if (N <= 128) {
    const int np = N <= 32 ? 32 : N <= 64 ? 64 : 128, rpb = 256 / (np / 4);
    const int nrb = (m + rpb - 1) / rpb;
    const int npk = pk.params ? (pk.start[4] + 255) / 256 : 0;
    *nblk = nrb;
    const dim3 g(nrb + npk);
    if (np == 32)
      hipLaunchKernelGGL(k_feat_rows2<32>, g, dim3(256), 0, s, n, m, N, k, Xf, idx, hw, y, eps,
                         Dtmp, var, cpart, err, nrb, pk);
    else if (np == 64)
      hipLaunchKernelGGL(k_feat_rows2<64>, g, dim3(256), 0, s, n, m, N, k, Xf, idx, hw, y, eps,
                         Dtmp, var, cpart, err, nrb, pk);
    else
      hipLaunchKernelGGL(k_feat_rows2<128>, g, dim3(256), 0, s, n, m, N, k, Xf, idx, hw, y, eps,
                         Dtmp, var, cpart, err, nrb, pk);
    return hipGetLastError();
  }
  const int rpb = 32;
  *nblk = (m + rpb - 1) / rpb;
  const size_t sh = sizeof(double) * (size_t)rpb * N;
  hipLaunchKernelGGL(k_feat_rows, dim3(*nblk), dim3(256), sh, s, n, m, N, k, Xf, idx, hw, y, eps,
                     Dtmp, var, cpart, rpb, err);
  return hipGetLastError();
}

FwdPack fwd_pack(const float* params, unsigned char* ws, const WsLayout& L) {
  FwdPack P;
  memset(&P, 0, sizeof(P));
  P.params = params;
  int at = 0;
  for (int l = 0; l < 4; ++l) {
    P.Wf[l] = (__bf16*)(ws + L.Wf[l]);
    P.bias[l] = (float*)(ws + L.bias[l]);
    P.off[l] = (int)wsnet_param_offset(l);
    P.cin[l] = kCin[l];
    P.cout[l] = kCout[l];
    P.cinp[l] = kCinP[l];
    P.coutp[l] = kCoutP[l];
    P.tpf[l] = tpf(l);
    P.start[l] = at;
    at += kCoutP[l] * tpf(l) * kCinP[l] + kCoutP[l];
  }
  P.start[4] = at;
  return P;
}

}  // namespace

hipError_t wsnet_features(int n, int m, int N, int k, const float* Xf, const int32_t* idx,
                          const float* hw, const float* y, const float* rdiag, const float* eps,
                          float* feat, float* scale, float* Dtmp, float* var, double* cpart,
                          int* err, hipStream_t s) {
  FwdPack none;
  memset(&none, 0, sizeof(none));
  int nblk = 0;
  hipError_t e = feature_rows(n, m, N, k, Xf, idx, hw, y, eps, Dtmp, var, cpart, err, none,
                              &nblk, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_feat_cols, dim3(N), dim3(256), 0, s, m, N, nblk, Dtmp, var, rdiag, cpart,
                     feat, scale);
  return hipGetLastError();
}

hipError_t wsnet_predict_z0(int n, int m, int N, int k, const float* Xf, const int32_t* idx,
                           const float* hw, const float* y, const float* rdiag, const float* eps,
                           const float* params, float* z0, unsigned char* ws, const WsLayout& L,
                           float* Dtmp, float* var, double* cpart, int* err, float* feat,
                           float* scale, hipStream_t s) {
  if (N > 128) {
    hipError_t e = wsnet_features(n, m, N, k, Xf, idx, hw, y, rdiag, eps, feat, scale, Dtmp, var,
                                  cpart, err, s);
    if (e != hipSuccess) return e;
    if ((e = wsnet_pack(params, ws, L, s)) != hipSuccess) return e;
    float* out = (float*)(ws + L.out);
    if ((e = wsnet_forward(N, m, feat, ws, L, out, s)) != hipSuccess) return e;
    return wsnet_z0(m, N, out, scale, z0, s);
  }
  int nblk = 0;
  hipError_t e = feature_rows(n, m, N, k, Xf, idx, hw, y, eps, Dtmp, var, cpart, err,
                              fwd_pack(params, ws, L), &nblk, s);
  if (e != hipSuccess) return e;
  constexpr int T = kInfTile;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu < 1)
    ncu = 256;
  InferArgs a;
  a.m = m;
  a.N = N;
  a.nblk = nblk;
  a.tiles = (m + T - 1) / T;
  const int items = a.tiles * N, grid = items < ncu ? items : ncu;
  a.per = (items + grid - 1) / grid;
  a.D = Dtmp;
  a.var = var;
  a.rdiag = rdiag;
  a.cpart = cpart;
  for (int l = 0; l < 4; ++l) {
    a.W[l] = (const __bf16*)(ws + L.Wf[l]);
    a.bias[l] = (const float*)(ws + L.bias[l]);
  }
  a.z0 = z0;
  const size_t lds = InfCfg<T>::lds;
  if ((e = hipFuncSetAttribute((const void*)k_infer<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_infer<T>, dim3((items + a.per - 1) / a.per), dim3(512), lds, s, a);
  return hipGetLastError();
}

hipError_t wsnet_z0(int m, int N, const float* out, const float* scale, float* z0, hipStream_t s) {
  hipLaunchKernelGGL(k_z0, dim3((m * N + 255) / 256), dim3(256), 0, s, m, N, out, scale, z0);
  return hipGetLastError();
}

hipError_t wsnet_target(int m, int N, const float* Z, const float* scale, float* target,
                        hipStream_t s) {
  long nb = ((long)m * N + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_target, dim3((unsigned)nb), dim3(256), 0, s, m, N, Z, scale, target);
  return hipGetLastError();
}

hipError_t wsnet_jacobi_z0(int m, int N, const float* feat, const float* scale, float* z0,
                          hipStream_t s) {
  long nb = ((long)m * N + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_jacobi_z0, dim3((unsigned)nb), dim3(256), 0, s, m, N, feat, scale, z0);
  return hipGetLastError();
}

}  // namespace cgd
