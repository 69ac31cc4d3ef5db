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

// Column pass: s_j = RMS of d_j (fixed-order sum of the block partials), then
// feat[j][i] = (d_ij / s_j, var_i, r_i, 0).
__global__ void k_feat_cols(int m, int N, int nblk, const float* D, const float* var,
                            const float* rdiag, const double* cpart, float* feat, float* scale) {
  __shared__ float s_sh;
  const int j = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += cpart[(size_t)b * N + j];
    double rms = sqrt(s / m);
    if (!(rms > 0.0)) rms = 1.0;
    s_sh = (float)rms;
    scale[j] = (float)rms;
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

hipError_t wsnet_features(int n, int m, int N, int k, const float* Xf, const int32_t* idx,
                          const float* hw, const float* y, const float* rdiag, const float* eps,
                          float* feat, float* scale, float* Dtmp, float* var, double* cpart,
                          int* err, hipStream_t s) {
  const int rpb = 32;
  const int nblk = (m + rpb - 1) / rpb;
  const size_t sh = sizeof(double) * (size_t)rpb * N;
  hipLaunchKernelGGL(k_feat_rows, dim3(nblk), dim3(256), sh, s, n, m, N, k, Xf, idx, hw, y, eps,
                     Dtmp, var, cpart, rpb, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_feat_cols, dim3(N), dim3(256), 0, s, m, N, nblk, Dtmp, var, rdiag, cpart,
                     feat, scale);
  return hipGetLastError();
}

hipError_t wsnet_z0(int m, int N, const float* out, const float* scale, float* z0, hipStream_t s) {
  hipLaunchKernelGGL(k_z0, dim3((m * N + 255) / 256), dim3(256), 0, s, m, N, out, scale, z0);
  return hipGetLastError();
}

}  // namespace cgd
