// MFMA and vector-load helpers shared by the gfx950 solver kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace cgd {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

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

// U contiguous values from a 16-byte aligned pointer (LDS or global).
template <int U>
__device__ inline void vload(const float* p, float (&v)[U]) {
  static_assert(U % 4 == 0, "U");
#pragma unroll
  for (int u = 0; u < U; u += 4) {
    const v4f x = *reinterpret_cast<const v4f*>(p + u);
    v[u] = x[0]; v[u + 1] = x[1]; v[u + 2] = x[2]; v[u + 3] = x[3];
  }
}
template <int U>
__device__ inline void vload(const double* p, double (&v)[U]) {
  static_assert(U % 2 == 0, "U");
#pragma unroll
  for (int u = 0; u < U; u += 2) {
    const v2d x = *reinterpret_cast<const v2d*>(p + u);
    v[u] = x[0]; v[u + 1] = x[1];
  }
}
// Four consecutive values widened to double.
__device__ inline void load4d(const float* p, double (&v)[4]) {
  const v4f x = *reinterpret_cast<const v4f*>(p);
  v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
}
__device__ inline void load4d(const double* p, double (&v)[4]) {
  const v2d x = *reinterpret_cast<const v2d*>(p), y = *reinterpret_cast<const v2d*>(p + 2);
  v[0] = x[0]; v[1] = x[1]; v[2] = y[0]; v[3] = y[1];
}

}  // namespace
}  // namespace cgd

namespace cgd {
namespace {

// Data-parallel-primitive (DPP) lane exchanges: VALU-speed alternatives to
// the LDS crossbar for reductions inside a wavefront.  dpp<CTRL>(v) returns
// the value of v in the lane that CTRL selects (quad_perm, row_mirror and
// row_half_mirror and row_ror stay inside a row of 16 lanes, so every source
// is valid; no lane keeps an old value, so none is supplied (a plain mov_dpp,
// which the compiler can also fold into the add that consumes it).
template <int CTRL>
__device__ inline float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ inline double dpp(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7-i within 8
constexpr int kDppMirror = 0x140;      // lane i <-> 15-i within 16

// Sum over aligned groups of L lanes (L = 1, 2, 4, 8, 16, 32); every lane of
// a group gets the same bits (each step adds a commutative pair).
template <int L, typename T>
__device__ inline T group_sum(T v) {
  if constexpr (L >= 2) v += dpp<kDppXor1>(v);
  if constexpr (L >= 4) v += dpp<kDppXor2>(v);
  if constexpr (L >= 8) v += dpp<kDppHalfMirror>(v);
  if constexpr (L >= 16) v += dpp<kDppMirror>(v);
  if constexpr (L >= 32) v += __shfl_xor(v, 16);
  return v;
}

__device__ inline double readlane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ inline int readlane(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// Sum over the 64 lanes of the wavefront in a fixed order, returned
// (bitwise identical) to every lane.
__device__ inline double wave_sum(double v) {
  v = group_sum<16>(v);
  return (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
}

}  // namespace
}  // namespace cgd
