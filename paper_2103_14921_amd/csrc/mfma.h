// 16x16x4 matrix-core steps in complex-FP32 and FP64 work, shared by the
// batched local solves and the factorisation.  Lane l of a wave supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; output element v of lane group
// lg = l / 16 sits in column l % 16 and in the tile row given by row(lg, v).
#pragma once
#include "common.h"

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element v of lane group lg (lane / 16) sits in tile row 4 lg + v
  static __device__ __forceinline__ int row(int lg, int v) { return 4 * lg + v; }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the f64 variant interleaves its rows: element v of lane group lg is tile row lg + 4 v
  static __device__ __forceinline__ int row(int lg, int v) { return lg + 4 * v; }
};
