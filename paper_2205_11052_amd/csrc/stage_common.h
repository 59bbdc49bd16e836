// Device helpers shared by the stage kernels (stage.hip, stage_split.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace dgw {
namespace stagec {

template <int N>
struct Sz {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
};

__device__ inline double ricker_d(double tau, double f0, double t0, double amp) {
  const double pi = 3.14159265358979323846;
  double a = pi * f0 * (tau - t0);
  a = a * a;
  return amp * (1.0 - 2.0 * a) * exp(-a);
}

// Linear work-group id -> item index such that each XCD (id % 8) owns one
// contiguous range of items.
__device__ inline int64_t xcd_item(int64_t L, int64_t total) {
  const int x = (int)(L & 7);
  int64_t start = 0;
  for (int y = 0; y < x; ++y) start += (total - y + 7) >> 3;
  return start + (L >> 3);
}

template <typename real>
struct real2v {
  real r, q;
};

// Matrix-core (MFMA) 16x16x4 tiles.  Lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16] of the 16x4 and 4x16 operands (both precisions); the
// 16x16 accumulator lives in four registers per lane, lane l holding column
// l % 16 and, for register r, row 4 (l / 16) + r (FP32) or (l / 16) + 4 r
// (FP64).  (Layouts checked on the device.)
template <typename real>
struct Mma;
template <>
struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int g, int r) { return 4 * g + r; }
};
template <>
struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int g, int r) { return g + 4 * r; }
};

}  // namespace stagec
}  // namespace dgw
