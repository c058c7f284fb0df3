// Internal declarations shared by the libyand translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdio>

namespace yand {

// Rows of A are padded to a multiple of this many bars (zero rows), columns
// to a multiple of kColPad elements (zero columns).  Zero rows and columns
// contribute nothing to any product with A.
constexpr int kRowPad = 128;
constexpr int kColPad = 128;

// Pass kernels: one 512-thread workgroup per compute unit.
constexpr int kPassThreads = 512;
constexpr int kPassWaves = kPassThreads / 64;
constexpr int kMaxPassGroups = 1024;

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// ---- storage element types ------------------------------------------------
struct bf16_t {
  uint16_t bits;
};

__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(bf16_t v) {
  return (double)__uint_as_float(((uint32_t)v.bits) << 16);
}
__device__ __forceinline__ float to_f32(double v) { return (float)v; }
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(bf16_t v) {
  return __uint_as_float(((uint32_t)v.bits) << 16);
}

// Round a float to bfloat16 with round-to-nearest-even (NaN kept quiet).
__device__ __forceinline__ bf16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  bf16_t r;
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
    r.bits = (uint16_t)((u >> 16) | 0x0040u);
    return r;
  }
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  r.bits = (uint16_t)(u >> 16);
  return r;
}

template <typename S> struct StoreConv;
template <> struct StoreConv<double> {
  __device__ static double from(double v) { return v; }
};
template <> struct StoreConv<float> {
  __device__ static float from(double v) { return (float)v; }
};
template <> struct StoreConv<bf16_t> {
  __device__ static bf16_t from(double v) { return f32_to_bf16((float)v); }
};

// ---- wave / block reductions (FP64, fixed order) --------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// ---- preference polynomial psi(s) = c2 s^2 - c3 s^3 + c4 s^4 --------------
struct Coef {
  double c1, c2, c3, c4;
};
__device__ __forceinline__ double dpsi(const Coef& c, double s) {
  return s * (2.0 * c.c2 + s * (-3.0 * c.c3 + s * (4.0 * c.c4)));
}
__device__ __forceinline__ double d2psi(const Coef& c, double s) {
  return 2.0 * c.c2 + s * (-6.0 * c.c3 + s * (12.0 * c.c4));
}
__device__ __forceinline__ double d3psi(const Coef& c, double s) {
  return -6.0 * c.c3 + 24.0 * c.c4 * s;
}

}  // namespace yand

#define YAND_HIP_CHECK(expr)                                              \
  do {                                                                    \
    hipError_t _e = (expr);                                               \
    if (_e != hipSuccess) {                                               \
      fprintf(stderr, "libyand: %s failed: %s (%s:%d)\n", #expr,          \
              hipGetErrorString(_e), __FILE__, __LINE__);                 \
      return YAND_ERR_HIP;                                                \
    }                                                                     \
  } while (0)
