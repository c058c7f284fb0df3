// Dense kernels of the exact trace for FP32 and BF16 storage of A: the
// products run on the matrix cores with FP32 or BF16 inputs and FP32
// accumulation (v_mfma_f32_16x16x4f32, v_mfma_f32_16x16x32_bf16), and their
// results leave in FP64 for the factorisation, which stays in FP64.
//
// Both contractions are written as C = P Q^T with P and Q stored row-major
// and contiguous along the contraction index k, which is the layout a BF16
// MFMA lane wants (8 consecutive k per lane):
//  - B = A^T diag(s) A: P = A^T (kept transposed in the context), Q = the
//    rows of A^T scaled by s_t and rounded to the storage precision (one
//    elementwise pass per iteration);
//  - the trace rows W = A X^T: P = A, Q = X = L^-1 rounded to the storage
//    precision (one elementwise pass per iteration).
// P is the stored matrix itself, exact at its precision; only Q is rounded.
// In BF16 one rounding of Q (2^-9 relative) perturbs B by about 2^-9 |B| in
// norm, which exceeds the smallest curvature of the tangent Hessian once its
// condition number passes a few hundred (n = 5440: about 5e4), so BF16 keeps
// Q as an unevaluated sum Q = Q_hi + Q_lo of two BF16 matrices (Q_hi the
// rounding of the FP32 value, Q_lo the rounding of the remainder; about 16
// significant bits) and runs the product over both: C = P Q_hi^T + P Q_lo^T.
// 128 x 128 output tiles, 256 threads = 4 waves in a 2 x 2 grid, 64 x 64 per
// wave as 4 x 4 blocks of 16 x 16 MFMA outputs.  Slices of BK k-values of
// both operands move global -> registers -> LDS (rows of BK elements, padded
// pitch) with two LDS buffers and the next-but-one slice in registers.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace yand {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int LT = 128;  // output tile
constexpr int LNT = 256; // threads

// One 16-byte fragment per lane and operand feeds MPI MFMAs.
//  FP32: lane l holds k = 4 (l / 16) .. + 3 of a 16-deep block; MFMA u takes
//        element u, so MFMA u sums k = {4 q + u}: the four MFMAs together
//        cover the block (both operands use the same lane -> k map).
//  BF16: lane l holds k = 8 (l / 16) .. + 7 of a 32-deep block, one MFMA.
template <typename S> struct Lp;
template <> struct Lp<float> {
  static constexpr int SPLIT = 1;     // parts of the rounded operand Q
  static constexpr int E = 4;         // elements per 16 bytes
  static constexpr int BK = 16;       // slice depth (one k-block)
  static constexpr int PITCH = BK + 4;  // LDS row pitch in elements (80 B)
  static constexpr int MPI = 4;
  __device__ static f32x4 mma(const u32x4& a, const u32x4& b, int u,
                              const f32x4& c) {
    const unsigned av = u == 0 ? a.x : u == 1 ? a.y : u == 2 ? a.z : a.w;
    const unsigned bv = u == 0 ? b.x : u == 1 ? b.y : u == 2 ? b.z : b.w;
    return __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av),
                                                __uint_as_float(bv), c, 0, 0,
                                                0);
  }
};
template <> struct Lp<bf16_t> {
  static constexpr int SPLIT = 2;
  static constexpr int E = 8;
  static constexpr int BK = 64;       // two k-blocks of 32
  static constexpr int PITCH = BK + 8;  // 144 B
  static constexpr int MPI = 1;
  __device__ static f32x4 mma(const u32x4& a, const u32x4& b, int,
                              const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
        0);
  }
};

// k-depth of one fragment read (one k-block)
template <typename S>
constexpr int kblock() { return 4 * Lp<S>::E; }

// One slice of one 128-row operand: chunk i of this thread is row m = idx /
// CPR, 16-byte column c = idx % CPR of the slice (idx = tid + i LNT), so
// consecutive threads read consecutive 16-byte pieces of a row.
template <typename S>
struct LpStage {
  static constexpr int CPR = Lp<S>::BK / Lp<S>::E;
  static constexpr int PER = LT * CPR / LNT;
  u32x4 r[PER];
  __device__ __forceinline__ void load(const S* base, int64_t ld, int64_t k0,
                                       int tid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + i * LNT, m = idx / CPR, c = idx % CPR;
      r[i] = *(const u32x4*)(base + (int64_t)m * ld + k0 + c * Lp<S>::E);
    }
  }
  __device__ __forceinline__ void store(S* s, int tid) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + i * LNT, m = idx / CPR, c = idx % CPR;
      *(u32x4*)(s + m * Lp<S>::PITCH + c * Lp<S>::E) = r[i];
    }
  }
};

template <typename S>
constexpr int lp_stage_elems() { return LT * Lp<S>::PITCH; }

// acc (this wave's 64 x 64 block) (+)= sum_{k in [0, K)} P[m][k] Q[n][k] for
// the 128 rows of P at Pb and of Q at Qb (row stride ld, K a multiple of BK);
// ZERO clears acc first.
template <typename S, bool ZERO = true>
__device__ void lp_core(const S* Pb, int64_t ldp, const S* Qb, int64_t ldq,
                        int64_t K, f32x4 (&acc)[4][4], S* sP, S* sQ) {
  using L = Lp<S>;
  constexpr int ST = lp_stage_elems<S>();
  constexpr int KB = kblock<S>();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  const int fr = lane & 15, fk = (lane >> 4) * L::E;
  if constexpr (ZERO) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const int64_t ns = K / L::BK;
  if (ns <= 0) return;
  LpStage<S> gp, gq;
  gp.load(Pb, ldp, 0, tid);
  gq.load(Qb, ldq, 0, tid);
  gp.store(sP, tid);
  gq.store(sQ, tid);
  if (ns > 1) {
    gp.load(Pb, ldp, L::BK, tid);
    gq.load(Qb, ldq, L::BK, tid);
  }
  __syncthreads();
  for (int64_t s = 0; s < ns; ++s) {
    const int b = (int)(s & 1);
    const S* rp = sP + b * ST;
    const S* rq = sQ + b * ST;
#pragma unroll
    for (int kb = 0; kb < L::BK / KB; ++kb) {
      u32x4 a[4], bq[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *(const u32x4*)(rp + (wm + i * 16 + fr) * L::PITCH + kb * KB + fk);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bq[j] = *(const u32x4*)(rq + (wn + j * 16 + fr) * L::PITCH + kb * KB + fk);
      if (kb == 0 && s + 1 < ns) {
        // the next slice into the other buffer (last read before the
        // previous barrier), then the one after it into the registers
        gp.store(sP + (b ^ 1) * ST, tid);
        gq.store(sQ + (b ^ 1) * ST, tid);
        if (s + 2 < ns) {
          gp.load(Pb, ldp, (s + 2) * L::BK, tid);
          gq.load(Qb, ldq, (s + 2) * L::BK, tid);
        }
      }
#pragma unroll
      for (int u = 0; u < L::MPI; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = L::mma(a[i], bq[j], u, acc[i][j]);
    }
    __syncthreads();
  }
}

// Visit this wave's accumulator entries as (row, col) of the 128 x 128 tile:
// a 16 x 16 FP32 MFMA output holds row 4 (l / 16) + r, column l % 16 in
// register r of lane l.
template <class F>
__device__ __forceinline__ void lp_for_each(const f32x4 (&acc)[4][4], F f) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        f(wm + i * 16 + 4 * (lane >> 4) + r, wn + j * 16 + (lane & 15),
          acc[i][j][r]);
}

__device__ __forceinline__ void lp_lower_tile(int64_t b, int* I, int* J) {
  int i = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((int64_t)i * (i + 1) / 2 > b) --i;
  while ((int64_t)(i + 1) * (i + 2) / 2 <= b) ++i;
  *I = i;
  *J = (int)(b - (int64_t)i * (i + 1) / 2);
}

// B = At SAt^T (n x n, FP64 out): lower tiles, mirrored.  A diagonal tile
// writes its lower half and mirrors it, so B is exactly symmetric.  order
// (nullable): the tile (I, J) of each workgroup, -1 for an idle one (the
// XCD-aware order of the FP64 SYRK).
template <typename S>
__global__ void __launch_bounds__(LNT) __attribute__((amdgpu_waves_per_eu(2, 2)))
syrk_lp_kernel(const S* __restrict__ At, const S* __restrict__ SAt,
               int64_t ldt, int64_t K, int64_t qsplit,
               double* __restrict__ B, int64_t ldb, const int* skip,
               const int* __restrict__ order) {
  if (skip && *skip) return;
  __shared__ __align__(16) S sP[2 * lp_stage_elems<S>()];
  __shared__ __align__(16) S sQ[2 * lp_stage_elems<S>()];
  int I, J;
  if (order) {
    I = order[2 * blockIdx.x];
    J = order[2 * blockIdx.x + 1];
    if (I < 0) return;
  } else {
    lp_lower_tile(blockIdx.x, &I, &J);
  }
  f32x4 acc[4][4];
  lp_core<S>(At + (int64_t)I * LT * ldt, ldt, SAt + (int64_t)J * LT * ldt,
             ldt, K, acc, sP, sQ);
  if constexpr (Lp<S>::SPLIT == 2)
    lp_core<S, false>(At + (int64_t)I * LT * ldt, ldt,
                      SAt + qsplit + (int64_t)J * LT * ldt, ldt, K, acc, sP,
                      sQ);
  double* Bij = B + (int64_t)I * LT * ldb + (int64_t)J * LT;
  double* Bji = B + (int64_t)J * LT * ldb + (int64_t)I * LT;
  if (I != J) {
    lp_for_each(acc, [&](int r, int c, float v) {
      Bij[(int64_t)r * ldb + c] = (double)v;
      Bji[(int64_t)c * ldb + r] = (double)v;
    });
  } else {
    lp_for_each(acc, [&](int r, int c, float v) {
      if (r >= c) {
        Bij[(int64_t)r * ldb + c] = (double)v;
        Bij[(int64_t)c * ldb + r] = (double)v;
      }
    });
  }
}

// rn[J][t] = sum_{j in tile J} (sum_{k < 128 (J + 1)} A[t][k] Xl[j][k])^2:
// the rows of W = A X^T restricted to the lower triangle of X, squared and
// summed per row in FP64.  Tile order as the FP64 trace kernel: longest
// reductions first, row tiles padded to a multiple of 8 so that a row tile
// of A always lands on the same XCD.
template <typename S>
__global__ void __launch_bounds__(LNT) __attribute__((amdgpu_waves_per_eu(2, 2)))
trace_lp_kernel(const S* __restrict__ A, int64_t lda, int64_t Tp,
                const S* __restrict__ Xl, int64_t ldx, int64_t qsplit,
                double* __restrict__ rn, const int* skip) {
  if (skip && *skip) return;
  __shared__ __align__(16) S sP[2 * lp_stage_elems<S>()];
  __shared__ __align__(16) S sQ[2 * lp_stage_elems<S>()];
  __shared__ double rows[2][LT];
  const int ntt = (int)(Tp / LT), ntp = (ntt + 7) / 8 * 8;
  const int nJ = gridDim.x / ntp;
  const int ti = (int)blockIdx.x % ntp;
  if (ti >= ntt) return;
  const int J = nJ - 1 - (int)blockIdx.x / ntp;
  const int64_t t0 = (int64_t)ti * LT;
  f32x4 acc[4][4];
  lp_core<S>(A + t0 * lda, lda, Xl + (int64_t)J * LT * ldx, ldx,
             (int64_t)(J + 1) * LT, acc, sP, sQ);
  if constexpr (Lp<S>::SPLIT == 2)
    lp_core<S, false>(A + t0 * lda, lda, Xl + qsplit + (int64_t)J * LT * ldx,
                      ldx, (int64_t)(J + 1) * LT, acc, sP, sQ);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double x = (double)acc[i][j][r];
        v += x * x;
      }
      // the 16 lanes of one row group hold the 16 columns of a block
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      if ((lane & 15) == 0) rows[w & 1][wm + i * 16 + 4 * (lane >> 4) + r] = v;
    }
  __syncthreads();
  if (tid < LT) rn[(int64_t)J * Tp + t0 + tid] = rows[0][tid] + rows[1][tid];
}

// ------------------------------------------------------- elementwise ----

// At (lda x Tp) = A^T (A is Tp x lda), 64 x 64 tiles through LDS.
template <typename S>
__global__ void __launch_bounds__(256)
transpose_kernel(const S* __restrict__ A, int64_t lda, int64_t Tp,
                 S* __restrict__ At) {
  __shared__ S tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) tile[r][tx] = A[(r0 + r) * lda + c0 + tx];
  __syncthreads();
  for (int c = ty; c < 64; c += 4) At[(c0 + c) * Tp + r0 + tx] = tile[tx][c];
}

__device__ __forceinline__ u32x4 scale_pack(const u32x4& v, const float* s,
                                            float, u32x4*) {
  u32x4 o;
  o.x = __float_as_uint(__uint_as_float(v.x) * s[0]);
  o.y = __float_as_uint(__uint_as_float(v.y) * s[1]);
  o.z = __float_as_uint(__uint_as_float(v.z) * s[2]);
  o.w = __float_as_uint(__uint_as_float(v.w) * s[3]);
  return o;
}
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) {
  return (uint32_t)f32_to_bf16(lo).bits | ((uint32_t)f32_to_bf16(hi).bits << 16);
}
__device__ __forceinline__ float bf16_val(bf16_t b) {
  return __uint_as_float((uint32_t)b.bits << 16);
}
// FP32 products s a of eight BF16 values, split into BF16 hi = round(s a)
// and lo = round(s a - hi).
__device__ __forceinline__ u32x4 scale_pack(const u32x4& v, const float* s,
                                            bf16_t, u32x4* lo) {
  const uint32_t in[4] = {v.x, v.y, v.z, v.w};
  uint32_t hi[4], lw[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float p0 = __uint_as_float(in[q] << 16) * s[2 * q];
    const float p1 = __uint_as_float(in[q] & 0xffff0000u) * s[2 * q + 1];
    const bf16_t h0 = f32_to_bf16(p0), h1 = f32_to_bf16(p1);
    hi[q] = (uint32_t)h0.bits | ((uint32_t)h1.bits << 16);
    lw[q] = bf16_pair(p0 - bf16_val(h0), p1 - bf16_val(h1));
  }
  *lo = u32x4{lw[0], lw[1], lw[2], lw[3]};
  return u32x4{hi[0], hi[1], hi[2], hi[3]};
}

// SAt[i][t] = s_t At[i][t], rounded to the storage precision (products in
// FP32); BF16 also writes the remainder part at SAt + rows Tp.  One 16-byte
// chunk per thread and step.
template <typename S>
__global__ void __launch_bounds__(256)
scale_cols_kernel(const S* __restrict__ At, int64_t rows, int64_t Tp,
                  const double* __restrict__ s, S* __restrict__ SAt,
                  const int* skip) {
  if (skip && *skip) return;
  constexpr int E = Lp<S>::E;
  const int64_t cpr = Tp / E, total = rows * cpr;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
       idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / cpr, t = (idx % cpr) * E;
    float sv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) sv[e] = (float)s[t + e];
    const u32x4 v = *(const u32x4*)(At + i * Tp + t);
    u32x4 lo;
    *(u32x4*)(SAt + i * Tp + t) = scale_pack(v, sv, S{}, &lo);
    if constexpr (Lp<S>::SPLIT == 2)
      *(u32x4*)(SAt + rows * Tp + i * Tp + t) = lo;
  }
}

// Xl = X rounded to the storage precision on the tiles I >= J of the
// 128-tile grid (X = L^-1 is block lower triangular; tiles above are not
// read); BF16 also writes the remainder part at Xl + np^2.
template <typename S>
__global__ void __launch_bounds__(256)
xconv_kernel(const double* __restrict__ X, int64_t np, S* __restrict__ Xl,
             const int* skip) {
  if (skip && *skip) return;
  int I, J;
  lp_lower_tile(blockIdx.x, &I, &J);
  const double* src = X + (int64_t)I * LT * np + (int64_t)J * LT;
  S* dst = Xl + (int64_t)I * LT * np + (int64_t)J * LT;
  for (int e = threadIdx.x; e < LT * LT; e += blockDim.x) {
    const int r = e / LT, c = e % LT;
    const double x = src[(int64_t)r * np + c];
    const S h = StoreConv<S>::from(x);
    dst[(int64_t)r * np + c] = h;
    if constexpr (Lp<S>::SPLIT == 2)
      dst[np * np + (int64_t)r * np + c] =
          StoreConv<S>::from(x - (double)bf16_val(h));
  }
}

template <typename S>
hipError_t syrk_lp(const S* At, S* SAt, int64_t np, int64_t Tp,
                   const double* s, double* B, hipStream_t st,
                   const int* skip, const int* order, int64_t order_slots) {
  const int64_t chunks = np * (Tp / Lp<S>::E);
  const unsigned g = (unsigned)std::min<int64_t>((chunks + 255) / 256, 8192);
  hipLaunchKernelGGL(scale_cols_kernel<S>, dim3(g), dim3(256), 0, st, At, np,
                     Tp, s, SAt, skip);
  const int64_t nt = np / LT;
  const int64_t nwg = order ? order_slots : nt * (nt + 1) / 2;
  hipLaunchKernelGGL(syrk_lp_kernel<S>, dim3((unsigned)nwg), dim3(LNT), 0, st,
                     At, SAt, Tp, Tp, np * Tp, B, np, skip, order);
  return hipGetLastError();
}

template <typename S>
hipError_t trace_lp(const S* A, int64_t lda, int64_t Tp, const double* X,
                    int64_t np, S* Xl, double* rn, hipStream_t st,
                    const int* skip) {
  const int64_t nt = np / LT;
  hipLaunchKernelGGL(xconv_kernel<S>, dim3((unsigned)(nt * (nt + 1) / 2)),
                     dim3(256), 0, st, X, np, Xl, skip);
  dim3 g((unsigned)(nt * ((Tp / LT + 7) / 8 * 8)));
  hipLaunchKernelGGL(trace_lp_kernel<S>, g, dim3(LNT), 0, st, A, lda, Tp, Xl,
                     np, np * np, rn, skip);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_transpose_lp(int precision, const void* A, int64_t lda,
                               int64_t Tp, void* At, hipStream_t st) {
  dim3 g((unsigned)(lda / 64), (unsigned)(Tp / 64)), b(256);
  if (precision == 1)
    hipLaunchKernelGGL(transpose_kernel<float>, g, b, 0, st, (const float*)A,
                       lda, Tp, (float*)At);
  else if (precision == 2)
    hipLaunchKernelGGL(transpose_kernel<bf16_t>, g, b, 0, st,
                       (const bf16_t*)A, lda, Tp, (bf16_t*)At);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_syrk_lp(int precision, const void* At, void* SAt,
                          int64_t np, int64_t Tp, const double* s, double* B,
                          hipStream_t st, const int* skip, const int* order,
                          int64_t order_slots) {
  if (precision == 1)
    return syrk_lp<float>((const float*)At, (float*)SAt, np, Tp, s, B, st,
                          skip, order, order_slots);
  if (precision == 2)
    return syrk_lp<bf16_t>((const bf16_t*)At, (bf16_t*)SAt, np, Tp, s, B, st,
                           skip, order, order_slots);
  return hipErrorInvalidValue;
}

hipError_t launch_trace_lp(int precision, const void* A, int64_t lda,
                           int64_t Tp, const double* X, int64_t np, void* Xl,
                           double* rn, hipStream_t st, const int* skip) {
  if (precision == 1)
    return trace_lp<float>((const float*)A, lda, Tp, X, np, (float*)Xl, rn,
                           st, skip);
  if (precision == 2)
    return trace_lp<bf16_t>((const bf16_t*)A, lda, Tp, X, np, (bf16_t*)Xl, rn,
                            st, skip);
  return hipErrorInvalidValue;
}

}  // namespace yand
