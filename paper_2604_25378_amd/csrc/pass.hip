// Streaming passes over the centered return matrix A (HBM-bound kernels).
//
// Every oracle quantity of the exact sample oracle (Proposition "Exact
// operator representation", equations (operator-f) to (operator-third)) and
// every line-search power sum (Proposition "Quartic exact line search from
// sample power sums") is one read of A: a row dot a_t^T v, a scalar function
// of the row results, and a weighted back-projection sum_t omega_t a_t.
//
// Layout: A is row-major, Tp x lda (Tp = T rounded up to kRowPad, lda = n
// rounded up to kColPad), zero in the padding.  A 512-thread workgroup owns a
// contiguous band of rows; each thread owns NCH 16-byte column chunks of every
// row, keeps the dot operand for those chunks in registers, and accumulates its
// columns of the back-projection in FP64 registers.  The row dot is reduced
// across the workgroup in a fixed order (wave butterfly, then the 8 wave
// results in order), so results are bit-reproducible.  Each workgroup writes
// one FP64 partial row; reduce_partials sums them in workgroup order.
#include "common.h"
#include "kernels.h"

namespace yand {

// ------------------------------------------------------------- centering --

// Column partial sums of R over a chunk of rows (a1: mu = T^-1 R^T 1).
__global__ void colsum_kernel(const double* __restrict__ R, int64_t T,
                              int64_t n, int64_t ldr, int64_t chunk,
                              double* __restrict__ part) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t t0 = (int64_t)blockIdx.y * chunk;
  if (j >= n) return;
  int64_t t1 = t0 + chunk < T ? t0 + chunk : T;
  double s = 0.0;
  for (int64_t t = t0; t < t1; ++t) s += R[t * ldr + j];
  part[(int64_t)blockIdx.y * n + j] = s;
}

__global__ void colsum_finish_kernel(const double* __restrict__ part,
                                     int64_t nchunks, int64_t n, int64_t T,
                                     double* __restrict__ mu,
                                     int* __restrict__ nonfinite) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int64_t b = 0; b < nchunks; ++b) s += part[b * n + j];
  double m = s / (double)T;
  mu[j] = m;
  if (!isfinite(m)) atomicOr(nonfinite, 1);
}

// A = R - 1 mu^T rounded to the storage type; zero padding.
template <typename S>
__global__ void center_convert_kernel(const double* __restrict__ R, int64_t T,
                                      int64_t n, int64_t ldr,
                                      const double* __restrict__ mu,
                                      S* __restrict__ A, int64_t lda,
                                      int64_t Tp) {
  for (int64_t t = blockIdx.y; t < Tp; t += gridDim.y) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < lda;
         j += (int64_t)gridDim.x * blockDim.x) {
      double v = (t < T && j < n) ? R[t * ldr + j] - mu[j] : 0.0;
      A[t * lda + j] = StoreConv<S>::from(v);
    }
  }
}

// -------------------------------------------------------------- the pass --

// Per-row scalar work of each pass.  s is the finished row dot (if any),
// t the row index; the op returns the back-projection weight and updates its
// running scalar sums (kept by thread 0 only).
struct OpOracle {   // a2: z = Ax, psi'(z)/T, sum z^2, z^3, z^4
  static constexpr bool kDot = true, kBack = true, kZ = false, kQ = false;
  static constexpr int kSums = 3;
  __device__ static double row(const PassArgs& a, int64_t t, double s,
                               double* sums, bool lead, double, double) {
    if (lead) {
      a.tout[t] = s;
      double s2 = s * s;
      sums[0] += s2;
      sums[1] += s2 * s;
      sums[2] += s2 * s2;
    }
    return dpsi(a.c, s) * a.invT;
  }
};
struct OpValue {    // z = Ax and sum z^2, z^3, z^4 only
  static constexpr bool kDot = true, kBack = false, kZ = false, kQ = false;
  static constexpr int kSums = 3;
  __device__ static double row(const PassArgs& a, int64_t t, double s,
                               double* sums, bool lead, double, double) {
    return OpOracle::row(a, t, s, sums, lead, 0.0, 0.0);
  }
};
struct OpHvp {      // a4: psi''(z_t) (Av)_t / T; (Av)_t optionally stored
  static constexpr bool kDot = true, kBack = true, kZ = true, kQ = false;
  static constexpr int kSums = 0;
  __device__ static double row(const PassArgs& a, int64_t t, double s,
                               double*, bool lead, double z, double) {
    if (lead && a.tout) a.tout[t] = s;
    return d2psi(a.c, z) * s * a.invT;
  }
};
struct OpLine {     // a8: w = Ad and the nine mixed power sums with z
  static constexpr bool kDot = true, kBack = false, kZ = true, kQ = false;
  static constexpr int kSums = 9;
  __device__ static double row(const PassArgs& a, int64_t t, double w,
                               double* sums, bool lead, double z, double) {
    if (lead) {
      if (a.tout) a.tout[t] = w;
      double z2 = z * z, w2 = w * w;
      sums[0] += z * w;        // s11
      sums[1] += z2 * w;       // s21
      sums[2] += z2 * z * w;   // s31
      sums[3] += w2;           // s02
      sums[4] += z * w2;       // s12
      sums[5] += z2 * w2;      // s22
      sums[6] += w2 * w;       // s03
      sums[7] += z * w2 * w;   // s13
      sums[8] += w2 * w2;      // s04
    }
    return 0.0;
  }
};
struct OpDot {      // plain row dot (Av)_t, stored
  static constexpr bool kDot = true, kBack = false, kZ = false, kQ = false;
  static constexpr int kSums = 0;
  __device__ static double row(const PassArgs& a, int64_t t, double s,
                               double*, bool lead, double, double) {
    if (lead) a.tout[t] = s;
    return 0.0;
  }
};
struct OpThird {    // a6: psi'''(z_t) q_t / T (third-order back-projection)
  static constexpr bool kDot = false, kBack = true, kZ = true, kQ = true;
  static constexpr int kSums = 0;
  __device__ static double row(const PassArgs& a, int64_t, double, double*,
                               bool, double z, double q) {
    return d3psi(a.c, z) * q * a.invT;
  }
};

// Sum of p[r] over the 64 lanes for R = 2^b rows at once: b transposing
// exchange steps (each lane keeps half of its rows and adds the partner's
// copy of them) leave lane l with one row, r = l / (64 / R); the remaining
// 6 - b butterfly steps finish the sum.  R - 1 + 6 - b exchanges instead of
// 6 R.  Every lane of row r's group of 64 / R lanes ends with the same bits.
template <int R>
__device__ __forceinline__ double wave_sum_rows(double (&p)[R], int lane) {
  static_assert((R & (R - 1)) == 0 && R <= 64, "R must be a power of two");
#pragma unroll
  for (int half = R / 2, off = 32; half >= 1; half /= 2, off /= 2) {
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int q = 0; q < half; ++q) {
      const double send = up ? p[q] : p[q + half];
      const double keep = up ? p[q + half] : p[q];
      p[q] = keep + __shfl_xor(send, off, 64);
    }
  }
  double v = p[0];
#pragma unroll
  for (int off = 32 / R; off >= 1; off /= 2) v += __shfl_xor(v, off, 64);
  return v;
}

// TPB threads per workgroup; each thread owns NCH 16-byte chunks of every
// row; R rows per step share one reduction and one barrier.
//
// Loads run two row blocks ahead in two register slots.  Once a block's row
// dots are formed, the thread parks its packed chunks in LDS (a private,
// conflict-free slot per thread: it reads back only what it wrote) and
// refills the register slot with the block two steps ahead, so two blocks
// stay in flight through the reduction, the barrier and the back-projection,
// which reads the parked copy.
template <typename S, int TPB, int NCH, int R, class Op>
__global__ void __launch_bounds__(TPB)
pass_kernel(PassArgs a) {
  if (a.skip && *a.skip) return;
  constexpr int VEC = Vec16<S>::N;
  constexpr int NW = TPB / 64;
  constexpr bool kPark = Op::kDot && Op::kBack;
  __shared__ double red[2][R][NW];
  __shared__ u32x4 park[kPark ? R * NCH * TPB : 1];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int64_t nvec = a.lda / VEC;   // 16-byte chunks per row
  const int64_t row0 = (int64_t)blockIdx.x * a.rows_per_wg;
  int64_t row1 = row0 + a.rows_per_wg;
  if (row1 > a.Tp) row1 = a.Tp;
  const char* base = (const char*)a.A;
  const int64_t row_bytes = a.lda * (int64_t)sizeof(S);

  bool valid[NCH];
  double v[NCH][VEC];
  double acc[NCH][VEC];
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    int64_t c = tid + (int64_t)k * TPB;
    valid[k] = c < nvec;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      int64_t j = c * VEC + e;
      v[k][e] = (Op::kDot && valid[k] && j < a.n) ? a.v[j] : 0.0;
      acc[k][e] = 0.0;
    }
  }
  double sums[Op::kSums > 0 ? Op::kSums : 1];
#pragma unroll
  for (int i = 0; i < (Op::kSums > 0 ? Op::kSums : 1); ++i) sums[i] = 0.0;

  u32x4 slot[2][R][NCH];
  // per-row scalars of the op (cached z, q), fetched with their block
  double zs[2][R], qs[2][R];
  auto load_block = [&](int64_t r0, u32x4 (&dst)[R][NCH], double (&zd)[R],
                        double (&qd)[R]) {
    if (r0 >= row1) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      zd[r] = Op::kZ ? a.zc[r0 + r] : 0.0;
      qd[r] = Op::kQ ? a.q[r0 + r] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const u32x4* rowp = (const u32x4*)(base + (r0 + r) * row_bytes);
#pragma unroll
      for (int k = 0; k < NCH; ++k) {
        int64_t c = tid + (int64_t)k * TPB;
        dst[r][k] = valid[k] ? __builtin_nontemporal_load(rowp + c)
                             : u32x4{0u, 0u, 0u, 0u};
      }
    }
  };

  load_block(row0, slot[0], zs[0], qs[0]);
  load_block(row0 + R, slot[1], zs[1], qs[1]);
  int parity = 0;
  for (int64_t r0 = row0; r0 < row1; r0 += 2 * R) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t rb = r0 + h * R;
      if (rb >= row1) break;
      u32x4 (&cur)[R][NCH] = slot[h];
      double zr[R], qr[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        zr[r] = zs[h][r];
        qr[r] = qs[h][r];
      }
      double s[R];
      if constexpr (Op::kDot) {
        double p[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          p[r] = 0.0;
#pragma unroll
          for (int k = 0; k < NCH; ++k) {
            double x[VEC];
            unpack16<S>(cur[r][k], x);
#pragma unroll
            for (int e = 0; e < VEC; ++e) p[r] = fma(x[e], v[k][e], p[r]);
          }
        }
        const double ws = wave_sum_rows<R>(p, lane);
        if ((lane & (64 / R - 1)) == 0)
          red[parity][lane / (64 / R)][wave] = ws;
        if constexpr (kPark) {
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < NCH; ++k)
              park[(r * NCH + k) * TPB + tid] = cur[r][k];
        }
        // the slot is free once the dots are formed (or parked)
        if constexpr (kPark || !Op::kBack)
          load_block(rb + 2 * R, cur, zs[h], qs[h]);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
          double q = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) q += red[parity][r][w];
          s[r] = q;
        }
        parity ^= 1;
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] = 0.0;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double om = Op::row(a, rb + r, s[r], sums, tid == 0, zr[r], qr[r]);
        if constexpr (Op::kBack) {
#pragma unroll
          for (int k = 0; k < NCH; ++k) {
            const u32x4 w =
                kPark ? park[(r * NCH + k) * TPB + tid] : cur[r][k];
            double x[VEC];
            unpack16<S>(w, x);
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[k][e] = fma(om, x[e], acc[k][e]);
          }
        }
      }
      if constexpr (!Op::kDot) load_block(rb + 2 * R, cur, zs[h], qs[h]);
    }
  }

  if constexpr (Op::kBack) {
    double* prow = a.part + (int64_t)blockIdx.x * a.lda;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      if (!valid[k]) continue;
      int64_t c = tid + (int64_t)k * TPB;
#pragma unroll
      for (int e = 0; e < VEC; ++e) prow[c * VEC + e] = acc[k][e];
    }
  }
  if constexpr (Op::kSums > 0) {
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < Op::kSums; ++i)
        a.psums[(int64_t)blockIdx.x * kMaxSums + i] = sums[i];
    }
  }
}

// out[j] = alpha * sum_b part[b][j] + beta * y[j]   (j < n, fixed order):
// 64 columns per workgroup, 16 row groups each summing a strided subset of the
// partial rows, combined in group order.
__global__ void __launch_bounds__(1024)
reduce_partials_kernel(const double* __restrict__ part, int nwg, int64_t lda,
                       int64_t n, double alpha, double beta,
                       const double* __restrict__ y, double* __restrict__ out,
                       const int* skip) {
  if (skip && *skip) return;
  __shared__ double sh[16][64];
  const int x = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + x;
  double s = 0.0;
  if (j < n)
    for (int b = g; b < nwg; b += 16) s += part[(int64_t)b * lda + j];
  sh[g][x] = s;
  __syncthreads();
  if (g == 0 && j < n) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += sh[i][x];
    double r = alpha * t;
    if (y) r += beta * y[j];
    out[j] = r;
  }
}

// sums[i] = sum_b psums[b][i] for i < nsum (one wave per sum, fixed order).
__global__ void reduce_sums_kernel(const double* __restrict__ psums, int nwg,
                                   int nsum, double* __restrict__ out,
                                   const int* skip) {
  if (skip && *skip) return;
  int i = blockIdx.x;
  if (i >= nsum) return;
  int lane = threadIdx.x;
  double s = 0.0;
  for (int b = lane; b < nwg; b += 64) s += psums[(int64_t)b * kMaxSums + i];
  s = wave_sum(s);
  if (lane == 0) out[i] = s;
}

// ------------------------------------------------------------ launchers --

// Launch shape per storage type: the row block R grows as rows get shorter
// so one reduction serves more rows; BF16 rows are short enough that 256
// threads per row (two workgroups per CU) give each thread whole chunks.
template <typename S> struct PassShape;
template <> struct PassShape<double> {
  static constexpr int TPB = 512, R = 2, GROUPS = 256;
};
template <> struct PassShape<float> {
  static constexpr int TPB = 512, R = 4, GROUPS = 256;
};
template <> struct PassShape<bf16_t> {
  static constexpr int TPB = 256, R = 2, GROUPS = 512;
};
static_assert(PassShape<float>::GROUPS <= kMaxPassGroups, "partials buffer");
static_assert(PassShape<bf16_t>::GROUPS <= kMaxPassGroups, "partials buffer");

int pass_groups(int64_t Tp, int R, int groups, int64_t* rows_per_wg) {
  int64_t blocks = Tp / R;
  int64_t nwg = blocks < groups ? blocks : groups;
  int64_t bpw = (blocks + nwg - 1) / nwg;
  *rows_per_wg = bpw * R;
  return (int)((Tp + *rows_per_wg - 1) / *rows_per_wg);
}

// Rows per block for NCH chunks per thread: the shape's R, halved while the
// two register slots would hold more than 12 chunks of 16 bytes each per
// row block (register budget) or the parked block would exceed 128 KB.
template <typename S>
constexpr int rows_for(int nch) {
  int r = PassShape<S>::R;
  while (r > 1 && (r * nch > 12 ||
                   (int64_t)r * nch * PassShape<S>::TPB * 16 > 131072))
    r /= 2;
  return r;
}

// One instance per block height up to the shape's budget; a requested
// height above it (or 0) takes the budget's.
template <typename S, int K, class Op>
static void launch_rows(int rows, PassArgs a, dim3 g, dim3 b, hipStream_t st) {
  constexpr int TPB = PassShape<S>::TPB, RMAX = rows_for<S>(K);
  if (RMAX >= 4 && (rows == 0 || rows >= 4)) {
    hipLaunchKernelGGL((pass_kernel<S, TPB, K, (RMAX >= 4 ? 4 : 1), Op>), g,
                       b, 0, st, a);
  } else if (RMAX >= 2 && (rows == 0 || rows >= 2)) {
    hipLaunchKernelGGL((pass_kernel<S, TPB, K, (RMAX >= 2 ? 2 : 1), Op>), g,
                       b, 0, st, a);
  } else {
    hipLaunchKernelGGL((pass_kernel<S, TPB, K, 1, Op>), g, b, 0, st, a);
  }
}

template <typename S, class Op>
static hipError_t launch_nch(int nch, PassArgs a, int nwg, hipStream_t st) {
  constexpr int TPB = PassShape<S>::TPB;
  dim3 g(nwg), b(TPB);
  switch (nch) {
#define YAND_NCH_CASE(K)                           \
  case K:                                          \
    launch_rows<S, K, Op>(a.rows, a, g, b, st);    \
    break;
    YAND_NCH_CASE(1)
    YAND_NCH_CASE(2)
    YAND_NCH_CASE(3)
    YAND_NCH_CASE(4)
    YAND_NCH_CASE(5)
    YAND_NCH_CASE(6)
    YAND_NCH_CASE(7)
    YAND_NCH_CASE(8)
#undef YAND_NCH_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename S>
static hipError_t launch_pass_t(PassKind kind, PassArgs a, hipStream_t st,
                                int* nwg_out) {
  constexpr int TPB = PassShape<S>::TPB;
  constexpr int VEC = Vec16<S>::N;
  int64_t nvec = a.lda / VEC;
  int nch = (int)((nvec + TPB - 1) / TPB);
  if (nch < 1) nch = 1;
  if (nch > kMaxPassChunks) return hipErrorInvalidValue;
  // rows per workgroup: a multiple of every block height in use (R <= 8)
  int groups = a.groups > 0 ? a.groups : PassShape<S>::GROUPS;
  if (groups > kMaxPassGroups) groups = kMaxPassGroups;
  int nwg = pass_groups(a.Tp, 8, groups, &a.rows_per_wg);
  *nwg_out = nwg;
  switch (kind) {
    case PassKind::Oracle: return launch_nch<S, OpOracle>(nch, a, nwg, st);
    case PassKind::Value: return launch_nch<S, OpValue>(nch, a, nwg, st);
    case PassKind::Hvp: return launch_nch<S, OpHvp>(nch, a, nwg, st);
    case PassKind::Line: return launch_nch<S, OpLine>(nch, a, nwg, st);
    case PassKind::Dot: return launch_nch<S, OpDot>(nch, a, nwg, st);
    case PassKind::Third: return launch_nch<S, OpThird>(nch, a, nwg, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pass(int precision, PassKind kind, const PassArgs& a,
                       hipStream_t st, int* nwg) {
  switch (precision) {
    case 0: return launch_pass_t<double>(kind, a, st, nwg);
    case 1: return launch_pass_t<float>(kind, a, st, nwg);
    case 2: return launch_pass_t<bf16_t>(kind, a, st, nwg);
  }
  return hipErrorInvalidValue;
}

template <typename S>
static int rows_cap_t(int64_t lda) {
  constexpr int TPB = PassShape<S>::TPB;
  constexpr int VEC = Vec16<S>::N;
  const int nch = (int)((lda / VEC + TPB - 1) / TPB);
  return rows_for<S>(nch < 1 ? 1 : nch);
}

int pass_rows_cap(int precision, int64_t lda) {
  switch (precision) {
    case 0: return rows_cap_t<double>(lda);
    case 1: return rows_cap_t<float>(lda);
    default: return rows_cap_t<bf16_t>(lda);
  }
}

int64_t max_pass_columns(int precision) {
  switch (precision) {
    case 0: return (int64_t)kMaxPassChunks * PassShape<double>::TPB * 2;
    case 1: return (int64_t)kMaxPassChunks * PassShape<float>::TPB * 4;
    default: return (int64_t)kMaxPassChunks * PassShape<bf16_t>::TPB * 8;
  }
}

hipError_t launch_reduce_partials(const double* part, int nwg, int64_t lda,
                                  int64_t n, double alpha, double beta,
                                  const double* y, double* out,
                                  hipStream_t st, const int* skip) {
  dim3 b(1024), g((unsigned)((n + 63) / 64));
  hipLaunchKernelGGL(reduce_partials_kernel, g, b, 0, st, part, nwg, lda, n,
                     alpha, beta, y, out, skip);
  return hipGetLastError();
}

hipError_t launch_reduce_sums(const double* psums, int nwg, int nsum,
                              double* out, hipStream_t st, const int* skip) {
  hipLaunchKernelGGL(reduce_sums_kernel, dim3(nsum), dim3(64), 0, st, psums,
                     nwg, nsum, out, skip);
  return hipGetLastError();
}

hipError_t launch_center(const double* R, int64_t T, int64_t n, int64_t ldr,
                         int precision, void* A, int64_t Tp, int64_t lda,
                         double* mu, double* scratch, int* nonfinite,
                         hipStream_t st) {
  const int64_t chunk = 256;
  int64_t nchunks = (T + chunk - 1) / chunk;
  dim3 b(256);
  dim3 g1((unsigned)((n + 255) / 256), (unsigned)nchunks);
  hipLaunchKernelGGL(colsum_kernel, g1, b, 0, st, R, T, n, ldr, chunk,
                     scratch);
  dim3 g2((unsigned)((n + 255) / 256));
  hipLaunchKernelGGL(colsum_finish_kernel, g2, b, 0, st, scratch, nchunks, n,
                     T, mu, nonfinite);
  int64_t gx = (lda + 255) / 256;
  if (gx > 64) gx = 64;
  dim3 g3((unsigned)gx, (unsigned)(Tp < 16384 ? Tp : 16384));
  switch (precision) {
    case 0:
      hipLaunchKernelGGL(center_convert_kernel<double>, g3, b, 0, st, R, T, n,
                         ldr, mu, (double*)A, lda, Tp);
      break;
    case 1:
      hipLaunchKernelGGL(center_convert_kernel<float>, g3, b, 0, st, R, T, n,
                         ldr, mu, (float*)A, lda, Tp);
      break;
    case 2:
      hipLaunchKernelGGL(center_convert_kernel<bf16_t>, g3, b, 0, st, R, T,
                         n, ldr, mu, (bf16_t*)A, lda, Tp);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace yand
