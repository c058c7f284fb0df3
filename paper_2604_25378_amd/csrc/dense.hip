// Dense FP64 kernels of the exact trace (MFMA-bound).
//
// The exact log-det correction needs q_t = a_t^T K a_t for every bar, with
// K = V (V^T H V + lambda I)^-1 V^T the inverse tangent Hessian on the
// tangent space S of the level set (Section 4.2).  The library forms
//     M = P_S B P_S + lambda P_S + gamma (I - P_S),   B = A^T diag(psi'') A / T,
// factors M = L L^T, inverts X = L^-1 and reads q_t = |X a_t|^2 minus the
// rank-p correction of the (I - P_S) block.  Every contraction here runs on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64) in 128 x 128 output tiles:
// 256 threads = 4 waves in a 2 x 2 grid, each wave 64 x 64 = 4 x 4 MFMA
// blocks; operands are staged through LDS k-major (contiguous along m / n).
#include "common.h"
#include "kernels.h"

namespace yand {
namespace {

constexpr int BM = kTile;
constexpr int BKK = 16;
constexpr int NT = 256;
constexpr int LDP = BM + 1;   // padded LDS row (k-major tiles)

// Loads one BKK-deep slice of a 128-wide operand into registers and writes it
// to LDS as s[k][m] (FP64).  KC: element (m, k) at base[m * ld + k] (contiguous
// in k); otherwise element (m, k) at base[k * ld + m] (contiguous in m).
template <typename T, bool KC>
struct Stage {
  static constexpr int VEC = Vec16<T>::N;
  static constexpr int PER = BM * BKK / VEC / NT;
  u32x4 r[PER];

  __device__ __forceinline__ void load(const T* base, int64_t ld, int64_t k0,
                                       int tid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      int idx = tid + i * NT;
      const T* p;
      if constexpr (KC) {
        constexpr int CPR = BKK / VEC;
        int m = idx / CPR, k = (idx % CPR) * VEC;
        p = base + (int64_t)m * ld + k0 + k;
      } else {
        constexpr int CPR = BM / VEC;
        int k = idx / CPR, m = (idx % CPR) * VEC;
        p = base + (k0 + k) * ld + m;
      }
      r[i] = *(const u32x4*)p;
    }
  }

  __device__ __forceinline__ void store(double* s, int tid,
                                        const double* scale, int64_t k0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      int idx = tid + i * NT;
      double x[VEC];
      unpack16<T>(r[i], x);
      if constexpr (KC) {
        constexpr int CPR = BKK / VEC;
        int m = idx / CPR, k = (idx % CPR) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          double sc = scale ? scale[k0 + k + e] : 1.0;
          s[(k + e) * LDP + m] = x[e] * sc;
        }
      } else {
        constexpr int CPR = BM / VEC;
        int k = idx / CPR, m = (idx % CPR) * VEC;
        double sc = scale ? scale[k0 + k] : 1.0;
#pragma unroll
        for (int e = 0; e < VEC; ++e) s[k * LDP + m + e] = x[e] * sc;
      }
    }
  }
};

__device__ __forceinline__ void mma_slice(const double* sA, const double* sB,
                                          f64x4 (&acc)[4][4], int wm, int wn,
                                          int lane) {
#pragma unroll
  for (int kk = 0; kk < BKK; kk += 4) {
    const int kr = kk + (lane >> 4), c = lane & 15;
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = sA[kr * LDP + wm + i * 16 + c];
      b[i] = sB[kr * LDP + wn + i * 16 + c];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j],
                                                         acc[i][j], 0, 0, 0);
  }
}

// acc (this wave's 64 x 64 block) = sum_{k in [kbeg, kend)} opA(m,k) opB(k,n),
// opB optionally scaled by bscale[k].  kend - kbeg must be a multiple of BKK.
template <typename TA, bool AKC, typename TB, bool BKC>
__device__ void gemm_core(const TA* Ab, int64_t lda, const TB* Bb,
                          int64_t ldb, const double* bscale, int64_t kbeg,
                          int64_t kend, f64x4 (&acc)[4][4], double* sA,
                          double* sB) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (kbeg >= kend) return;
  Stage<TA, AKC> sa;
  Stage<TB, BKC> sb;
  sa.load(Ab, lda, kbeg, tid);
  sb.load(Bb, ldb, kbeg, tid);
  sa.store(sA, tid, nullptr, kbeg);
  sb.store(sB, tid, bscale, kbeg);
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < kend; k0 += BKK) {
    const bool more = k0 + BKK < kend;
    if (more) {
      sa.load(Ab, lda, k0 + BKK, tid);
      sb.load(Bb, ldb, k0 + BKK, tid);
    }
    mma_slice(sA, sB, acc, wm, wn, lane);
    __syncthreads();
    if (more) {
      sa.store(sA, tid, nullptr, k0 + BKK);
      sb.store(sB, tid, bscale, k0 + BKK);
      __syncthreads();
    }
  }
}

// Visit this wave's accumulator entries as (row, col) inside the 128 x 128
// tile: D[row][col] of 16x16x4 f64 MFMA block (i, j) is held by lane l in
// register r with row = l / 16 + 4 r and col = l % 16 (gfx950 layout).
template <class F>
__device__ __forceinline__ void for_each_acc(const f64x4 (&acc)[4][4], F f) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        f(wm + i * 16 + (lane >> 4) + 4 * r, wn + j * 16 + (lane & 15),
          acc[i][j][r]);
}

__device__ __forceinline__ void lower_tile(int64_t b, int* I, int* J) {
  int i = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((int64_t)i * (i + 1) / 2 > b) --i;
  while ((int64_t)(i + 1) * (i + 2) / 2 <= b) ++i;
  *I = i;
  *J = (int)(b - (int64_t)i * (i + 1) / 2);
}

// ------------------------------------------------------------------ SYRK --
// B = A^T diag(s) A, lower tiles computed, written to both triangles.
template <typename S>
__global__ void __launch_bounds__(NT) syrk_kernel(const S* __restrict__ A,
                                                  int64_t lda, int64_t Tp,
                                                  const double* __restrict__ s,
                                                  double* __restrict__ B,
                                                  const int* skip) {
  if (skip && *skip) return;
  __shared__ double sA[BKK * LDP], sB[BKK * LDP];
  int I, J;
  lower_tile(blockIdx.x, &I, &J);
  f64x4 acc[4][4];
  gemm_core<S, false, S, false>(A + (int64_t)I * BM, lda, A + (int64_t)J * BM,
                                lda, s, 0, Tp, acc, sA, sB);
  double* Bij = B + (int64_t)I * BM * lda + (int64_t)J * BM;
  double* Bji = B + (int64_t)J * BM * lda + (int64_t)I * BM;
  const bool mirror = I != J;
  for_each_acc(acc, [&](int r, int c, double v) {
    Bij[(int64_t)r * lda + c] = v;
    if (mirror) Bji[(int64_t)c * lda + r] = v;
  });
}

// ------------------------------------------------------- trace row norms --
// rn[J][t] = sum_{j in tile J} (sum_k A[t][k] X[j][k])^2 for X lower.
template <typename S>
__global__ void __launch_bounds__(NT)
trace_gemm_kernel(const S* __restrict__ A, int64_t lda, int64_t Tp,
                  const double* __restrict__ X, int64_t ldx,
                  double* __restrict__ rn, const int* skip) {
  if (skip && *skip) return;
  __shared__ double sA[BKK * LDP], sB[BKK * LDP];
  __shared__ double rows[2][BM];
  const int J = blockIdx.x;
  const int64_t t0 = (int64_t)blockIdx.y * BM;
  f64x4 acc[4][4];
  gemm_core<S, true, double, true>(A + t0 * lda, lda,
                                   X + (int64_t)J * BM * ldx, ldx, nullptr, 0,
                                   (int64_t)(J + 1) * BM, acc, sA, sB);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) v += acc[i][j][r] * acc[i][j][r];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      if ((lane & 15) == 0) rows[w & 1][wm + i * 16 + (lane >> 4) + 4 * r] = v;
    }
  __syncthreads();
  if (tid < BM) rn[(int64_t)J * Tp + t0 + tid] = rows[0][tid] + rows[1][tid];
}

// ------------------------------------------------------ blocked Cholesky --
// Diagonal block k: Cholesky of the 128 x 128 block in LDS and its inverse,
// blocked in 32-column sub-panels.  Wave 0 factors and inverts each 32 x 32
// diagonal sub-block in registers (lane r owns row r; column values move by
// lane shuffles); the panel below is L21 = A21 X11^T and the trailing update
// A22 -= L21 L21^T, both spread over all threads.  The inverse is assembled
// from the last sub-panel: X21 = -(X22 L21) X11.  X11 blocks are parked
// transposed in the free upper triangle.  L_kk goes to M (lower) and L_kk^-1
// to the diagonal block of X.  LDS rows are padded to 129 doubles.
constexpr int DT = 512;      // threads of the diagonal-block kernel
constexpr int SB = 32;       // sub-panel width
constexpr int LDD = BM + 1;  // padded LDS row

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(DT) diag_block_kernel(double* M, double* X,
                                                        int64_t ld, int k,
                                                        int* fail,
                                                        const int* skip) {
  if (skip && *skip) return;
  extern __shared__ double L[];  // BM x LDD
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Mk = M + (int64_t)k * BM * ld + (int64_t)k * BM;
  double* Xk = X + (int64_t)k * BM * ld + (int64_t)k * BM;
  constexpr int PER = BM * BM / DT;   // 32 elements per thread
  {
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * DT, i = idx / BM, c = idx % BM;
      v[q] = c <= i ? Mk[(int64_t)i * ld + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * DT, i = idx / BM, c = idx % BM;
      L[i * LDD + c] = v[q];
    }
  }
  __syncthreads();
  for (int c0 = 0; c0 < BM; c0 += SB) {
    if (wave == 0) {
      const int r = lane & (SB - 1);
      double a[SB];
#pragma unroll
      for (int j = 0; j < SB; ++j) a[j] = L[(c0 + r) * LDD + c0 + j];
      bool bad = false;
#pragma unroll
      for (int j = 0; j < SB; ++j) {
        double p = __shfl(a[j], j, 64);
        if (!(p > 0.0) || !isfinite(p)) {
          bad = true;
          p = 1.0;
        }
        const double piv = sqrt(p);
        if (r == j) a[j] = piv;
        if (r > j) a[j] /= piv;
#pragma unroll
        for (int c = j + 1; c < SB; ++c) {
          const double lcj = __shfl(a[j], c, 64);
          if (c <= r) a[c] -= a[j] * lcj;
        }
      }
      if (bad && lane == 0) atomicOr(fail, 1);
      if (lane < SB) {
#pragma unroll
        for (int j = 0; j < SB; ++j)
          if (j <= r) L[(c0 + r) * LDD + c0 + j] = a[j];
      }
      wave_sync();
      // column r of X11 = L11^-1 by forward substitution (lane r -> column
      // r): X11[i][r] for i > r is parked at (c0 + r, c0 + i), in the free
      // upper part of row r, and read back from there.
      if (lane < SB) {
        double* pr = L + (c0 + r) * LDD + c0;
        const double xr = 1.0 / pr[r];
        for (int i = r + 1; i < SB; ++i) {
          const double* li = L + (c0 + i) * LDD + c0;
          double v = li[r] * xr;
#pragma unroll 4
          for (int m = r + 1; m < i; ++m) v += li[m] * pr[m];
          pr[i] = -v / li[i];
        }
      }
    }
    __syncthreads();
    const int r0 = c0 + SB, rem = BM - r0;
    if (rem == 0) break;
    // L21[i][j] = sum_{m<=j} A21[i][m] X11[j][m]; results staged in registers
    {
      constexpr int MAXO = (BM - SB) * SB / DT;   // 6
      double o[MAXO];
#pragma unroll
      for (int q = 0; q < MAXO; ++q) {
        const int idx = tid + q * DT, i = idx / SB, j = idx % SB;
        double v = 0.0;
        if (i < rem) {
          const double* ai = L + (r0 + i) * LDD + c0;
          for (int m = 0; m < j; ++m)
            v += ai[m] * L[(c0 + m) * LDD + c0 + j];   // X11[j][m], m < j
          v += ai[j] / L[(c0 + j) * LDD + c0 + j];     // X11[j][j]
        }
        o[q] = v;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < MAXO; ++q) {
        const int idx = tid + q * DT, i = idx / SB, j = idx % SB;
        if (i < rem) L[(r0 + i) * LDD + c0 + j] = o[q];
      }
    }
    __syncthreads();
    // trailing update A22 -= L21 L21^T (lower part)
    for (int idx = tid; idx < rem * rem; idx += DT) {
      const int i = r0 + idx / rem, c = r0 + idx % rem;
      if (c > i) continue;
      const double* li = L + i * LDD + c0;
      const double* lc = L + c * LDD + c0;
      double v = 0.0;
#pragma unroll 8
      for (int m = 0; m < SB; ++m) v += li[m] * lc[m];
      L[i * LDD + c] -= v;
    }
    __syncthreads();
  }
  // write L_kk (lower)
  for (int idx = tid; idx < BM * BM; idx += DT) {
    const int i = idx / BM, c = idx % BM;
    Mk[(int64_t)i * ld + c] = c <= i ? L[i * LDD + c] : 0.0;
  }
  __syncthreads();
  // ---- assemble the inverse, sub-panels from the last ---------------------
  for (int c0 = BM - SB; c0 >= 0; c0 -= SB) {
    const int r0 = c0 + SB, rem = BM - r0;
    // T[i][c] = sum_{m<=i} X[r0+i][r0+m] L[r0+m][c0+c], parked at (c0+c, r0+i)
    if (rem > 0) {
      for (int idx = tid; idx < rem * SB; idx += DT) {
        const int i = idx / SB, c = idx % SB;
        const double* xi = L + (r0 + i) * LDD + r0;
        double v = 0.0;
        for (int m = 0; m <= i; ++m) v += xi[m] * L[(r0 + m) * LDD + c0 + c];
        L[(c0 + c) * LDD + r0 + i] = v;
      }
    }
    __syncthreads();
    // move X11 into the lower part of the sub-block
    {
      double v[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int idx = tid + q * DT, i = idx / SB, c = idx % SB;
        v[q] = i > c ? L[(c0 + c) * LDD + c0 + i]
                     : (i == c ? 1.0 / L[(c0 + i) * LDD + c0 + i] : 0.0);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int idx = tid + q * DT, i = idx / SB, c = idx % SB;
        if (i >= c) L[(c0 + i) * LDD + c0 + c] = v[q];
      }
    }
    __syncthreads();
    // X[r0+i][c0+c] = -sum_{m>=c} T[i][m] X11[m][c]
    if (rem > 0) {
      for (int idx = tid; idx < rem * SB; idx += DT) {
        const int i = idx / SB, c = idx % SB;
        double v = 0.0;
        for (int m = c; m < SB; ++m)
          v += L[(c0 + m) * LDD + r0 + i] * L[(c0 + m) * LDD + c0 + c];
        L[(r0 + i) * LDD + c0 + c] = -v;
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < BM * BM; idx += DT) {
    const int i = idx / BM, c = idx % BM;
    Xk[(int64_t)i * ld + c] = c <= i ? L[i * LDD + c] : 0.0;
  }
}

// L[I, k] = M[I, k] L_kk^-T for I > k (in place).
__global__ void __launch_bounds__(NT) panel_kernel(double* M,
                                                   const double* X,
                                                   int64_t ld, int k,
                                                   const int* skip) {
  if (skip && *skip) return;
  __shared__ double sA[BKK * LDP], sB[BKK * LDP];
  const int I = k + 1 + blockIdx.x;
  double* Mik = M + (int64_t)I * BM * ld + (int64_t)k * BM;
  const double* Xkk = X + (int64_t)k * BM * ld + (int64_t)k * BM;
  f64x4 acc[4][4];
  gemm_core<double, true, double, true>(Mik, ld, Xkk, ld, nullptr, 0, BM, acc,
                                        sA, sB);
  for_each_acc(acc, [&](int r, int c, double v) { Mik[(int64_t)r * ld + c] = v; });
}

// M[I, J] -= L[I, k] L[J, k]^T for k < J <= I.
__global__ void __launch_bounds__(NT) update_kernel(double* M, int64_t ld,
                                                    int k, const int* skip) {
  if (skip && *skip) return;
  __shared__ double sA[BKK * LDP], sB[BKK * LDP];
  int I, J;
  lower_tile(blockIdx.x, &I, &J);
  I += k + 1;
  J += k + 1;
  const double* Lik = M + (int64_t)I * BM * ld + (int64_t)k * BM;
  const double* Ljk = M + (int64_t)J * BM * ld + (int64_t)k * BM;
  f64x4 acc[4][4];
  gemm_core<double, true, double, true>(Lik, ld, Ljk, ld, nullptr, 0, BM, acc,
                                        sA, sB);
  double* Mij = M + (int64_t)I * BM * ld + (int64_t)J * BM;
  for_each_acc(acc, [&](int r, int c, double v) { Mij[(int64_t)r * ld + c] -= v; });
}

// X[k, j] = -L_kk^-1 S[k, j] for j < k (S accumulated in place in X).
__global__ void __launch_bounds__(NT) inv_finalize_kernel(double* X,
                                                          int64_t ld, int k,
                                                          const int* skip) {
  if (skip && *skip) return;
  __shared__ double sA[BKK * LDP], sB[BKK * LDP];
  const int j = blockIdx.x;
  const double* Xkk = X + (int64_t)k * BM * ld + (int64_t)k * BM;
  double* Skj = X + (int64_t)k * BM * ld + (int64_t)j * BM;
  f64x4 acc[4][4];
  gemm_core<double, true, double, false>(Xkk, ld, Skj, ld, nullptr, 0, BM, acc,
                                         sA, sB);
  for_each_acc(acc, [&](int r, int c, double v) { Skj[(int64_t)r * ld + c] = -v; });
}

// S[i, j] += L[i, k] X[k, j] for i > k, j <= k.
__global__ void __launch_bounds__(NT) inv_update_kernel(double* X,
                                                        const double* M,
                                                        int64_t ld, int k,
                                                        const int* skip) {
  if (skip && *skip) return;
  __shared__ double sA[BKK * LDP], sB[BKK * LDP];
  const int i = k + 1 + blockIdx.x / (k + 1);
  const int j = blockIdx.x % (k + 1);
  const double* Lik = M + (int64_t)i * BM * ld + (int64_t)k * BM;
  const double* Xkj = X + (int64_t)k * BM * ld + (int64_t)j * BM;
  f64x4 acc[4][4];
  gemm_core<double, true, double, false>(Lik, ld, Xkj, ld, nullptr, 0, BM, acc,
                                         sA, sB);
  double* Sij = X + (int64_t)i * BM * ld + (int64_t)j * BM;
  for_each_acc(acc, [&](int r, int c, double v) { Sij[(int64_t)r * ld + c] += v; });
}

// ------------------------------------------------------ matrix-vectors ----
// y = X v, X lower (np x np); one wave per row, rows < n.
__global__ void trmv_n_kernel(const double* __restrict__ X, int64_t ld,
                              int64_t n, const double* __restrict__ v,
                              double* __restrict__ y, const int* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t k = lane; k <= i; k += 64) s += X[i * ld + k] * v[k];
  s = wave_sum(s);
  if (lane == 0) y[i] = s;
}

// part[b][j] = sum_{i in rows of block b, i >= j} X[i][j] v[i].
constexpr int kTrmvRows = 64;
__global__ void trmv_t_kernel(const double* __restrict__ X, int64_t ld,
                              int64_t n, const double* __restrict__ v,
                              double* __restrict__ part, const int* skip) {
  if (skip && *skip) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * kTrmvRows;
  if (j >= n) return;
  int64_t i1 = i0 + kTrmvRows < n ? i0 + kTrmvRows : n;
  double s = 0.0;
  for (int64_t i = i0 > j ? i0 : j; i < i1; ++i) s += X[i * ld + j] * v[i];
  part[(int64_t)blockIdx.y * n + j] = s;
}

// W[a*n + i] = sum_j B[i][j] E[a*n + j], a < p (B full symmetric).
__global__ void symm_multi_kernel(const double* __restrict__ B, int64_t ld,
                                  int64_t n, const double* __restrict__ E,
                                  int p, double* __restrict__ W,
                                  const int* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t j = lane; j < n; j += 64) {
    double b = B[i * ld + j];
    for (int a = 0; a < p; ++a) s[a] += b * E[a * n + j];
  }
  for (int a = 0; a < p; ++a) {
    double t = wave_sum(s[a]);
    if (lane == 0) W[a * n + i] = t;
  }
}

}  // namespace

// ------------------------------------------------------------ launchers --

hipError_t launch_syrk(int precision, const void* A, int64_t lda, int64_t Tp,
                       const double* s, double* B, hipStream_t st,
                       const int* skip) {
  const int64_t nt = lda / BM;
  dim3 g((unsigned)(nt * (nt + 1) / 2)), b(NT);
  switch (precision) {
    case 0:
      hipLaunchKernelGGL(syrk_kernel<double>, g, b, 0, st, (const double*)A,
                         lda, Tp, s, B, skip);
      break;
    case 1:
      hipLaunchKernelGGL(syrk_kernel<float>, g, b, 0, st, (const float*)A, lda,
                         Tp, s, B, skip);
      break;
    case 2:
      hipLaunchKernelGGL(syrk_kernel<bf16_t>, g, b, 0, st, (const bf16_t*)A,
                         lda, Tp, s, B, skip);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t prepare_dense_kernels() {
  static bool attr_set = false;
  if (!attr_set) {
    const size_t lds = (size_t)BM * LDD * sizeof(double);
    hipError_t e = hipFuncSetAttribute(
        (const void*)diag_block_kernel,
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  return hipSuccess;
}

hipError_t launch_potrf_trtri(double* M, double* X, int64_t np, int* fail,
                              hipStream_t st, const int* skip) {
  const int nt = (int)(np / BM);
  const size_t lds = (size_t)BM * LDD * sizeof(double);
  hipError_t pe = prepare_dense_kernels();
  if (pe != hipSuccess) return pe;
  for (int k = 0; k < nt; ++k) {
    hipLaunchKernelGGL(diag_block_kernel, dim3(1), dim3(DT), lds, st, M, X,
                       np, k, fail, skip);
    const int rem = nt - k - 1;
    if (rem > 0)
      hipLaunchKernelGGL(panel_kernel, dim3(rem), dim3(NT), 0, st, M,
                         (const double*)X, np, k, skip);
    if (k > 0)
      hipLaunchKernelGGL(inv_finalize_kernel, dim3(k), dim3(NT), 0, st, X, np,
                         k, skip);
    if (rem > 0) {
      hipLaunchKernelGGL(update_kernel, dim3(rem * (rem + 1) / 2), dim3(NT), 0,
                         st, M, np, k, skip);
      hipLaunchKernelGGL(inv_update_kernel, dim3(rem * (k + 1)), dim3(NT), 0,
                         st, X, (const double*)M, np, k, skip);
    }
  }
  return hipGetLastError();
}

hipError_t launch_trace_gemm(int precision, const void* A, int64_t lda,
                             int64_t Tp, const double* X, int64_t np,
                             double* rn, hipStream_t st, const int* skip) {
  dim3 g((unsigned)(np / BM), (unsigned)(Tp / BM)), b(NT);
  switch (precision) {
    case 0:
      hipLaunchKernelGGL(trace_gemm_kernel<double>, g, b, 0, st,
                         (const double*)A, lda, Tp, X, np, rn, skip);
      break;
    case 1:
      hipLaunchKernelGGL(trace_gemm_kernel<float>, g, b, 0, st,
                         (const float*)A, lda, Tp, X, np, rn, skip);
      break;
    case 2:
      hipLaunchKernelGGL(trace_gemm_kernel<bf16_t>, g, b, 0, st,
                         (const bf16_t*)A, lda, Tp, X, np, rn, skip);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_trmv(const double* X, int64_t np, int64_t n,
                       const double* v, double* y, double* part, bool trans,
                       hipStream_t st, const int* skip) {
  if (!trans) {
    hipLaunchKernelGGL(trmv_n_kernel, dim3((unsigned)((n + 3) / 4)),
                       dim3(256), 0, st, X, np, n, v, y, skip);
    return hipGetLastError();
  }
  const int64_t nb = (n + kTrmvRows - 1) / kTrmvRows;
  hipLaunchKernelGGL(trmv_t_kernel,
                     dim3((unsigned)((n + 255) / 256), (unsigned)nb),
                     dim3(256), 0, st, X, np, n, v, part, skip);
  return launch_reduce_partials(part, (int)nb, n, n, 1.0, 0.0, nullptr, y,
                                st, skip);
}

hipError_t launch_symm_multi(const double* B, int64_t ldb, int64_t n,
                             const double* E, int p, double* W,
                             hipStream_t st, const int* skip) {
  hipLaunchKernelGGL(symm_multi_kernel, dim3((unsigned)((n + 3) / 4)),
                     dim3(256), 0, st, B, ldb, n, E, p, W, skip);
  return hipGetLastError();
}

}  // namespace yand
