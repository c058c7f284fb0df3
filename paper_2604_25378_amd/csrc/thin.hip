// Exact trace for T < n in the PCG configuration by the push-through
// identity, with no n x n matrix.
//
// With P = A V (V an orthonormal basis of the tangent space without the
// normal direction, so V V^T = P_S), S = diag(psi''(z) / T) and
// B_m = P^T S P + lambda I, the trace weights of Section 4.4 are
// q_t = p_t^T B_m^-1 p_t.  For lambda > 0 and S > 0,
//   P B_m^-1 P^T = S^-1/2 [I - lambda C^-1] S^-1/2,
//   C = S^1/2 G S^1/2 + lambda I,   G = P P^T = A P_S A^T   (T x T),
// so q_t = (1 - lambda (C^-1)_tt) / s_t.  G costs T^2 n, C's Cholesky and
// inverse T^3 / 2, instead of the n^2 T SYRK, the n^3 factorisation and the
// n^2 T trace GEMM.  The PCG solve for u never needed the factor; its
// Jacobi preconditioner takes diag(A^T S A) from one pass over A.
#include "common.h"
#include "kernels.h"
#include "vec.h"

namespace yand {

namespace {

constexpr int GT = 64;    // G tile edge
constexpr int GJ = 32;    // columns of A per LDS stage
constexpr int GTH = 256;  // threads: a 64 x 64 tile, 4 x 4 outputs each
constexpr int RT = 256;   // threads of the single-workgroup kernels

__device__ double rt_sum(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < RT / 64; ++i) s += sh[i];
  __syncthreads();
  return s;
}

__device__ double rt_min(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = INFINITY;
  for (int i = 0; i < RT / 64; ++i) s = fmin(s, sh[i]);
  __syncthreads();
  return s;
}

// Partial Gram blocks Gp[k][t][u] = sum_{j in chunk k} m_j A_tj A_uj for the
// lower tiles (u-tile <= t-tile).  blockIdx.x walks the lower tiles row by
// row, blockIdx.y the column chunks of width `chunk`.  Each thread holds a
// 4 x 4 block of the 64 x 64 tile; the stage is stored k-major in LDS.
template <typename S>
__global__ void __launch_bounds__(GTH)
gram_kernel(const S* __restrict__ A, int64_t lda, int64_t T, int64_t n,
            const double* __restrict__ mask, int64_t chunk,
            double* __restrict__ Gp, int64_t ldg) {
  int tI = 0, rem = (int)blockIdx.x;
  while (rem > tI) {
    rem -= tI + 1;
    ++tI;
  }
  const int64_t t0 = (int64_t)tI * GT, u0 = (int64_t)rem * GT;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
  __shared__ double sa[GJ][GT + 2], sb[GJ][GT + 2];
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[i][q] = 0.0;
  for (int64_t jb = j0; jb < j1; jb += GJ) {
    for (int e = tid; e < GT * GJ; e += GTH) {
      const int rr = e / GJ, cc = e % GJ;
      const int64_t j = jb + cc;
      const int64_t ta = t0 + rr, ub = u0 + rr;
      const bool inj = j < j1;
      const double m = inj ? (mask ? mask[j] : 1.0) : 0.0;
      sa[cc][rr] = (inj && ta < T) ? m * to_f64(A[ta * lda + j]) : 0.0;
      sb[cc][rr] = (inj && ub < T) ? to_f64(A[ub * lda + j]) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < GJ; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = sa[k][ty * 4 + i];
        b[i] = sb[k][tx * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] += a[i] * b[q];
    }
    __syncthreads();
  }
  double* out = Gp + (int64_t)blockIdx.y * ldg * ldg + (t0 + ty * 4) * ldg +
                u0 + tx * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) out[(int64_t)i * ldg + q] = acc[i][q];
}

// G[t][u] = sum_k Gp[k][t][u] - sum_a (A e_a)_t (A e_a)_u, lower triangle,
// t, u < T: the Gram matrix of the rows of A P_S.
__global__ void gram_finish_kernel(const double* __restrict__ Gp, int K,
                                   int64_t ldg, int64_t T,
                                   const double* __restrict__ AE, int64_t Tp,
                                   int p, double* __restrict__ G) {
  const int64_t t = blockIdx.y;
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u > t || t >= T) return;
  double v = 0.0;
  for (int k = 0; k < K; ++k) v += Gp[(int64_t)k * ldg * ldg + t * ldg + u];
  for (int a = 0; a < p; ++a) v -= AE[a * Tp + t] * AE[a * Tp + u];
  G[t * ldg + u] = v;
}

// Scales from G and s: the tangent-Hessian trace sum_t s_t G_tt, its mean
// over the tangent dimension (nfree - p), lambda = reg * mean, gamma and
// trace(B); ptbad when some s_t <= 0 or lambda <= 0 (the identity needs both
// positive).
__global__ void __launch_bounds__(RT)
thin_scale_kernel(const double* __restrict__ G, int64_t ldg, int64_t T,
                  const double* __restrict__ s, const double* __restrict__ AE,
                  int64_t Tp, int p, int64_t n, double reg,
                  const double* __restrict__ mask, DevScalars* sc) {
  __shared__ double sh[RT / 64];
  double tg = 0.0, tb = 0.0, smin = INFINITY;
  for (int64_t t = threadIdx.x; t < T; t += RT) {
    double e = 0.0;
    for (int a = 0; a < p; ++a) e += AE[a * Tp + t] * AE[a * Tp + t];
    tg += s[t] * G[t * ldg + t];
    tb += s[t] * (G[t * ldg + t] + e);
    smin = fmin(smin, s[t]);
  }
  tg = rt_sum(tg, sh);
  tb = rt_sum(tb, sh);
  smin = rt_min(smin, sh);
  if (threadIdx.x == 0) {
    const double neff = mask ? sc->nfree : (double)n;
    double gam = tb / neff;
    if (!(gam > 0.0) || !isfinite(gam)) gam = 1.0;
    double tang = tg / (neff - (double)p);
    if (!(tang > 0.0) || !isfinite(tang)) tang = gam;
    sc->tr = tb;
    sc->gamma = gam;
    sc->tang_scale = tang;
    sc->lambda = reg * tang;
    sc->ptbad = (smin > 0.0 && sc->lambda > 0.0) ? 0 : 1;
    sc->fail = 0;
  }
}

// Lower triangle of C = S^1/2 G S^1/2 + lambda I (T x T), identity on the
// padding up to ldg; the identity throughout when ptbad.
__global__ void thin_build_kernel(const double* __restrict__ G, int64_t ldg,
                                  int64_t T, const double* __restrict__ s,
                                  const DevScalars* __restrict__ sc,
                                  double* __restrict__ C) {
  const int64_t t = blockIdx.y;
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u > t || t >= ldg) return;
  double v = t == u ? 1.0 : 0.0;
  if (!sc->ptbad && t < T)
    v = sqrt(s[t]) * G[t * ldg + u] * sqrt(s[u]) + (t == u ? sc->lambda : 0.0);
  C[t * ldg + u] = v;
}

// Partial column norms of X = L^-1 (lower, row-major): part[b][t] =
// sum_{i in rows [64 b, 64 b + 64), i >= t, i < T} X_it^2; a workgroup takes
// 64 columns and 64 rows (4 groups of 16 rows, summed in LDS).
__global__ void __launch_bounds__(256)
thin_colnorm_kernel(const double* __restrict__ X, int64_t ldg, int64_t T,
                    double* __restrict__ part) {
  __shared__ double sh[4][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t t = (int64_t)blockIdx.x * 64 + c;
  const int64_t i0 = (int64_t)blockIdx.y * 64 + g * 16;
  double v = 0.0;
  if (t < T)
    for (int64_t i = i0 > t ? i0 : t; i < i0 + 16 && i < T; ++i) {
      const double x = X[i * ldg + t];
      v += x * x;
    }
  sh[g][c] = v;
  __syncthreads();
  if (g == 0 && t < T)
    part[(int64_t)blockIdx.y * ldg + t] = sh[0][c] + sh[1][c] + sh[2][c] +
                                          sh[3][c];
}

// q_t = (1 - lambda (C^-1)_tt) / s_t with (C^-1)_tt the sum of the nb
// partial column norms; 0 on the padding rows.
__global__ void thin_q_kernel(const double* __restrict__ part, int nb,
                              int64_t ldg, int64_t T, int64_t Tp,
                              const double* __restrict__ s,
                              const DevScalars* __restrict__ sc,
                              double* __restrict__ q) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Tp) return;
  if (t >= T) {
    q[t] = 0.0;
    return;
  }
  double c = 0.0;
  for (int b = 0; b < nb; ++b) c += part[(int64_t)b * ldg + t];
  q[t] = (1.0 - sc->lambda * c) / s[t];
}

// Partial Jacobi diagonal: part[b][j] = sum_{t in [16 b, 16 b + 16), t < T}
// s_t A_tj^2; bd_j = sum_b part[b][j] = diag(A^T S A).
constexpr int kBdRows = 16;
template <typename S>
__global__ void bdiag_part_kernel(const S* __restrict__ A, int64_t lda,
                                  int64_t T, int64_t n,
                                  const double* __restrict__ s,
                                  double* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t t0 = (int64_t)blockIdx.y * kBdRows;
  double v = 0.0;
  for (int64_t t = t0; t < t0 + kBdRows && t < T; ++t) {
    const double a = to_f64(A[t * lda + j]);
    v += s[t] * a * a;
  }
  part[(int64_t)blockIdx.y * lda + j] = v;
}

__global__ void bdiag_sum_kernel(const double* __restrict__ part, int nb,
                                 int64_t lda, int64_t n,
                                 double* __restrict__ bd) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double v = 0.0;
  for (int b = 0; b < nb; ++b) v += part[(int64_t)b * lda + j];
  bd[j] = v;
}

template <typename S>
hipError_t gram_t(const void* A, int64_t lda, int64_t T, int64_t n,
                  const double* mask, int K, double* Gp, int64_t ldg,
                  hipStream_t st) {
  const int nT = (int)((T + GT - 1) / GT);
  const int ntile = nT * (nT + 1) / 2;
  int64_t chunk = (n + K - 1) / K;
  chunk = (chunk + GJ - 1) / GJ * GJ;
  hipLaunchKernelGGL(gram_kernel<S>, dim3(ntile, K), dim3(GTH), 0, st,
                     (const S*)A, lda, T, n, mask, chunk, Gp, ldg);
  return hipGetLastError();
}

template <typename S>
hipError_t bdiag_t(const void* A, int64_t lda, int64_t T, int64_t n,
                   const double* s, double* part, double* bd, hipStream_t st) {
  const int nb = (int)((T + kBdRows - 1) / kBdRows);
  hipLaunchKernelGGL(bdiag_part_kernel<S>,
                     dim3((unsigned)((n + 255) / 256), (unsigned)nb),
                     dim3(256), 0, st, (const S*)A, lda, T, n, s, part);
  hipLaunchKernelGGL(bdiag_sum_kernel, dim3((unsigned)((n + 255) / 256)),
                     dim3(256), 0, st, part, nb, lda, n, bd);
  return hipGetLastError();
}

}  // namespace

int thin_splits(int64_t T) {
  const int64_t nT = (T + GT - 1) / GT;
  const int64_t ntile = nT * (nT + 1) / 2;
  const int64_t ldg = round_up(T, 128);
  int64_t K = (1024 + ntile - 1) / ntile;
  // partials at most 64 MiB
  const int64_t kmem = ((int64_t)64 << 20) / (ldg * ldg * 8);
  if (K > kmem) K = kmem;
  return (int)(K < 1 ? 1 : (K > 64 ? 64 : K));
}

int64_t thin_part_rows(int64_t T) {
  const int64_t a = (T + 63) / 64, b = (T + kBdRows - 1) / kBdRows;
  return a > b ? a : b;
}

hipError_t launch_thin_gram(int precision, const void* A, int64_t lda,
                            int64_t T, int64_t n, const double* mask, int K,
                            double* Gp, int64_t ldg, const double* AE,
                            int64_t Tp, int p, double* G, hipStream_t st) {
  hipError_t e;
  switch (precision) {
    case 1: e = gram_t<float>(A, lda, T, n, mask, K, Gp, ldg, st); break;
    case 2: e = gram_t<bf16_t>(A, lda, T, n, mask, K, Gp, ldg, st); break;
    default: e = gram_t<double>(A, lda, T, n, mask, K, Gp, ldg, st); break;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_finish_kernel,
                     dim3((unsigned)((T + 255) / 256), (unsigned)T), dim3(256),
                     0, st, Gp, K, ldg, T, AE, Tp, p, G);
  return hipGetLastError();
}

hipError_t launch_thin_factor_input(const double* G, int64_t ldg, int64_t T,
                                    const double* s, const double* AE,
                                    int64_t Tp, int p, int64_t n, double reg,
                                    const double* mask, DevScalars* sc,
                                    double* C, hipStream_t st) {
  hipLaunchKernelGGL(thin_scale_kernel, dim3(1), dim3(RT), 0, st, G, ldg, T, s,
                     AE, Tp, p, n, reg, mask, sc);
  hipLaunchKernelGGL(thin_build_kernel,
                     dim3((unsigned)((ldg + 255) / 256), (unsigned)ldg),
                     dim3(256), 0, st, G, ldg, T, s, sc, C);
  return hipGetLastError();
}

hipError_t launch_thin_q(const double* X, int64_t ldg, int64_t T, int64_t Tp,
                         const double* s, const DevScalars* sc, double* part,
                         double* q, hipStream_t st) {
  const int nb = (int)((T + 63) / 64);
  hipLaunchKernelGGL(thin_colnorm_kernel, dim3((unsigned)nb, (unsigned)nb),
                     dim3(256), 0, st, X, ldg, T, part);
  hipLaunchKernelGGL(thin_q_kernel, dim3((unsigned)((Tp + 255) / 256)),
                     dim3(256), 0, st, part, nb, ldg, T, Tp, s, sc, q);
  return hipGetLastError();
}

hipError_t launch_bdiag(int precision, const void* A, int64_t lda, int64_t T,
                        int64_t n, const double* s, double* part, double* bd,
                        hipStream_t st) {
  switch (precision) {
    case 1: return bdiag_t<float>(A, lda, T, n, s, part, bd, st);
    case 2: return bdiag_t<bf16_t>(A, lda, T, n, s, part, bd, st);
    default: return bdiag_t<double>(A, lda, T, n, s, part, bd, st);
  }
}

}  // namespace yand
