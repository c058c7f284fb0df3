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
//
// Indefinite S (some psi'' < 0, none zero).  By Woodbury, for any
// invertible S, P B_m^-1 P^T = S^-1 - lambda S^-1 W^-1 S^-1 with
// W = lambda S^-1 + G, so q_t = (1 - lambda (W^-1)_tt / s_t) / s_t (C above
// is S^1/2 W S^1/2).  W is indefinite; with the bars of positive s first,
//   W = [[W_PP, W_PN], [W_NP, W_NN]],  W_PP = L1 L1^T,
//   Sigma = W_NN - W_NP W_PP^-1 W_PN = -L2 L2^T,
// a signed factorisation W = L diag(I, -I) L^T that exists exactly when
// B_m is positive definite: by Haynsworth's inertia additivity applied to
// [[lambda I, P^T], [P, -S^-1]], nu_-(B_m) = nu_+(W) - nu_+(S), and
// nu_+(W) = nu_+(W_PP) + nu_+(Sigma) = |P| + nu_+(Sigma), so B_m > 0 iff
// -Sigma > 0.  Both factors are Cholesky factors (the blocked kernels of
// the dense route); a failed one means B_m is not positive definite and the
// caller raises lambda, as the dense route does.  With X1 = L1^-1,
// M^T = X1 W_PN, X2 = L2^-1 and Y = X2 M X1,
//   (W^-1)_tt = |X1 e_t|^2 - |Y e_t|^2  (t among the positive bars),
//   (W^-1)_tt = -|X2 e_t|^2              (t among the negative bars).
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
// trace(B); sneg, the bars with s_t < 0; ptbad when some s_t is zero or not
// finite, or lambda <= 0 (the identity needs S invertible and lambda > 0).
__global__ void __launch_bounds__(RT)
thin_scale_kernel(const double* __restrict__ G, int64_t ldg, int64_t T,
                  const double* __restrict__ s, const double* __restrict__ AE,
                  int64_t Tp, int p, int64_t n, double reg,
                  const double* __restrict__ mask, DevScalars* sc) {
  __shared__ double sh[RT / 64];
  double tg = 0.0, tb = 0.0, nneg = 0.0, nbad = 0.0;
  for (int64_t t = threadIdx.x; t < T; t += RT) {
    double e = 0.0;
    for (int a = 0; a < p; ++a) e += AE[a * Tp + t] * AE[a * Tp + t];
    tg += s[t] * G[t * ldg + t];
    tb += s[t] * (G[t * ldg + t] + e);
    nneg += s[t] < 0.0 ? 1.0 : 0.0;
    nbad += (s[t] != 0.0 && isfinite(s[t])) ? 0.0 : 1.0;
  }
  tg = rt_sum(tg, sh);
  tb = rt_sum(tb, sh);
  nneg = rt_sum(nneg, sh);
  nbad = rt_sum(nbad, sh);
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
    sc->sneg = (int)nneg;
    sc->ptbad = (nbad == 0.0 && sc->lambda > 0.0) ? 0 : 1;
    sc->fail = 0;
  }
}

// Lower triangle of C = S^1/2 G S^1/2 + lambda I (T x T), identity on the
// padding up to ldg; the identity throughout when ptbad or S is indefinite.
__global__ void thin_build_kernel(const double* __restrict__ G, int64_t ldg,
                                  int64_t T, const double* __restrict__ s,
                                  const DevScalars* __restrict__ sc,
                                  double* __restrict__ C) {
  const int64_t t = blockIdx.y;
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u > t || t >= ldg) return;
  double v = t == u ? 1.0 : 0.0;
  if (!sc->ptbad && !sc->sneg && t < T)
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

// Indefinite S: bars of positive s_t first, each set in bar order
// (perm[i] = bar at position i, pos[t] = position of bar t).
__global__ void thin_perm_kernel(const double* __restrict__ s, int64_t T,
                                 int* __restrict__ perm, int* __restrict__ pos) {
  if (threadIdx.x != 0) return;
  int k = 0;
  for (int64_t t = 0; t < T; ++t)
    if (s[t] > 0.0) {
      perm[k] = (int)t;
      pos[t] = k++;
    }
  for (int64_t t = 0; t < T; ++t)
    if (!(s[t] > 0.0)) {
      perm[k] = (int)t;
      pos[t] = k++;
    }
}

__device__ __forceinline__ double gsym(const double* G, int64_t ldg, int a,
                                       int b) {
  return a >= b ? G[(int64_t)a * ldg + b] : G[(int64_t)b * ldg + a];
}

// The blocks of the permuted W = lambda S^-1 + G: W_PP (ldp x ldp, the
// identity on its padding), W_PN (ldp x ldn, zero padding) and W_NN
// (ldn x ldn, minus the identity on its padding, so that
// M M^T - W_NN is the identity there).  Row i of the grid block (y) and
// column j (x) index the largest of the three shapes.
__global__ void thin_split_kernel(const double* __restrict__ G, int64_t ldg,
                                  const double* __restrict__ s,
                                  const int* __restrict__ perm, int np_,
                                  int nn, int64_t ldp, int64_t ldn,
                                  const DevScalars* __restrict__ sc,
                                  double* __restrict__ Wpp,
                                  double* __restrict__ Wpn,
                                  double* __restrict__ Wnn) {
  const int64_t i = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double lam = sc->lambda;
  if (i < ldp && j < ldp) {
    double v = i == j ? 1.0 : 0.0;
    if (i < np_ && j < np_) {
      v = gsym(G, ldg, perm[i], perm[j]);
      if (i == j) v += lam / s[perm[i]];
    }
    Wpp[i * ldp + j] = v;
  }
  if (i < ldp && j < ldn)
    Wpn[i * ldn + j] =
        (i < np_ && j < nn) ? gsym(G, ldg, perm[i], perm[np_ + j]) : 0.0;
  if (i < ldn && j < ldn) {
    double v = i == j ? -1.0 : 0.0;
    if (i < nn && j < nn) {
      v = gsym(G, ldg, perm[np_ + i], perm[np_ + j]);
      if (i == j) v += lam / s[perm[np_ + i]];
    }
    Wnn[i * ldn + j] = v;
  }
}

__global__ void fill_kernel(double* __restrict__ x, int64_t len, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void negate_kernel(double* __restrict__ x, int64_t len) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = -x[i];
}

// q_t = (1 - lambda (W^-1)_tt / s_t) / s_t from the signed factorisation
// (see the head of this file); 0 on the padding rows.
__global__ void thin_q_indef_kernel(const double* __restrict__ X1,
                                    const double* __restrict__ X2,
                                    const double* __restrict__ Y,
                                    const int* __restrict__ pos, int np_,
                                    int nn, int64_t ldp, int64_t ldn,
                                    int64_t T, int64_t Tp,
                                    const double* __restrict__ s,
                                    const DevScalars* __restrict__ sc,
                                    double* __restrict__ q) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Tp) return;
  if (t >= T) {
    q[t] = 0.0;
    return;
  }
  const int i = pos[t];
  double w = 0.0;
  if (i < np_) {
    for (int k = i; k < np_; ++k) {
      const double x = X1[(int64_t)k * ldp + i];
      w += x * x;
    }
    for (int k = 0; k < nn; ++k) {
      const double y = Y[(int64_t)k * ldp + i];
      w -= y * y;
    }
  } else {
    const int j = i - np_;
    for (int k = j; k < nn; ++k) {
      const double x = X2[(int64_t)k * ldn + j];
      w -= x * x;
    }
  }
  q[t] = (1.0 - sc->lambda * w / s[t]) / s[t];
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

int64_t thin_indef_doubles(int64_t T) {
  const int64_t l = round_up(T, 128) + 128;
  return 5 * l * l + 2 * T;
}

hipError_t launch_thin_indef_factor(const double* G, int64_t ldg, int64_t T,
                                    const double* s, int np_, int chol_group,
                                    DevScalars* sc, double* ws,
                                    hipStream_t st) {
  const int nn = (int)T - np_;
  if (np_ < 0 || nn < 1) return hipErrorInvalidValue;
  const int64_t ldp = round_up(np_ > 0 ? np_ : 1, 128);
  const int64_t ldn = round_up(nn, 128);
  const int64_t l = round_up(T, 128) + 128;
  double *Wpp = ws, *X1 = ws + l * l, *Mt = ws + 2 * l * l,
         *Wnn = ws + 3 * l * l, *X2 = ws + 4 * l * l;
  int* perm = (int*)(ws + 5 * l * l);
  int* pos = perm + T;
  hipLaunchKernelGGL(thin_perm_kernel, dim3(1), dim3(64), 0, st, s, T, perm,
                     pos);
  const int64_t big = ldp > ldn ? ldp : ldn;
  hipLaunchKernelGGL(thin_split_kernel,
                     dim3((unsigned)((big + 255) / 256), (unsigned)big),
                     dim3(256), 0, st, G, ldg, s, perm, np_, nn, ldp, ldn, sc,
                     Wpp, Mt, Wnn);
  // the products read the inverses as full matrices
  hipLaunchKernelGGL(fill_kernel, dim3(256), dim3(256), 0, st, X1, ldp * ldp,
                     0.0);
  hipLaunchKernelGGL(fill_kernel, dim3(256), dim3(256), 0, st, X2, ldn * ldn,
                     0.0);
  hipError_t e = hipSuccess;
  if (np_ > 0) {
    e = launch_potrf_trtri(Wpp, X1, ldp, &sc->fail, st, nullptr, chol_group);
    if (e != hipSuccess) return e;
    // M^T = X1 W_PN (ldp x ldn) into Wpp's storage, whose factor is no
    // longer needed
    e = launch_gemm64(X1, ldp, false, Mt, ldn, false, Wpp, ldn, ldp, ldn, ldp,
                      1.0, 0.0, st);
    if (e != hipSuccess) return e;
    // -Sigma = M M^T - W_NN
    e = launch_gemm64(Wpp, ldn, true, Wpp, ldn, false, Wnn, ldn, ldn, ldn, ldp,
                      1.0, -1.0, st);
    if (e != hipSuccess) return e;
  } else {
    // no positive bars: -Sigma = -W_NN (the identity on the padding)
    hipLaunchKernelGGL(negate_kernel, dim3(256), dim3(256), 0, st, Wnn,
                       ldn * ldn);
  }
  return launch_potrf_trtri(Wnn, X2, ldn, &sc->fail, st, nullptr, chol_group);
}

hipError_t launch_thin_indef_q(int64_t T, int64_t Tp, const double* s,
                               int np_, const DevScalars* sc, double* ws,
                               double* q, hipStream_t st) {
  const int nn = (int)T - np_;
  const int64_t ldp = round_up(np_ > 0 ? np_ : 1, 128);
  const int64_t ldn = round_up(nn, 128);
  const int64_t l = round_up(T, 128) + 128;
  double *Mt = ws, *X1 = ws + l * l, *Z = ws + 2 * l * l, *X2 = ws + 4 * l * l;
  int* pos = (int*)(ws + 5 * l * l) + T;
  double* Y = ws + 3 * l * l;  // over -Sigma, whose factor is not needed
  if (np_ > 0) {
    // Z = M X1 (ldn x ldp), Y = X2 Z
    hipError_t e = launch_gemm64(Mt, ldn, true, X1, ldp, false, Z, ldp, ldn,
                                 ldp, ldp, 1.0, 0.0, st);
    if (e != hipSuccess) return e;
    e = launch_gemm64(X2, ldn, false, Z, ldp, false, Y, ldp, ldn, ldp, ldn, 1.0,
                      0.0, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(thin_q_indef_kernel, dim3((unsigned)((Tp + 255) / 256)),
                     dim3(256), 0, st, X1, X2, Y, pos, np_, nn, ldp, ldn, T,
                     Tp, s, sc, q);
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
