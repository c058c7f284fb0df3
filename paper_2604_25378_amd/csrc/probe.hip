// Probe estimate of the exact trace q_t = a_t^T K a_t (the Krylov reduced
// solve of Appendix C with Hutchinson's diagonal estimator): with k random
// sign vectors xi_j in {+-1}^T,
//     q_t ~ k^-1 sum_j xi_tj (A K A^T xi_j)_t,
// where K = P_S (H + lambda)^-1 P_S is applied by k projected PCG solves run
// side by side.  Every product with A is a block product over all k columns
// at once (dense.hip, FP64 MFMA): U = A^T Xi, the Hessian products
// A^T diag(psi''/T) (A P) of each CG step, and A Y at the end.  The column
// updates are the single-vector PCG step of the tangent solve applied to
// each column by its own workgroup, so every column follows the same
// arithmetic as a single solve.
//
// Signs come from SplitMix64 (Steele, Lea and Flood 2014) evaluated at a
// counter: xi_tj is the sign bit of the output for the Weyl state
// seed + gamma (draw 2^42 + t 2^10 + j).
#include "common.h"
#include "kernels.h"
#include "vec.h"

namespace yand {
namespace {

constexpr int PB = 1024;  // threads of the per-column kernels

__device__ __forceinline__ uint64_t splitmix64_out(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Xi (Tp x 64, row-major): signs for t < T and j < k, zero elsewhere.
__global__ void rademacher_kernel(uint64_t seed, uint64_t draw, int64_t T,
                                  int64_t Tp, int k, double* __restrict__ Xi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Tp * kBlockWidth) return;
  const int64_t t = i / kBlockWidth;
  const int j = (int)(i % kBlockWidth);
  double v = 0.0;
  if (t < T && j < k) {
    const uint64_t ctr = (draw << 42) | ((uint64_t)t << 10) | (uint64_t)j;
    const uint64_t r = splitmix64_out(seed + ctr * 0x9E3779B97F4A7C15ull);
    v = (r >> 63) ? -1.0 : 1.0;
  }
  Xi[i] = v;
}

// Sum of K values over the workgroup (fixed order: wave butterfly, then the
// waves in order); every thread gets the sums.
template <int K>
__device__ void col_bsum(double (&v)[K], double* sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = PB / 64;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) sh[k * NW + wv] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += sh[k * NW + w];
    v[k] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ double jacobi(const double* bd, int64_t j,
                                         double lam) {
  const double dj = bd[j] + lam;
  return dj > 0.0 ? dj : 1.0;
}

// Per-column scalars: cs[8 j + 0] r^T z, 1 r^T r, 2 r0^T r0; flags[1 + j]
// done, flags[65 + j] iterations.
// Column j: r = P_S u_j (the probe's right-hand side projected onto the
// tangent space), y = 0, z = P_S diag(B + lambda)^-1 r, p = z.
__global__ void __launch_bounds__(PB)
bpcg_init_kernel(const double* __restrict__ U, const double* __restrict__ bd,
                 const double* __restrict__ E, int p, int64_t n, int64_t ld,
                 int k, double* Y, double* Rr, double* Z, double* P,
                 double* cs, int* flags, const DevScalars* sc,
                 const double* __restrict__ mask) {
  __shared__ double sh[8 * (PB / 64)];
  const int j = blockIdx.x, tid = threadIdx.x;
  const int64_t o = (int64_t)j * ld;
  if (j >= k) {
    for (int64_t i = tid; i < n; i += PB) {
      Y[o + i] = 0.0;
      P[o + i] = 0.0;
    }
    if (tid == 0) {
      flags[1 + j] = 1;
      flags[65 + j] = 0;
    }
    return;
  }
  const double lam = sc->lambda;
  double e[3] = {0.0, 0.0, 0.0};
  for (int64_t i = tid; i < n; i += PB) {
    const double ui = (mask ? mask[i] : 1.0) * U[o + i];
    for (int a = 0; a < p; ++a) e[a] += E[a * n + i] * ui;
  }
  col_bsum(e, sh);
  double dt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = tid; i < n; i += PB) {
    double ri = (mask ? mask[i] : 1.0) * U[o + i];
    for (int a = 0; a < p; ++a) ri -= e[a] * E[a * n + i];
    Rr[o + i] = ri;
    Y[o + i] = 0.0;
    const double zi = (mask ? mask[i] : 1.0) * ri / jacobi(bd, i, lam);
    Z[o + i] = zi;
    for (int a = 0; a < p; ++a) {
      dt[a] += E[a * n + i] * zi;
      dt[3 + a] += E[a * n + i] * ri;
    }
    dt[6] += ri * zi;
    dt[7] += ri * ri;
  }
  col_bsum(dt, sh);
  double rz = dt[6];
  for (int a = 0; a < p; ++a) rz -= dt[3 + a] * dt[a];
  for (int64_t i = tid; i < n; i += PB) {
    double zi = Z[o + i];
    for (int a = 0; a < p; ++a) zi -= dt[a] * E[a * n + i];
    Z[o + i] = zi;
    P[o + i] = zi;
  }
  if (tid == 0) {
    cs[8 * j + 0] = rz;
    cs[8 * j + 1] = dt[7];
    cs[8 * j + 2] = dt[7];
    flags[1 + j] = dt[7] > 0.0 ? 0 : 1;
    flags[65 + j] = 0;
  }
}

// One PCG step of column j (skipped once the column is done): the search
// direction's product HP (from the block pass) plus lambda p, the projected
// curvature, the step, the new residual, its preconditioned projection and
// the next direction; done at |r| <= tol |r0| or a curvature breakdown.
__global__ void __launch_bounds__(PB)
bpcg_update_kernel(const double* __restrict__ HP,
                   const double* __restrict__ bd,
                   const double* __restrict__ E, int p, int64_t n, int64_t ld,
                   double* Y, double* Rr, double* Z, double* P, double* AP,
                   double* cs, int* flags, const DevScalars* sc,
                   const double* __restrict__ mask, double tol) {
  const int j = blockIdx.x, tid = threadIdx.x;
  if (flags[0] || flags[1 + j]) return;
  __shared__ double sh[8 * (PB / 64)];
  const int64_t o = (int64_t)j * ld;
  const double lam = sc->lambda;
  double d1[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = tid; i < n; i += PB) {
    const double a = (mask ? mask[i] : 1.0) * (HP[o + i] + lam * P[o + i]);
    AP[o + i] = a;
    for (int q = 0; q < p; ++q) {
      d1[q] += E[q * n + i] * a;
      d1[3 + q] += E[q * n + i] * P[o + i];
    }
    d1[6] += P[o + i] * a;
  }
  col_bsum(d1, sh);
  double pap = d1[6];
  for (int q = 0; q < p; ++q) pap -= d1[3 + q] * d1[q];
  const double rz = cs[8 * j + 0];
  const double al = pap > 0.0 ? rz / pap : 0.0;
  double d2[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = tid; i < n; i += PB) {
    double a = AP[o + i];
    for (int q = 0; q < p; ++q) a -= d1[q] * E[q * n + i];
    Y[o + i] += al * P[o + i];
    const double ri = Rr[o + i] - al * a;
    Rr[o + i] = ri;
    const double zi = (mask ? mask[i] : 1.0) * ri / jacobi(bd, i, lam);
    Z[o + i] = zi;
    for (int q = 0; q < p; ++q) {
      d2[q] += E[q * n + i] * zi;
      d2[3 + q] += E[q * n + i] * ri;
    }
    d2[6] += ri * zi;
    d2[7] += ri * ri;
  }
  col_bsum(d2, sh);
  double rzn = d2[6];
  const double rr = d2[7];
  for (int q = 0; q < p; ++q) rzn -= d2[3 + q] * d2[q];
  const double beta = rz > 0.0 ? rzn / rz : 0.0;
  for (int64_t i = tid; i < n; i += PB) {
    double zi = Z[o + i];
    for (int q = 0; q < p; ++q) zi -= d2[q] * E[q * n + i];
    Z[o + i] = zi;
    P[o + i] = zi + beta * P[o + i];
  }
  if (tid == 0) {
    cs[8 * j + 0] = rzn;
    cs[8 * j + 1] = rr;
    flags[65 + j] += 1;
    if (sqrt(rr) <= tol * sqrt(cs[8 * j + 2]) || !(pap > 0.0))
      flags[1 + j] = 1;
  }
}

// flags[0] = every column done (the remaining block passes and updates
// return at once); flags[129] = total column iterations.
__global__ void bpcg_alldone_kernel(int* flags) {
  const int j = threadIdx.x;  // 64 threads
  int done = flags[1 + j], it = flags[65 + j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    done &= __shfl_xor(done, off, 64);
    it += __shfl_xor(it, off, 64);
  }
  if (j == 0) {
    flags[0] = done;
    flags[129] = it;
  }
}

// lambda = reg * (trace of the tangent Hessian) / (tangent dimension - 1):
// sum_j mask_j bd_j - sum_t s_t sum_a (A e_a)_t^2 over m - 1 = (free
// coordinates) - p; the same scale as the exact routes.
__global__ void __launch_bounds__(PB)
probe_scale_kernel(const double* __restrict__ bd, int64_t n,
                   const double* __restrict__ s, const double* __restrict__ AE,
                   int64_t T, int64_t Tp, int p, double reg,
                   const double* __restrict__ mask, DevScalars* sc) {
  __shared__ double sh[2 * (PB / 64)];
  double v[2] = {0.0, 0.0};
  for (int64_t j = threadIdx.x; j < n; j += PB) v[0] += (mask ? mask[j] : 1.0) * bd[j];
  for (int64_t t = threadIdx.x; t < T; t += PB) {
    double e = 0.0;
    for (int a = 0; a < p; ++a) e += AE[a * Tp + t] * AE[a * Tp + t];
    v[1] += s[t] * e;
  }
  col_bsum(v, sh);
  if (threadIdx.x == 0) {
    const double neff = mask ? sc->nfree : (double)n;
    double tang = (v[0] - v[1]) / (neff - (double)p);
    if (!(tang > 0.0) || !isfinite(tang)) tang = 1.0;
    sc->tang_scale = tang;
    sc->lambda = reg * tang;
    sc->fail = 0;
  }
}

// q_t = k^-1 sum_j Xi_tj Q_tj (Q = A Y), zero on the padding rows.
__global__ void probe_q_kernel(const double* __restrict__ Xi,
                               const double* __restrict__ Q, int64_t T,
                               int64_t Tp, int k, double* __restrict__ q) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Tp) return;
  double v = 0.0;
  if (t < T) {
    for (int j = 0; j < k; ++j)
      v += Xi[t * kBlockWidth + j] * Q[t * kBlockWidth + j];
    v /= (double)k;
  }
  q[t] = v;
}

}  // namespace

hipError_t launch_rademacher(uint64_t seed, uint64_t draw, int64_t T,
                             int64_t Tp, int k, double* Xi, hipStream_t st) {
  const int64_t total = Tp * kBlockWidth;
  hipLaunchKernelGGL(rademacher_kernel, dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, st, seed, draw, T, Tp, k, Xi);
  return hipGetLastError();
}

hipError_t launch_probe_scale(const double* bd, int64_t n, const double* s,
                              const double* AE, int64_t T, int64_t Tp, int p,
                              double reg, const double* mask, DevScalars* sc,
                              hipStream_t st) {
  hipLaunchKernelGGL(probe_scale_kernel, dim3(1), dim3(PB), 0, st, bd, n, s,
                     AE, T, Tp, p, reg, mask, sc);
  return hipGetLastError();
}

hipError_t launch_bpcg_init(const double* U, const double* bd, const double* E,
                            int p, int64_t n, int64_t ld, int k, double* Y,
                            double* Rr, double* Z, double* P, double* cs,
                            int* flags, const DevScalars* sc,
                            const double* mask, hipStream_t st) {
  hipLaunchKernelGGL(bpcg_init_kernel, dim3(kBlockWidth), dim3(PB), 0, st, U,
                     bd, E, p, n, ld, k, Y, Rr, Z, P, cs, flags, sc, mask);
  hipLaunchKernelGGL(bpcg_alldone_kernel, dim3(1), dim3(64), 0, st, flags);
  return hipGetLastError();
}

hipError_t launch_bpcg_update(const double* HP, const double* bd,
                              const double* E, int p, int64_t n, int64_t ld,
                              double* Y, double* Rr, double* Z, double* P,
                              double* AP, double* cs, int* flags,
                              const DevScalars* sc, const double* mask,
                              double tol, hipStream_t st) {
  hipLaunchKernelGGL(bpcg_update_kernel, dim3(kBlockWidth), dim3(PB), 0, st,
                     HP, bd, E, p, n, ld, Y, Rr, Z, P, AP, cs, flags, sc, mask,
                     tol);
  hipLaunchKernelGGL(bpcg_alldone_kernel, dim3(1), dim3(64), 0, st, flags);
  return hipGetLastError();
}

hipError_t launch_probe_q(const double* Xi, const double* Q, int64_t T,
                          int64_t Tp, int k, double* q, hipStream_t st) {
  hipLaunchKernelGGL(probe_q_kernel, dim3((unsigned)((Tp + 255) / 256)),
                     dim3(256), 0, st, Xi, Q, T, Tp, k, q);
  return hipGetLastError();
}

}  // namespace yand
