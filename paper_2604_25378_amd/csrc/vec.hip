// Small FP64 kernels on n-vectors and scalars: projections onto the tangent
// spaces, the regularisation scale, the projected Hessian, the exact trace
// weights, the direction assembly, the quartic step and the update.  All
// reductions run in one workgroup in a fixed order (bit-reproducible).
#include "common.h"
#include "kernels.h"
#include "vec.h"

namespace yand {

constexpr int VT = 1024;               // threads of the single-group kernels
constexpr int VW = VT / 64;

// Fixed-order block reduction of up to 4 values (all threads get results).
template <int K>
__device__ void block_sum(double (&v)[K], double* sh) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) sh[k * VW + w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int i = 0; i < VW; ++i) s += sh[k * VW + i];
    v[k] = s;
  }
  __syncthreads();
}

// G = g - sum_{a<p0} (e_a^T g) e_a, gn = |G|, nu = G / gn stored as E[p0].
// (Definition "Tangent-gradient residual"; Proposition "Affine-subspace
// reduction": |gbar| = |P_T g|.)
__global__ void __launch_bounds__(VT)
grad_project_kernel(const double* __restrict__ g, double* __restrict__ E,
                    int p0, int64_t n, DevScalars* sc, double eps) {
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  double dots[2] = {0.0, 0.0};
  for (int64_t j = tid; j < n; j += VT)
    for (int a = 0; a < p0; ++a) dots[a] += E[a * n + j] * g[j];
  block_sum(dots, sh);
  double ss[1] = {0.0};
  for (int64_t j = tid; j < n; j += VT) {
    double G = g[j];
    for (int a = 0; a < p0; ++a) G -= dots[a] * E[a * n + j];
    ss[0] += G * G;
  }
  block_sum(ss, sh);
  const double gn = sqrt(ss[0]);
  const double inv = gn > 0.0 ? 1.0 / gn : 0.0;
  for (int64_t j = tid; j < n; j += VT) {
    double G = g[j];
    for (int a = 0; a < p0; ++a) G -= dots[a] * E[a * n + j];
    E[p0 * n + j] = G * inv;
  }
  if (tid == 0) {
    sc->gn = gn;
    if (!isfinite(gn)) sc->nonfinite = 1;
    sc->done = (eps >= 0.0 && (sc->frozen || gn <= eps)) || !isfinite(gn)
                   ? 1
                   : 0;
    sc->fail = 0;
    sc->status = 0;
    sc->alpha = 0.0;
  }
}

// tr = trace(B); GE = E^T W (W = B E); gamma = tr / n;
// lambda = reg * (tr - trace GE) / (n - p)  (mean tangent-Hessian diagonal).
__global__ void __launch_bounds__(VT)
trace_scale_kernel(const double* __restrict__ B, int64_t ld, int64_t n,
                   const double* __restrict__ E, const double* __restrict__ W,
                   int p, double reg, DevScalars* sc) {
  if (sc->done) return;
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  double t[1] = {0.0};
  for (int64_t j = tid; j < n; j += VT) t[0] += B[j * ld + j];
  block_sum(t, sh);
  double ge[9];
  for (int a = 0; a < p; ++a) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t j = tid; j < n; j += VT)
      for (int b = 0; b < p; ++b) v[b] += E[a * n + j] * W[b * n + j];
    block_sum(v, sh);
    for (int b = 0; b < 3; ++b) ge[a * 3 + b] = v[b];
  }
  if (tid == 0) {
    double trg = 0.0;
    for (int a = 0; a < p; ++a) trg += ge[a * 3 + a];
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b)
        sc->GE[a * 3 + b] = 0.5 * (ge[a * 3 + b] + ge[b * 3 + a]);
    sc->tr = t[0];
    double gam = t[0] / (double)n;
    if (!(gam > 0.0) || !isfinite(gam)) gam = 1.0;
    sc->gamma = gam;
    double tang = (t[0] - trg) / (double)(n - p);
    if (!(tang > 0.0) || !isfinite(tang)) tang = gam;
    sc->tang_scale = tang;
    sc->lambda = reg * tang;
  }
}

// Lower triangle of M = P_S B P_S + lambda P_S + gamma (I - P_S), with
// P_S = I - E E^T; identity on the padding.
__global__ void project_kernel(const double* __restrict__ B, double* M,
                               int64_t ld, int64_t n, int64_t np,
                               const double* __restrict__ E,
                               const double* __restrict__ W, int p,
                               const DevScalars* __restrict__ sc) {
  if (sc->done) return;
  const int64_t i = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > i || i >= np) return;
  double v;
  if (i < n && j < n) {
    const double lam = sc->lambda, gam = sc->gamma;
    double ei[3], ej[3], wi[3], wj[3];
    for (int a = 0; a < p; ++a) {
      ei[a] = E[a * n + i];
      ej[a] = E[a * n + j];
      wi[a] = W[a * n + i];
      wj[a] = W[a * n + j];
    }
    v = B[i * ld + j];
    double ee = 0.0;
    for (int a = 0; a < p; ++a) {
      v -= ei[a] * wj[a] + wi[a] * ej[a];
      ee += ei[a] * ej[a];
      for (int b = 0; b < p; ++b) v += ei[a] * sc->GE[a * 3 + b] * ej[b];
    }
    v += (gam - lam) * ee;
    if (i == j) v += lam;
  } else {
    v = i == j ? 1.0 : 0.0;
  }
  M[i * ld + j] = v;
}

// q_t = sum_J rn[J][t] - gamma^-1 sum_a (A e_a)_t^2  (a_t^T K a_t).
__global__ void trace_weight_kernel(const double* __restrict__ rn, int nt,
                                    int64_t Tp, const double* __restrict__ AE,
                                    int p, const DevScalars* __restrict__ sc,
                                    double* __restrict__ q) {
  if (sc->done) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Tp) return;
  double s = 0.0;
  for (int J = 0; J < nt; ++J) s += rn[(int64_t)J * Tp + t];
  double c = 0.0;
  for (int a = 0; a < p; ++a) {
    double v = AE[a * Tp + t];
    c += v * v;
  }
  q[t] = s - c / sc->gamma;
}

// r = B nu - |G|/(m+1) t3, then r <- P_S r.  (Direction of Section 4.4 with
// the factor of Appendix B, bounded-direction proposition.)
__global__ void __launch_bounds__(VT)
rhs_kernel(const double* __restrict__ Bnu, const double* __restrict__ t3,
           const double* __restrict__ E, int p, int64_t n, double mp1,
           const DevScalars* __restrict__ sc, double* __restrict__ r) {
  if (sc->done) return;
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  const double coef = sc->gn / mp1;
  double dots[3] = {0.0, 0.0, 0.0};
  for (int64_t j = tid; j < n; j += VT) {
    double v = Bnu[j] - coef * t3[j];
    for (int a = 0; a < p; ++a) dots[a] += E[a * n + j] * v;
  }
  block_sum(dots, sh);
  for (int64_t j = tid; j < n; j += VT) {
    double v = Bnu[j] - coef * t3[j];
    for (int a = 0; a < p; ++a) v -= dots[a] * E[a * n + j];
    r[j] = v;
  }
}

// d = P_S y - nu; also mu^T d and, on the simplex, alpha_max (Lemma
// "Interior-safe steplength cap").
__global__ void __launch_bounds__(VT)
direction_kernel(const double* __restrict__ y, const double* __restrict__ E,
                 int p, int64_t n, const double* __restrict__ x,
                 const double* __restrict__ mu, double tau, int simplex,
                 double* __restrict__ d, DevScalars* sc) {
  if (sc->done) return;
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  double dots[3] = {0.0, 0.0, 0.0};
  for (int64_t j = tid; j < n; j += VT)
    for (int a = 0; a < p; ++a) dots[a] += E[a * n + j] * y[j];
  block_sum(dots, sh);
  double md[1] = {0.0};
  double am = INFINITY;
  for (int64_t j = tid; j < n; j += VT) {
    double v = y[j];
    for (int a = 0; a < p; ++a) v -= dots[a] * E[a * n + j];
    v -= E[(p - 1) * n + j];
    d[j] = v;
    md[0] += mu[j] * v;
    if (v < 0.0) am = fmin(am, (x[j] - tau) / (-v));
  }
  block_sum(md, sh);
  am = wave_min(am);
  if ((tid & 63) == 0) sh[tid >> 6] = am;
  __syncthreads();
  if (tid == 0) {
    double m = INFINITY;
    for (int i = 0; i < VW; ++i) m = fmin(m, sh[i]);
    sc->mud = md[0];
    sc->amax = simplex ? m : INFINITY;
  }
}

// ---------------------------------------------------------- quartic step --
// Real roots of p(a) = A1 + 2 A2 a + 3 A3 a^2 + 4 A4 a^3 on (lo, hi): the
// stationary points of p split the line into monotone pieces; every sign
// change is bracketed and refined by safeguarded Newton/bisection.
__device__ double dphi(const double* A, double a) {
  return A[1] + a * (2.0 * A[2] + a * (3.0 * A[3] + a * 4.0 * A[4]));
}
__device__ double ddphi(const double* A, double a) {
  return 2.0 * A[2] + a * (6.0 * A[3] + a * 12.0 * A[4]);
}
__device__ double refine_root(const double* A, double lo, double hi) {
  double flo = dphi(A, lo);
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double fx = dphi(A, x);
    if (fx == 0.0) return x;
    if ((fx < 0.0) == (flo < 0.0)) {
      lo = x;
      flo = fx;
    } else {
      hi = x;
    }
    double dfx = ddphi(A, x);
    double xn = dfx != 0.0 ? x - fx / dfx : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (hi - lo <= 4.0 * 2.2204460492503131e-16 * fabs(hi)) return xn;
    if (xn == x) return x;
    x = xn;
  }
  return x;
}

__device__ int quartic_step(const double* A, double amax, double* alpha) {
  const bool finite_cap = isfinite(amax);
  double lead_p = A[4] != 0.0 ? A[4] : A[3] != 0.0 ? A[3]
                 : A[2] != 0.0 ? A[2] : 0.0;   // sign of p at +infinity
  if (!finite_cap) {
    double lead = A[4] != 0.0 ? A[4] : A[3] != 0.0 ? A[3]
                : A[2] != 0.0 ? A[2] : A[1];
    if (!(lead > 0.0)) {
      *alpha = 0.0;
      return -6;
    }
  }
  // stationary points of p in (0, amax)
  double bp[4];
  int nb = 0;
  bp[nb++] = 0.0;
  {
    const double a2 = 12.0 * A[4], a1 = 6.0 * A[3], a0 = 2.0 * A[2];
    double r[2];
    int nr = 0;
    if (a2 != 0.0) {
      double disc = a1 * a1 - 4.0 * a2 * a0;
      if (disc >= 0.0) {
        double q = -0.5 * (a1 + copysign(sqrt(disc), a1));
        if (q != 0.0) {
          r[nr++] = q / a2;
          r[nr++] = a0 / q;
        } else {
          r[nr++] = 0.0;
        }
      }
    } else if (a1 != 0.0) {
      r[nr++] = -a0 / a1;
    }
    if (nr == 2 && r[0] > r[1]) {
      double t = r[0];
      r[0] = r[1];
      r[1] = t;
    }
    for (int i = 0; i < nr; ++i)
      if (r[i] > 0.0 && r[i] < amax) bp[nb++] = r[i];
  }
  double cand[6];
  int nc = 0;
  cand[nc++] = 0.0;
  if (finite_cap) cand[nc++] = amax;
  for (int i = 0; i < nb; ++i) {
    double lo = bp[i];
    double hi;
    double flo = dphi(A, lo), fhi;
    if (i + 1 < nb) {
      hi = bp[i + 1];
      fhi = dphi(A, hi);
    } else if (finite_cap) {
      hi = amax;
      fhi = dphi(A, hi);
    } else {
      if (lead_p == 0.0) continue;            // p constant beyond lo
      if ((flo < 0.0) == (lead_p < 0.0) || flo == 0.0) {
        if (flo != 0.0) continue;             // no sign change to +inf
      }
      hi = fmax(2.0 * lo, 1.0);
      fhi = dphi(A, hi);
      for (int k = 0; k < 2100 && (fhi < 0.0) == (flo < 0.0) && fhi != 0.0;
           ++k) {
        lo = hi;
        flo = fhi;
        hi *= 2.0;
        fhi = dphi(A, hi);
      }
    }
    if (flo == 0.0) {
      if (lo > 0.0) cand[nc++] = lo;
      continue;
    }
    if (fhi == 0.0) {
      if (hi > 0.0 && hi < amax) cand[nc++] = hi;
      continue;
    }
    if ((flo < 0.0) != (fhi < 0.0)) {
      double rt = refine_root(A, lo, hi);
      if (rt > 0.0 && rt < amax) cand[nc++] = rt;
    }
  }
  // argmin of phi(a) - A0 with the tie rule toward the smallest step
  double best = 0.0, vbest = 0.0;
  double vals[6], scl[6];
  for (int i = 0; i < nc; ++i) {
    double a = cand[i];
    vals[i] = a * (A[1] + a * (A[2] + a * (A[3] + a * A[4])));
    scl[i] = a * (fabs(A[1]) + a * (fabs(A[2]) + a * (fabs(A[3]) + a * fabs(A[4]))));
    if (i == 0 || vals[i] < vbest) vbest = vals[i];
  }
  best = INFINITY;
  for (int i = 0; i < nc; ++i)
    if (vals[i] <= vbest + 1e-15 * scl[i] && cand[i] < best) best = cand[i];
  *alpha = best;
  return 0;
}

// Assemble A0..A4 (Proposition "Quartic exact line search from sample power
// sums") from the reduced sums and pick the step.
__global__ void coef_step_kernel(const double* __restrict__ sums, double invT,
                                 Coef c, int select, DevScalars* sc) {
  if (threadIdx.x != 0) return;
  if (select && (sc->done || sc->fail)) {
    sc->alpha = 0.0;
    return;
  }
  const double s11 = sums[0] * invT, s21 = sums[1] * invT,
               s31 = sums[2] * invT, s02 = sums[3] * invT,
               s12 = sums[4] * invT, s22 = sums[5] * invT,
               s03 = sums[6] * invT, s13 = sums[7] * invT,
               s04 = sums[8] * invT;
  double* A = sc->coef;
  A[0] = sc->f;
  A[1] = -c.c1 * sc->mud + 2.0 * c.c2 * s11 - 3.0 * c.c3 * s21 +
         4.0 * c.c4 * s31;
  A[2] = c.c2 * s02 - 3.0 * c.c3 * s12 + 6.0 * c.c4 * s22;
  A[3] = -c.c3 * s03 + 4.0 * c.c4 * s13;
  A[4] = c.c4 * s04;
  if (select) sc->status = quartic_step(A, sc->amax, &sc->alpha);
}

__global__ void select_step_kernel(DevScalars* sc) {
  if (threadIdx.x == 0) sc->status = quartic_step(sc->coef, sc->amax, &sc->alpha);
}

// f and the moments from the oracle-pass sums and mu^T x.
__global__ void objective_kernel(const double* __restrict__ sums, double invT,
                                 Coef c, DevScalars* sc) {
  if (threadIdx.x != 0) return;
  const double m2 = sums[0] * invT, m3 = sums[1] * invT, m4 = sums[2] * invT;
  const double m1 = sc->mux;
  sc->mom[0] = m1;
  sc->mom[1] = m2;
  sc->mom[2] = m3;
  sc->mom[3] = m4;
  sc->f = -c.c1 * m1 + c.c2 * m2 - c.c3 * m3 + c.c4 * m4;
  if (!isfinite(sc->f)) sc->nonfinite = 1;
}

// out = sum_j u_j v_j (single group, fixed order).
__global__ void __launch_bounds__(VT)
dot_kernel(const double* __restrict__ u, const double* __restrict__ v,
           int64_t n, double* out) {
  __shared__ double sh[4 * VW];
  double s[1] = {0.0};
  for (int64_t j = threadIdx.x; j < n; j += VT) s[0] += u[j] * v[j];
  block_sum(s, sh);
  if (threadIdx.x == 0) *out = s[0];
}

// x += alpha d (alpha from the device scalars).
__global__ void axpy_kernel(double* __restrict__ x,
                            const double* __restrict__ d, int64_t n,
                            const DevScalars* __restrict__ sc) {
  if (sc->done || sc->fail || sc->status != 0) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) x[j] += sc->alpha * d[j];
}

__global__ void copy_kernel(double* __restrict__ dst,
                            const double* __restrict__ src, int64_t count,
                            const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void fill_kernel(double* __restrict__ dst, int64_t count, double v,
                            const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

// ------------------------------------------------------------ launchers --

hipError_t launch_grad_project(const double* g, double* E, int p0, int64_t n,
                               DevScalars* sc, hipStream_t st, double eps) {
  hipLaunchKernelGGL(grad_project_kernel, dim3(1), dim3(VT), 0, st, g, E, p0,
                     n, sc, eps);
  return hipGetLastError();
}
hipError_t launch_trace_scale(const double* B, int64_t ld, int64_t n,
                              const double* E, const double* W, int p,
                              double reg, DevScalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(trace_scale_kernel, dim3(1), dim3(VT), 0, st, B, ld, n,
                     E, W, p, reg, sc);
  return hipGetLastError();
}
hipError_t launch_project(const double* B, double* M, int64_t ld, int64_t n,
                          int64_t np, const double* E, const double* W, int p,
                          const DevScalars* sc, hipStream_t st) {
  dim3 g((unsigned)((np + 255) / 256), (unsigned)np);
  hipLaunchKernelGGL(project_kernel, g, dim3(256), 0, st, B, M, ld, n, np, E,
                     W, p, sc);
  return hipGetLastError();
}
hipError_t launch_trace_weight(const double* rn, int nt, int64_t Tp,
                               const double* AE, int p, const DevScalars* sc,
                               double* q, hipStream_t st) {
  hipLaunchKernelGGL(trace_weight_kernel, dim3((unsigned)((Tp + 255) / 256)),
                     dim3(256), 0, st, rn, nt, Tp, AE, p, sc, q);
  return hipGetLastError();
}
hipError_t launch_rhs(const double* Bnu, const double* t3, const double* E,
                      int p, int64_t n, double mp1, const DevScalars* sc,
                      double* r, hipStream_t st) {
  hipLaunchKernelGGL(rhs_kernel, dim3(1), dim3(VT), 0, st, Bnu, t3, E, p, n,
                     mp1, sc, r);
  return hipGetLastError();
}
hipError_t launch_direction(const double* y, const double* E, int p,
                            int64_t n, const double* x, const double* mu,
                            double tau, int simplex, double* d,
                            DevScalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(direction_kernel, dim3(1), dim3(VT), 0, st, y, E, p, n,
                     x, mu, tau, simplex, d, sc);
  return hipGetLastError();
}
hipError_t launch_coef_step(const double* sums, double invT, Coef c,
                            int select, DevScalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(coef_step_kernel, dim3(1), dim3(64), 0, st, sums, invT, c,
                     select, sc);
  return hipGetLastError();
}
hipError_t launch_select_step(DevScalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(select_step_kernel, dim3(1), dim3(64), 0, st, sc);
  return hipGetLastError();
}
hipError_t launch_objective(const double* sums, double invT, Coef c,
                            DevScalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(64), 0, st, sums, invT, c,
                     sc);
  return hipGetLastError();
}
hipError_t launch_dot(const double* u, const double* v, int64_t n, double* out,
                      hipStream_t st) {
  hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(VT), 0, st, u, v, n, out);
  return hipGetLastError();
}
hipError_t launch_axpy(double* x, const double* d, int64_t n,
                       const DevScalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + 255) / 256)),
                     dim3(256), 0, st, x, d, n, sc);
  return hipGetLastError();
}

static unsigned grid_for(int64_t count) {
  int64_t b = (count + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}
hipError_t launch_copy(double* dst, const double* src, int64_t count,
                       hipStream_t st, const int* skip) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(count)), dim3(256), 0, st, dst,
                     src, count, skip);
  return hipGetLastError();
}
hipError_t launch_fill(double* dst, int64_t count, double v, hipStream_t st,
                       const int* skip) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(count)), dim3(256), 0, st, dst,
                     count, v, skip);
  return hipGetLastError();
}

}  // namespace yand
