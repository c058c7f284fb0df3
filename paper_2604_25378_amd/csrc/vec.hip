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

// Mask value of coordinate j (1 when there is no mask).
__device__ __forceinline__ double mk(const double* m, int64_t j) {
  return m ? m[j] : 1.0;
}

// G = g - sum_{a<p0} (e_a^T g) e_a, gn = |G|, nu = G / gn stored as E[p0].
// (Definition "Tangent-gradient residual"; Proposition "Affine-subspace
// reduction": |gbar| = |P_T g|.)
__global__ void __launch_bounds__(VT)
grad_project_kernel(const double* __restrict__ g, double* __restrict__ E,
                    int p0, int64_t n, DevScalars* sc, double eps,
                    const double* __restrict__ mask) {
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  double dots[2] = {0.0, 0.0};
  for (int64_t j = tid; j < n; j += VT)
    for (int a = 0; a < p0; ++a) dots[a] += E[a * n + j] * g[j];
  block_sum(dots, sh);
  double ss[1] = {0.0};
  for (int64_t j = tid; j < n; j += VT) {
    double G = mk(mask, j) * g[j];
    for (int a = 0; a < p0; ++a) G -= dots[a] * E[a * n + j];
    ss[0] += G * G;
  }
  block_sum(ss, sh);
  const double gn = sqrt(ss[0]);
  const double inv = gn > 0.0 ? 1.0 / gn : 0.0;
  for (int64_t j = tid; j < n; j += VT) {
    double G = mk(mask, j) * g[j];
    for (int a = 0; a < p0; ++a) G -= dots[a] * E[a * n + j];
    E[p0 * n + j] = G * inv;
  }
  if (tid == 0) {
    sc->gn = gn;
    if (!isfinite(gn)) sc->nonfinite = 1;
    // a face the face solver holds is only a stop once the holds are gone:
    // at a held face's stationary point they are dropped instead
    const bool flat = eps >= 0.0 && gn <= eps;
    sc->done = (eps >= 0.0 && (sc->frozen || (flat && sc->nhold == 0))) ||
                       !isfinite(gn)
                   ? 1
                   : 0;
    if (flat && sc->nhold > 0 && !sc->frozen) sc->release = 1;
    sc->fail = 0;
    sc->status = 0;
    sc->alpha = 0.0;
    sc->projected = 0;
  }
}

// tr = trace(B); GE = E^T W (W = B E); gamma = tr / n;
// lambda = reg * (tr - trace GE) / (n - p)  (mean tangent-Hessian diagonal).
__global__ void __launch_bounds__(VT)
trace_scale_kernel(const double* __restrict__ B, int64_t ld, int64_t n,
                   const double* __restrict__ E, const double* __restrict__ W,
                   int p, double reg, DevScalars* sc,
                   const double* __restrict__ mask) {
  if (sc->done) return;
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  // traces over the free coordinates of the face
  const double neff = mask ? sc->nfree : (double)n;
  double t[1] = {0.0};
  for (int64_t j = tid; j < n; j += VT) t[0] += mk(mask, j) * B[j * ld + j];
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
    double gam = t[0] / neff;
    if (!(gam > 0.0) || !isfinite(gam)) gam = 1.0;
    sc->gamma = gam;
    double tang = (t[0] - trg) / (neff - (double)p);
    if (!(tang > 0.0) || !isfinite(tang)) tang = gam;
    sc->tang_scale = tang;
    sc->lambda = reg * tang;
  }
}

// Lower triangle of M = P_S B P_S + lambda P_S + gamma (I - P_S), with
// P_S = diag(mask) - E E^T; identity on the padding.  A bound coordinate i
// of a face gets M_ii = 1e30 gamma instead of gamma: any positive scale of
// that block leaves K = P_S M^-1 P_S unchanged, and this one makes its share
// a_ti^2 / M_ii of |L^-1 a_t|^2 vanish below FP64 resolution, so the exact
// trace needs no correction for the bound coordinates.
// One workgroup per row i of the lower triangle; the row's own values are
// read once and each thread walks the row's columns j <= i, PU columns at a
// time with all their reads issued before the first write (a wait for a
// load also waits for the stores before it).  P = p, the frame's width.
template <int P>
__global__ void __launch_bounds__(256)
project_kernel(const double* __restrict__ B, double* M, int64_t ld, int64_t n,
               int64_t np, const double* __restrict__ E,
               const double* __restrict__ W,
               const DevScalars* __restrict__ sc,
               const double* __restrict__ mask) {
  if (sc->done) return;
  const int64_t i = blockIdx.x;
  double* Mi = M + i * ld;
  if (i >= n) {
    for (int64_t j = threadIdx.x; j <= i; j += blockDim.x)
      Mi[j] = i == j ? 1.0 : 0.0;
    return;
  }
  const double lam = sc->lambda, gam = sc->gamma;
  double ei[P], wi[P], ge[P][P];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    ei[a] = E[a * n + i];
    wi[a] = W[a * n + i];
#pragma unroll
    for (int b = 0; b < P; ++b) ge[a][b] = sc->GE[a * 3 + b];
  }
  const double mi = mk(mask, i);
  const double* Bi = B + i * ld;
  constexpr int PU = 4;
  const int64_t stride = blockDim.x;
  for (int64_t j0 = threadIdx.x; j0 <= i; j0 += PU * stride) {
    double ej[PU][P], wj[PU][P], mj[PU], bj[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      // columns past the row read column i (in bounds) and are not written
      const int64_t j = j0 + u * stride <= i ? j0 + u * stride : i;
#pragma unroll
      for (int a = 0; a < P; ++a) {
        ej[u][a] = E[a * n + j];
        wj[u][a] = W[a * n + j];
      }
      mj[u] = mk(mask, j);
      bj[u] = Bi[j];
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int64_t j = j0 + u * stride;
      if (j > i) break;
      double v = mi * mj[u] * bj[u];
      double ee = 0.0;
#pragma unroll
      for (int a = 0; a < P; ++a) {
        v -= ei[a] * (mj[u] * wj[u][a]) + (mi * wi[a]) * ej[u][a];
        ee += ei[a] * ej[u][a];
#pragma unroll
        for (int b = 0; b < P; ++b) v += ei[a] * ge[a][b] * ej[u][b];
      }
      v += (gam - lam) * ee;
      if (i == j) v += mi != 0.0 ? lam : 1e30 * gam;
      Mi[j] = v;
    }
  }
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
           const DevScalars* __restrict__ sc, double* __restrict__ r,
           const double* __restrict__ mask) {
  if (sc->done) return;
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  if (mp1 < 0.0) mp1 = sc->nfree - (double)p + 2.0;
  const double coef = sc->gn / mp1;
  double dots[3] = {0.0, 0.0, 0.0};
  for (int64_t j = tid; j < n; j += VT) {
    double v = mk(mask, j) * (Bnu[j] - coef * t3[j]);
    for (int a = 0; a < p; ++a) dots[a] += E[a * n + j] * v;
  }
  block_sum(dots, sh);
  for (int64_t j = tid; j < n; j += VT) {
    double v = mk(mask, j) * (Bnu[j] - coef * t3[j]);
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
                 double* __restrict__ d, DevScalars* sc,
                 const double* __restrict__ mask) {
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
    double v = mk(mask, j) * y[j];
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

// ------------------------------------------------ simplex boundary block --
// Largest value over the workgroup (all threads get it).
__device__ double block_max(double v, double* sh) {
  const int tid = threadIdx.x;
  v = -wave_min(-v);
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  double m = -INFINITY;
  for (int i = 0; i < VW; ++i) m = fmax(m, sh[i]);
  __syncthreads();
  return m;
}

// out = Pi_{Delta(tau)}(y), y_j = fy(j), by one workgroup: with u = y - tau
// and s = 1 - n tau, out_j = max(u_j - theta, 0) + tau where theta solves
// h(theta) = sum_j max(u_j - theta, 0) = s.
// Michelot's method first (Michelot 1986): theta from the current support,
// theta = (sum_S u_j - s) / |S|, then S = {u_j > theta}, until S stops
// shrinking; theta only grows (kept nondecreasing under rounding), so the
// support is monotone and the loop ends, usually within a few passes.
// Should it not settle within kMichelot passes, bisection on
// [max u - s, max u] (where h >= s and h = 0) runs until the interval stops
// shrinking and the support is {u_j > lo}.  Either way theta is formed from
// the final support.  Every loop bound and branch depends only on
// block-reduced values, so all threads take the same path.
constexpr int kMichelot = 64;
template <class FY>
__device__ void simplex_project(FY fy, int64_t n, double tau, double* out,
                                double* sh) {
  const int tid = threadIdx.x;
  const double s = 1.0 - (double)n * tau;
  double v[2] = {0.0, 0.0};
  for (int64_t j = tid; j < n; j += VT) v[0] += fy(j) - tau;
  block_sum(v, sh);
  double theta = (v[0] - s) / (double)n, cnt = (double)n;
  bool settled = false;
  for (int it = 0; it < kMichelot; ++it) {
    double w[2] = {0.0, 0.0};
    for (int64_t j = tid; j < n; j += VT) {
      const double u = fy(j) - tau;
      if (u > theta) {
        w[0] += u;
        w[1] += 1.0;
      }
    }
    block_sum(w, sh);
    if (!(w[1] > 0.0)) break;
    const double th = (w[0] - s) / w[1];
    if (w[1] == cnt) {
      theta = th;
      settled = true;
      break;
    }
    cnt = w[1];
    theta = fmax(theta, th);
  }
  if (!settled) {
    double mx = -INFINITY;
    for (int64_t j = tid; j < n; j += VT) mx = fmax(mx, fy(j) - tau);
    mx = block_max(mx, sh);
    double lo = mx - s, hi = mx;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      double h[1] = {0.0};
      for (int64_t j = tid; j < n; j += VT) h[0] += fmax(fy(j) - tau - mid, 0.0);
      block_sum(h, sh);
      if (h[0] >= s)
        lo = mid;
      else
        hi = mid;
    }
    double w[2] = {0.0, 0.0};
    for (int64_t j = tid; j < n; j += VT) {
      const double u = fy(j) - tau;
      if (u > lo) {
        w[0] += u;
        w[1] += 1.0;
      }
    }
    block_sum(w, sh);
    theta = (w[0] - s) / w[1];
  }
  for (int64_t j = tid; j < n; j += VT)
    out[j] = fmax(fy(j) - tau - theta, 0.0) + tau;
  __syncthreads();
}

__global__ void __launch_bounds__(VT)
project_simplex_kernel(const double* __restrict__ y, int64_t n, double tau,
                       double* __restrict__ out) {
  __shared__ double sh[4 * VW];
  simplex_project([&](int64_t j) { return y[j]; }, n, tau, out, sh);
}

// Face of Delta(tau) at x (boundary block of Algorithm 1: continuation on
// the exposed face).  Coordinates above the slice bound, x_j > tau (1 +
// 1e-6), are free; a bound coordinate is released when its multiplier
// g_j - nu is negative, nu the mean of g over the coordinates above the
// bound, unless the face solver holds it (hold[j] != 0).  When the previous
// stationarity test asked for it (sc->release), the holds are dropped
// first.  Writes the mask, E[0] = mask / sqrt(nfree) and sc->nfree.
__global__ void __launch_bounds__(VT)
face_kernel(const double* __restrict__ x, const double* __restrict__ g,
            int64_t n, double tau, double* __restrict__ E,
            double* __restrict__ mask, double* __restrict__ hold,
            DevScalars* sc) {
  if (sc->frozen) return;
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  const bool rel = sc->release != 0;
  const double thr = tau * (1.0 + 1e-6);
  double v[2] = {0.0, 0.0};
  for (int64_t j = tid; j < n; j += VT)
    if (x[j] > thr) {
      v[0] += g[j];
      v[1] += 1.0;
    }
  block_sum(v, sh);
  const double nu = v[0] / v[1];
  double cnt[1] = {0.0};
  for (int64_t j = tid; j < n; j += VT) {
    if (rel) hold[j] = 0.0;
    const bool held = !rel && hold[j] != 0.0;
    const double m = (x[j] > thr || (g[j] < nu && !held)) ? 1.0 : 0.0;
    mask[j] = m;
    cnt[0] += m;
  }
  block_sum(cnt, sh);
  const double inv = 1.0 / sqrt(cnt[0]);
  for (int64_t j = tid; j < n; j += VT) E[j] = mask[j] * inv;
  if (tid == 0) {
    sc->nfree = cnt[0];
    if (rel) {
      sc->nhold = 0;
      sc->release = 0;
    }
    sc->nhold0 = sc->nhold;
  }
}

__global__ void __launch_bounds__(VT)
reset_hold_kernel(double* __restrict__ hold, int64_t n, DevScalars* sc) {
  for (int64_t j = threadIdx.x; j < n; j += VT) hold[j] = 0.0;
  if (threadIdx.x == 0) {
    sc->nhold = 0;
    sc->nhold0 = 0;
    sc->release = 0;
  }
}

// Projected-simplex KKT residual |x - Pi_Delta(tau)(x - g)|_2.
__global__ void __launch_bounds__(VT)
kkt_kernel(const double* __restrict__ x, const double* __restrict__ g,
           int64_t n, double tau, double eps, double* __restrict__ tmp,
           DevScalars* sc) {
  if (sc->frozen) return;
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  simplex_project([&](int64_t j) { return x[j] - g[j]; }, n, tau, tmp, sh);
  double r[1] = {0.0};
  for (int64_t j = tid; j < n; j += VT) {
    const double e = x[j] - tmp[j];
    r[0] += e * e;
  }
  block_sum(r, sh);
  if (tid == 0) {
    const double k = sqrt(r[0]);
    sc->kkt = k;
    if (eps >= 0.0 && k <= eps) sc->done = 1;
  }
}

// Face solver: hold at the bound the free coordinates that d drives down
// and that are at the bound already (released ones) or stop the raw step
// (reach the bound at alpha_max = sc->amax); sc->nhold counts new holds.
__device__ void hold_blocking(const double* __restrict__ x,
                              const double* __restrict__ d,
                              const double* __restrict__ mask,
                              double* __restrict__ hold, int64_t n,
                              double tau, DevScalars* sc, double* sh) {
  const int tid = threadIdx.x;
  const double thr = tau * (1.0 + 1e-6);
  const double acap = sc->amax * (1.0 + 1e-12);
  double cnt[1] = {0.0};
  for (int64_t j = tid; j < n; j += VT) {
    const double dj = d[j];
    if (mask[j] != 0.0 && dj < 0.0 && hold[j] == 0.0 &&
        (x[j] <= thr || (x[j] - tau) / (-dj) <= acap)) {
      hold[j] = 1.0;
      cnt[0] += 1.0;
    }
  }
  block_sum(cnt, sh);
  if (tid == 0) sc->nhold += (int)cnt[0];
}

// Boundary block, first part: the raw step is capped below the nominal step
// eta, so the trial x + eta d is projected onto Delta(tau); the corrected
// segment dbar = xbar - x (kept in tmp) is the candidate when it is a
// descent direction (g^T dbar < 0) and not numerically zero (max |dbar| >
// 1e-15 max |x|).  Otherwise the face solver takes over at once.
__global__ void __launch_bounds__(VT)
boundary_kernel(const double* __restrict__ x, const double* __restrict__ g,
                const double* __restrict__ mu, int64_t n, double tau,
                double eta, double* __restrict__ d, double* __restrict__ tmp,
                const double* __restrict__ mask, double* __restrict__ hold,
                DevScalars* sc) {
  // nothing to do at a stop or after a failed factorisation (the host redoes
  // the direction): a direction from a failed factor must not set holds
  const bool run = !sc->done && !sc->fail && sc->amax < eta;
  __shared__ double sh[4 * VW];
  const int tid = threadIdx.x;
  __syncthreads();
  if (tid == 0) {
    sc->lsskip = sc->done;
    sc->segskip = 1;
  }
  if (!run) return;
  simplex_project([&](int64_t j) { return x[j] + eta * d[j]; }, n, tau, tmp,
                  sh);
  double dm = 0.0, xm = 0.0;
  double v[2] = {0.0, 0.0};
  for (int64_t j = tid; j < n; j += VT) {
    const double db = tmp[j] - x[j];
    tmp[j] = db;
    dm = fmax(dm, fabs(db));
    xm = fmax(xm, fabs(x[j]));
    v[0] += g[j] * db;
    v[1] += mu[j] * db;
  }
  dm = block_max(dm, sh);
  xm = block_max(xm, sh);
  block_sum(v, sh);
  if (!(dm > 1e-15 * xm && v[0] < 0.0)) {
    hold_blocking(x, d, mask, hold, n, tau, sc, sh);
    return;
  }
  if (tid == 0) {
    sc->segskip = 0;
    sc->mudseg = v[1];
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
  if (A[1] == 0.0 && A[2] == 0.0 && A[3] == 0.0 && A[4] == 0.0) {
    *alpha = 0.0;  // a constant model (zero direction): stay put
    return 0;
  }
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

// Armijo backtracking on the quartic line model: from min(1, amax), halve
// until phi(a) - phi(0) <= 1e-4 a phi'(0) (phi'(0) = A1), at most 60 times
// (then 0).  The model is exact, so no trial needs a pass over A.
__device__ double armijo_step(const double* A, double amax) {
  double a = fmin(1.0, amax);
  for (int k = 0; k < 60; ++k) {
    const double dec = a * (A[1] + a * (A[2] + a * (A[3] + a * A[4])));
    if (dec <= 1e-4 * a * A[1]) return a;
    a *= 0.5;
  }
  return 0.0;
}

// Assemble A0..A4 (Proposition "Quartic exact line search from sample power
// sums") from the reduced sums and pick the step: select 1 the exact rule,
// select 2 Armijo backtracking.
// A0..A4 of the quartic line model from the line-pass sums (Proposition
// "Quartic exact line search from sample power sums"), f and mu^T d given.
__device__ void line_coefs(const double* __restrict__ sums, double invT,
                           Coef c, double f, double mud, double* A) {
  const double s11 = sums[0] * invT, s21 = sums[1] * invT,
               s31 = sums[2] * invT, s02 = sums[3] * invT,
               s12 = sums[4] * invT, s22 = sums[5] * invT,
               s03 = sums[6] * invT, s13 = sums[7] * invT,
               s04 = sums[8] * invT;
  A[0] = f;
  A[1] = -c.c1 * mud + 2.0 * c.c2 * s11 - 3.0 * c.c3 * s21 + 4.0 * c.c4 * s31;
  A[2] = c.c2 * s02 - 3.0 * c.c3 * s12 + 6.0 * c.c4 * s22;
  A[3] = -c.c3 * s03 + 4.0 * c.c4 * s13;
  A[4] = c.c4 * s04;
}

__global__ void coef_step_kernel(const double* __restrict__ sums, double invT,
                                 Coef c, int select, DevScalars* sc,
                                 const int* skip) {
  if (threadIdx.x != 0) return;
  if (select && (sc->done || sc->fail)) {
    sc->alpha = 0.0;
    return;
  }
  if (skip && *skip) return;
  double* A = sc->coef;
  line_coefs(sums, invT, c, sc->f, sc->mud, A);
  if (select == 2) {
    sc->alpha = armijo_step(A, sc->amax);
    sc->status = 0;
  } else if (select) {
    sc->status = quartic_step(A, sc->amax, &sc->alpha);
  }
}

// A projected segment whose line search moves less than this fraction of it
// is no usable descent step (reading of the reduced-simplex wrapper).
constexpr double kSegmentUsable = 0.1;

__global__ void __launch_bounds__(VT)
segment_decide_kernel(const double* __restrict__ sums, double invT, Coef c,
                      int select, const double* __restrict__ x, int64_t n,
                      double tau, double* __restrict__ d,
                      const double* __restrict__ tmp,
                      const double* __restrict__ mask,
                      double* __restrict__ hold, DevScalars* sc) {
  if (sc->segskip) return;
  __shared__ double sh[4 * VW];
  __shared__ double As[5];
  __shared__ double a_s[1];
  __shared__ int st_s[1];
  const int tid = threadIdx.x;
  if (tid == 0) {
    line_coefs(sums, invT, c, sc->f, sc->mudseg, As);
    double a = 0.0;
    int st = 0;
    if (select == 2)
      a = armijo_step(As, 1.0);
    else
      st = quartic_step(As, 1.0, &a);
    a_s[0] = a;
    st_s[0] = st;
  }
  __syncthreads();
  if (a_s[0] >= kSegmentUsable) {
    for (int64_t j = tid; j < n; j += VT) d[j] = tmp[j];
    if (tid == 0) {
      for (int i = 0; i < 5; ++i) sc->coef[i] = As[i];
      sc->alpha = a_s[0];
      sc->status = st_s[0];
      sc->amax = 1.0;
      sc->mud = sc->mudseg;
      sc->projected = 1;
      sc->lsskip = 1;
    }
    return;
  }
  hold_blocking(x, d, mask, hold, n, tau, sc, sh);
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
                               DevScalars* sc, hipStream_t st, double eps,
                               const double* mask) {
  hipLaunchKernelGGL(grad_project_kernel, dim3(1), dim3(VT), 0, st, g, E, p0,
                     n, sc, eps, mask);
  return hipGetLastError();
}
hipError_t launch_trace_scale(const double* B, int64_t ld, int64_t n,
                              const double* E, const double* W, int p,
                              double reg, DevScalars* sc, hipStream_t st,
                              const double* mask) {
  hipLaunchKernelGGL(trace_scale_kernel, dim3(1), dim3(VT), 0, st, B, ld, n,
                     E, W, p, reg, sc, mask);
  return hipGetLastError();
}
hipError_t launch_project(const double* B, double* M, int64_t ld, int64_t n,
                          int64_t np, const double* E, const double* W, int p,
                          const DevScalars* sc, hipStream_t st,
                          const double* mask) {
  const dim3 g((unsigned)np), b(256);
  switch (p) {
    case 1:
      hipLaunchKernelGGL(project_kernel<1>, g, b, 0, st, B, M, ld, n, np, E, W,
                         sc, mask);
      break;
    case 2:
      hipLaunchKernelGGL(project_kernel<2>, g, b, 0, st, B, M, ld, n, np, E, W,
                         sc, mask);
      break;
    case 3:
      hipLaunchKernelGGL(project_kernel<3>, g, b, 0, st, B, M, ld, n, np, E, W,
                         sc, mask);
      break;
    default:
      return hipErrorInvalidValue;
  }
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
                      double* r, hipStream_t st, const double* mask) {
  hipLaunchKernelGGL(rhs_kernel, dim3(1), dim3(VT), 0, st, Bnu, t3, E, p, n,
                     mp1, sc, r, mask);
  return hipGetLastError();
}
hipError_t launch_direction(const double* y, const double* E, int p,
                            int64_t n, const double* x, const double* mu,
                            double tau, int simplex, double* d,
                            DevScalars* sc, hipStream_t st,
                            const double* mask) {
  hipLaunchKernelGGL(direction_kernel, dim3(1), dim3(VT), 0, st, y, E, p, n,
                     x, mu, tau, simplex, d, sc, mask);
  return hipGetLastError();
}
hipError_t launch_face(const double* x, const double* g, int64_t n, double tau,
                       double* E, double* mask, double* hold, DevScalars* sc,
                       hipStream_t st) {
  hipLaunchKernelGGL(face_kernel, dim3(1), dim3(VT), 0, st, x, g, n, tau, E,
                     mask, hold, sc);
  return hipGetLastError();
}
hipError_t launch_reset_hold(double* hold, int64_t n, DevScalars* sc,
                             hipStream_t st) {
  hipLaunchKernelGGL(reset_hold_kernel, dim3(1), dim3(VT), 0, st, hold, n,
                     sc);
  return hipGetLastError();
}
hipError_t launch_kkt(const double* x, const double* g, int64_t n, double tau,
                      double eps, double* tmp, DevScalars* sc,
                      hipStream_t st) {
  hipLaunchKernelGGL(kkt_kernel, dim3(1), dim3(VT), 0, st, x, g, n, tau, eps,
                     tmp, sc);
  return hipGetLastError();
}
hipError_t launch_boundary(const double* x, const double* g, const double* mu,
                           int64_t n, double tau, double eta, double* d,
                           double* tmp, const double* mask, double* hold,
                           DevScalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(boundary_kernel, dim3(1), dim3(VT), 0, st, x, g, mu, n,
                     tau, eta, d, tmp, mask, hold, sc);
  return hipGetLastError();
}
hipError_t launch_project_simplex(const double* y, int64_t n, double tau,
                                  double* out, hipStream_t st) {
  hipLaunchKernelGGL(project_simplex_kernel, dim3(1), dim3(VT), 0, st, y, n,
                     tau, out);
  return hipGetLastError();
}
hipError_t launch_coef_step(const double* sums, double invT, Coef c,
                            int select, DevScalars* sc, hipStream_t st,
                            const int* skip) {
  hipLaunchKernelGGL(coef_step_kernel, dim3(1), dim3(64), 0, st, sums, invT, c,
                     select, sc, skip);
  return hipGetLastError();
}
hipError_t launch_segment_decide(const double* sums, double invT, Coef c,
                                 int select, const double* x, int64_t n,
                                 double tau, double* d, const double* tmp,
                                 const double* mask, double* hold,
                                 DevScalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(segment_decide_kernel, dim3(1), dim3(VT), 0, st, sums,
                     invT, c, select, x, n, tau, d, tmp, mask, hold, sc);
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
