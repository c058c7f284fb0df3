// libyand C-ABI: context, sample-oracle entry points and the YAND-MVSK solve
// loop (Algorithm 1), driving the HIP kernels of pass.hip, dense.hip and
// vec.hip on the caller's stream.
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/yand.h"
#include "common.h"
#include "kernels.h"
#include "vec.h"

using namespace yand;

namespace {

struct TimedLaunch {
  const char* name;
  hipEvent_t a, b;
};

}  // namespace

struct yand_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int precision = 0;
  int64_t T = 0, n = 0, Tp = 0, lda = 0, nt = 0;
  size_t esize = 8;
  void* A = nullptr;
  double* mu = nullptr;
  double* Efix = nullptr;   // 2 x n: e1 = 1/sqrt(n), e2 = unit centred mu
  double* AEfix = nullptr;  // 2 x Tp: A e1, A e2
  bool have_e2 = false;
  // per-iteration vectors
  double *x = nullptr, *g = nullptr, *d = nullptr, *z = nullptr, *wv = nullptr,
         *q = nullptr, *AE = nullptr, *E = nullptr, *W = nullptr,
         *t3 = nullptr, *r = nullptr, *y = nullptr, *y2 = nullptr,
         *hv = nullptr, *s_t = nullptr;
  double *pcg_s = nullptr, *pcg_res = nullptr, *pcg_p = nullptr,
         *pcg_u = nullptr;
  double *part = nullptr, *psums = nullptr, *sums = nullptr,
         *trpart = nullptr;
  double *B = nullptr, *M = nullptr, *X = nullptr, *rn = nullptr;
  DevScalars* sc = nullptr;
  DevScalars hs{};
  // profiling
  bool profiling = false;
  std::vector<TimedLaunch> timed;
  std::vector<std::pair<std::string, std::pair<double, int64_t>>> prof;
};

namespace {

int alloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes < 256 ? 256 : bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return YAND_ERR_OOM;
  }
  return YAND_OK;
}

#define TRY(expr)                   \
  do {                              \
    int _rc = (expr);               \
    if (_rc != YAND_OK) return _rc; \
  } while (0)

#define HIPTRY(expr)                                                      \
  do {                                                                    \
    hipError_t _e = (expr);                                               \
    if (_e != hipSuccess) {                                               \
      fprintf(stderr, "libyand: %s: %s (%s:%d)\n", #expr,                 \
              hipGetErrorString(_e), __FILE__, __LINE__);                 \
      return YAND_ERR_HIP;                                                \
    }                                                                     \
  } while (0)

Coef to_coef(const double c[4]) { return Coef{c[0], c[1], c[2], c[3]}; }

int check_c(const double* c) {
  if (!c) return YAND_ERR_ARG;
  for (int i = 0; i < 4; ++i)
    if (!(c[i] >= 0.0) || !std::isfinite(c[i])) return YAND_ERR_ARG;
  return YAND_OK;
}

// Timed launch wrapper: records events around `fn` when profiling is on.
template <class F>
hipError_t timed(yand_ctx* ctx, const char* name, F fn) {
  if (!ctx->profiling) return fn();
  TimedLaunch t{name, nullptr, nullptr};
  if (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess)
    return hipErrorOutOfMemory;
  hipEventRecord(t.a, ctx->stream);
  hipError_t e = fn();
  hipEventRecord(t.b, ctx->stream);
  ctx->timed.push_back(t);
  return e;
}

void flush_timed(yand_ctx* ctx) {
  if (ctx->timed.empty()) return;
  hipStreamSynchronize(ctx->stream);
  for (auto& t : ctx->timed) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, t.a, t.b);
    bool found = false;
    for (auto& p : ctx->prof)
      if (p.first == t.name) {
        p.second.first += ms;
        p.second.second += 1;
        found = true;
        break;
      }
    if (!found) ctx->prof.push_back({t.name, {(double)ms, 1}});
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  ctx->timed.clear();
}

PassArgs pass_args(yand_ctx* ctx, const double c[4]) {
  PassArgs a{};
  a.A = ctx->A;
  a.lda = ctx->lda;
  a.Tp = ctx->Tp;
  a.n = ctx->n;
  a.part = ctx->part;
  a.psums = ctx->psums;
  a.c = c ? to_coef(c) : Coef{0, 0, 0, 0};
  a.invT = 1.0 / (double)ctx->T;
  return a;
}

int run_pass(yand_ctx* ctx, PassKind kind, const PassArgs& a, int* nwg,
             const char* name) {
  HIPTRY(timed(ctx, name, [&] {
    return launch_pass(ctx->precision, kind, a, ctx->stream, nwg);
  }));
  return YAND_OK;
}

int sync_scalars(yand_ctx* ctx) {
  HIPTRY(hipMemcpyAsync(&ctx->hs, ctx->sc, sizeof(DevScalars),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPTRY(hipStreamSynchronize(ctx->stream));
  return YAND_OK;
}

// Oracle pass at x: z (ctx->z), g (ctx->g), f and moments in ctx->sc.
int oracle_at(yand_ctx* ctx, const double c[4], const double* x,
              bool with_grad) {
  PassArgs a = pass_args(ctx, c);
  a.v = x;
  a.tout = ctx->z;
  int nwg = 0;
  TRY(run_pass(ctx, with_grad ? PassKind::Oracle : PassKind::Value, a, &nwg,
               "oracle_pass"));
  HIPTRY(launch_reduce_sums(ctx->psums, nwg, 3, ctx->sums, ctx->stream));
  HIPTRY(launch_dot(ctx->mu, x, ctx->n, &ctx->sc->mux, ctx->stream));
  HIPTRY(launch_objective(ctx->sums, a.invT, to_coef(c), ctx->sc,
                          ctx->stream));
  if (with_grad)
    HIPTRY(launch_reduce_partials(ctx->part, nwg, ctx->lda, ctx->n, 1.0,
                                  -c[0], ctx->mu, ctx->g, ctx->stream));
  return YAND_OK;
}

// hv = A^T (psi''(z) * Av) / T at the cached z; (Av)_t to tout if given.
int hvp_cached(yand_ctx* ctx, const double c[4], const double* v, double* hv,
               double* tout) {
  PassArgs a = pass_args(ctx, c);
  a.v = v;
  a.zc = ctx->z;
  a.tout = tout;
  int nwg = 0;
  TRY(run_pass(ctx, PassKind::Hvp, a, &nwg, "hvp_pass"));
  HIPTRY(launch_reduce_partials(ctx->part, nwg, ctx->lda, ctx->n, 1.0, 0.0,
                                nullptr, hv, ctx->stream));
  return YAND_OK;
}

// Line-search sums along d at the cached z; coefficients (and optionally the
// step) in ctx->sc.  mu^T d must already be in sc->mud.
int line_at(yand_ctx* ctx, const double c[4], const double* d, int select) {
  PassArgs a = pass_args(ctx, c);
  a.v = d;
  a.zc = ctx->z;
  a.tout = ctx->wv;
  int nwg = 0;
  TRY(run_pass(ctx, PassKind::Line, a, &nwg, "line_pass"));
  HIPTRY(launch_reduce_sums(ctx->psums, nwg, 9, ctx->sums, ctx->stream));
  HIPTRY(launch_coef_step(ctx->sums, a.invT, to_coef(c), select, ctx->sc,
                          ctx->stream));
  return YAND_OK;
}

int ensure_dense(yand_ctx* ctx) {
  if (ctx->B) return YAND_OK;
  const size_t nn = (size_t)ctx->lda * ctx->lda * sizeof(double);
  TRY(alloc((void**)&ctx->B, nn));
  TRY(alloc((void**)&ctx->M, nn));
  TRY(alloc((void**)&ctx->X, nn));
  TRY(alloc((void**)&ctx->rn, (size_t)ctx->nt * ctx->Tp * sizeof(double)));
  return YAND_OK;
}

__global__ void psi2_weight_kernel(const double* __restrict__ z, int64_t Tp,
                                   Coef c, double invT, double* __restrict__ s) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < Tp) s[t] = d2psi(c, z[t]) * invT;
}

__global__ void fill_kernel(double* p, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t fill(double* p, int64_t count, double v, hipStream_t st) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p,
                     count, v);
  return hipGetLastError();
}

__global__ void set_lambda_kernel(DevScalars* sc, double lam) {
  if (threadIdx.x == 0) sc->lambda = lam;
}

// Projected PCG on P_S (H + lambda) P_S s = r (s in S) with the Jacobi
// preconditioner P_S diag(B + lambda)^-1 P_S; r already in S.
constexpr int PT = 1024;
template <int K>
__device__ void bsum(double (&v)[K], double* sh) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) sh[k * 16 + w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int i = 0; i < 16; ++i) s += sh[k * 16 + i];
    v[k] = s;
  }
  __syncthreads();
}

__device__ double precond_diag(const double* B, int64_t ld, int64_t j,
                               double lam) {
  double dj = B[j * ld + j] + lam;
  return dj > 0.0 ? dj : 1.0;
}

__global__ void __launch_bounds__(PT)
pcg_init_kernel(const double* __restrict__ r, const double* __restrict__ B,
                int64_t ld, const double* __restrict__ E, int p, int64_t n,
                double* s, double* res, double* pv, double* u,
                DevScalars* sc) {
  __shared__ double sh[4 * 16];
  const int tid = threadIdx.x;
  const double lam = sc->lambda;
  double dots[4] = {0, 0, 0, 0};
  for (int64_t j = tid; j < n; j += PT) {
    s[j] = 0.0;
    res[j] = r[j];
    double uj = r[j] / precond_diag(B, ld, j, lam);
    u[j] = uj;
    for (int a = 0; a < p; ++a) dots[a] += E[a * n + j] * uj;
    dots[3] += r[j] * r[j];
  }
  bsum(dots, sh);
  double rz[1] = {0.0};
  for (int64_t j = tid; j < n; j += PT) {
    double uj = u[j];
    for (int a = 0; a < p; ++a) uj -= dots[a] * E[a * n + j];
    u[j] = uj;
    pv[j] = uj;
    rz[0] += res[j] * uj;
  }
  bsum(rz, sh);
  if (tid == 0) {
    sc->aux[0] = rz[0];
    sc->aux[1] = dots[3];
    sc->aux[2] = dots[3];
  }
}

__global__ void __launch_bounds__(PT)
pcg_update_kernel(const double* __restrict__ Hp, const double* __restrict__ B,
                  int64_t ld, const double* __restrict__ E, int p, int64_t n,
                  double* s, double* res, double* pv, double* u, double* Ap,
                  DevScalars* sc) {
  __shared__ double sh[4 * 16];
  const int tid = threadIdx.x;
  const double lam = sc->lambda;
  double dots[4] = {0, 0, 0, 0};
  for (int64_t j = tid; j < n; j += PT) {
    double a = Hp[j] + lam * pv[j];
    Ap[j] = a;
    for (int k = 0; k < p; ++k) dots[k] += E[k * n + j] * a;
  }
  bsum(dots, sh);
  double pap[1] = {0.0};
  for (int64_t j = tid; j < n; j += PT) {
    double a = Ap[j];
    for (int k = 0; k < p; ++k) a -= dots[k] * E[k * n + j];
    Ap[j] = a;
    pap[0] += pv[j] * a;
  }
  bsum(pap, sh);
  const double rz = sc->aux[0];
  const double al = pap[0] > 0.0 ? rz / pap[0] : 0.0;
  double d2[4] = {0, 0, 0, 0};
  for (int64_t j = tid; j < n; j += PT) {
    s[j] += al * pv[j];
    double rj = res[j] - al * Ap[j];
    res[j] = rj;
    double uj = rj / precond_diag(B, ld, j, lam);
    u[j] = uj;
    for (int k = 0; k < p; ++k) d2[k] += E[k * n + j] * uj;
    d2[3] += rj * rj;
  }
  bsum(d2, sh);
  double rzn[1] = {0.0};
  for (int64_t j = tid; j < n; j += PT) {
    double uj = u[j];
    for (int k = 0; k < p; ++k) uj -= d2[k] * E[k * n + j];
    u[j] = uj;
    rzn[0] += res[j] * uj;
  }
  bsum(rzn, sh);
  const double beta = rz > 0.0 ? rzn[0] / rz : 0.0;
  for (int64_t j = tid; j < n; j += PT) pv[j] = u[j] + beta * pv[j];
  if (tid == 0) {
    sc->aux[0] = rzn[0];
    sc->aux[1] = d2[3];
    if (!(pap[0] > 0.0)) sc->aux[3] = 1.0;  // curvature breakdown
  }
}

struct DirOpts {
  int solver = YAND_SOLVER_DIRECT;
  double reg = 0.0;
  double krylov_tol = 1e-3;
  int krylov_maxit = 15;
  double tau = 1e-8;
  int simplex = 0;
};

struct DirStats {
  int cg = 0;
  int escalations = 0;
};

// Affine-normal direction at x (oracle pass already done at x: z, g valid).
// p0 = number of equality constraints (1 budget, 2 budget + target).
int direction_at(yand_ctx* ctx, const double c[4], int p0, const double* x,
                 const DirOpts& o, double* d, DirStats* stats) {
  TRY(ensure_dense(ctx));
  hipStream_t st = ctx->stream;
  const int64_t n = ctx->n, np = ctx->lda, Tp = ctx->Tp;
  const int p = p0 + 1;
  const double invT = 1.0 / (double)ctx->T;
  // nu and |G|
  HIPTRY(launch_grad_project(ctx->g, ctx->E, p0, n, ctx->sc, st));
  // (A nu)_t -> AE[p0]
  {
    PassArgs a = pass_args(ctx, c);
    a.v = ctx->E + (int64_t)p0 * n;
    a.tout = ctx->AE + (int64_t)p0 * Tp;
    int nwg;
    TRY(run_pass(ctx, PassKind::Dot, a, &nwg, "dot_pass"));
  }
  // B = A^T diag(psi''(z)/T) A
  hipLaunchKernelGGL(psi2_weight_kernel, dim3((unsigned)((Tp + 255) / 256)),
                     dim3(256), 0, st, ctx->z, Tp, to_coef(c), invT, ctx->s_t);
  HIPTRY(timed(ctx, "syrk", [&] {
    return launch_syrk(ctx->precision, ctx->A, ctx->lda, Tp, ctx->s_t, ctx->B,
                       st);
  }));
  HIPTRY(launch_symm_multi(ctx->B, np, n, ctx->E, p, ctx->W, st));
  HIPTRY(launch_trace_scale(ctx->B, np, n, ctx->E, ctx->W, p, o.reg, ctx->sc,
                            st));
  // project, factor, invert (with regularisation escalation)
  double lam = -1.0;
  for (int attempt = 0;; ++attempt) {
    if (lam >= 0.0)
      hipLaunchKernelGGL(set_lambda_kernel, dim3(1), dim3(64), 0, st, ctx->sc,
                         lam);
    HIPTRY(launch_project(ctx->B, ctx->M, np, n, np, ctx->E, ctx->W, p,
                          ctx->sc, st));
    HIPTRY(fill(ctx->X, np * np, 0.0, st));
    HIPTRY(hipMemsetAsync(&ctx->sc->fail, 0, sizeof(int), st));
    HIPTRY(timed(ctx, "potrf_trtri", [&] {
      return launch_potrf_trtri(ctx->M, ctx->X, np, &ctx->sc->fail, st);
    }));
    TRY(sync_scalars(ctx));
    if (!ctx->hs.fail) break;
    if (attempt >= 8) return YAND_ERR_INDEFINITE;
    lam = std::max(10.0 * ctx->hs.lambda, 1e-12 * ctx->hs.tang_scale);
    if (stats) stats->escalations++;
  }
  // q_t and the third-order back-projection t3 = A^T(psi'''(z) q)/T
  HIPTRY(timed(ctx, "trace_gemm", [&] {
    return launch_trace_gemm(ctx->precision, ctx->A, ctx->lda, Tp, ctx->X, np,
                             ctx->rn, st);
  }));
  hipMemcpyAsync(ctx->AE, ctx->AEfix, (size_t)p0 * Tp * sizeof(double),
                 hipMemcpyDeviceToDevice, st);
  HIPTRY(launch_trace_weight(ctx->rn, (int)ctx->nt, Tp, ctx->AE, p, ctx->sc,
                             ctx->q, st));
  {
    PassArgs a = pass_args(ctx, c);
    a.zc = ctx->z;
    a.q = ctx->q;
    int nwg;
    TRY(run_pass(ctx, PassKind::Third, a, &nwg, "third_pass"));
    HIPTRY(launch_reduce_partials(ctx->part, nwg, ctx->lda, n, 1.0, 0.0,
                                  nullptr, ctx->t3, st));
  }
  // r = P_S (B nu - |G|/(m+1) t3), m = n - p0
  const double mp1 = (double)(n - p0 + 1);
  HIPTRY(launch_rhs(ctx->W + (int64_t)p0 * n, ctx->t3, ctx->E, p, n, mp1,
                    ctx->sc, ctx->r, st));
  if (o.solver == YAND_SOLVER_DIRECT) {
    HIPTRY(launch_trmv(ctx->X, np, n, ctx->r, ctx->y, ctx->trpart, false, st));
    HIPTRY(launch_trmv(ctx->X, np, n, ctx->y, ctx->y2, ctx->trpart, true, st));
    HIPTRY(launch_direction(ctx->y2, ctx->E, p, n, x, ctx->mu, o.tau,
                            o.simplex, d, ctx->sc, st));
  } else {
    hipLaunchKernelGGL(pcg_init_kernel, dim3(1), dim3(PT), 0, st, ctx->r,
                       ctx->B, np, ctx->E, p, n, ctx->pcg_s, ctx->pcg_res,
                       ctx->pcg_p, ctx->pcg_u, ctx->sc);
    TRY(sync_scalars(ctx));
    const double r0 = std::sqrt(ctx->hs.aux[2]);
    int it = 0;
    while (it < o.krylov_maxit && r0 > 0.0) {
      TRY(hvp_cached(ctx, c, ctx->pcg_p, ctx->hv, nullptr));
      hipLaunchKernelGGL(pcg_update_kernel, dim3(1), dim3(PT), 0, st, ctx->hv,
                         ctx->B, np, ctx->E, p, n, ctx->pcg_s, ctx->pcg_res,
                         ctx->pcg_p, ctx->pcg_u, ctx->y, ctx->sc);
      ++it;
      TRY(sync_scalars(ctx));
      if (std::sqrt(ctx->hs.aux[1]) <= o.krylov_tol * r0) break;
      if (ctx->hs.aux[3] != 0.0) break;
    }
    if (stats) stats->cg += it;
    HIPTRY(launch_direction(ctx->pcg_s, ctx->E, p, n, x, ctx->mu, o.tau,
                            o.simplex, d, ctx->sc, st));
  }
  return YAND_OK;
}

int setup_constraints(yand_ctx* ctx, const double* target, int* p0) {
  *p0 = target ? 2 : 1;
  if (target && !ctx->have_e2) return YAND_ERR_ARG;
  HIPTRY(hipMemcpyAsync(ctx->E, ctx->Efix, (size_t)(*p0) * ctx->n *
                        sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  return YAND_OK;
}

// Minimum-norm correction of x onto 1^T x = 1 (and mu^T x = r): with the
// orthonormal e1, e2 of span{1, mu}, x <- x + sum_a e_a (b_a' - e_a^T x),
// where b' are the right-hand sides in the e-basis.
__global__ void __launch_bounds__(PT)
feasible_kernel(double* x, const double* E, int p0, int64_t n,
                double b1, double b2) {
  __shared__ double sh[4 * 16];
  const int tid = threadIdx.x;
  double dots[2] = {0, 0};
  for (int64_t j = tid; j < n; j += PT)
    for (int a = 0; a < p0; ++a) dots[a] += E[a * n + j] * x[j];
  bsum(dots, sh);
  const double bb[2] = {b1, b2};
  for (int64_t j = tid; j < n; j += PT) {
    double v = x[j];
    for (int a = 0; a < p0; ++a) v += E[a * n + j] * (bb[a] - dots[a]);
    x[j] = v;
  }
}

__global__ void __launch_bounds__(PT)
efix_kernel(const double* __restrict__ mu, int64_t n, double* Efix,
            int* has_e2) {
  __shared__ double sh[4 * 16];
  const int tid = threadIdx.x;
  const double e1 = 1.0 / sqrt((double)n);
  double s[1] = {0.0};
  for (int64_t j = tid; j < n; j += PT) {
    Efix[j] = e1;
    s[0] += mu[j];
  }
  bsum(s, sh);
  const double mbar = s[0] / (double)n;
  double ss[1] = {0.0};
  for (int64_t j = tid; j < n; j += PT) {
    double v = mu[j] - mbar;
    ss[0] += v * v;
  }
  bsum(ss, sh);
  const double nrm = sqrt(ss[0]);
  for (int64_t j = tid; j < n; j += PT)
    Efix[n + j] = nrm > 0.0 ? (mu[j] - mbar) / nrm : 0.0;
  if (tid == 0) *has_e2 = nrm > 1e-300 ? 1 : 0;
}

}  // namespace

// ===================================================================== ABI ==

extern "C" {

void yand_default_opts(yand_opts* o) {
  if (!o) return;
  o->solver = YAND_SOLVER_DIRECT;
  o->feasible_set = YAND_SET_BUDGET;
  o->eps = 1e-8;
  o->max_iter = 300;
  o->max_elapsed = 0.0;
  o->regularization = 0.0;
  o->krylov_tol = 1e-3;
  o->krylov_maxit = 15;
  o->tau = 1e-8;
  o->stall_recovery = 1;
  o->restart_max_iter = 120;
}

void yand_large_opts(yand_opts* o) {
  yand_default_opts(o);
  if (!o) return;
  o->solver = YAND_SOLVER_PCG;
  o->max_iter = 40;
  o->max_elapsed = 60.0;
  o->regularization = 1e-4;
}

int yand_is_certified_convex(const double c[4]) {
  if (!c) return 0;
  return (c[3] > 0.0 && 8.0 * c[1] * c[3] > 3.0 * c[2] * c[2]) ? 1 : 0;
}

int yand_destroy(yand_ctx* ctx) {
  if (!ctx) return YAND_OK;
  flush_timed(ctx);
  void* ptrs[] = {ctx->A, ctx->mu, ctx->Efix, ctx->AEfix, ctx->x, ctx->g,
                  ctx->d, ctx->z, ctx->wv, ctx->q, ctx->AE, ctx->E, ctx->W,
                  ctx->t3, ctx->r, ctx->y, ctx->y2, ctx->hv, ctx->s_t,
                  ctx->pcg_s, ctx->pcg_res, ctx->pcg_p, ctx->pcg_u, ctx->part,
                  ctx->psums, ctx->sums, ctx->trpart, ctx->B, ctx->M, ctx->X,
                  ctx->rn, ctx->sc};
  for (void* p : ptrs)
    if (p) hipFree(p);
  delete ctx;
  return YAND_OK;
}

int yand_create(const double* R, int64_t T, int64_t n, int64_t ldr,
                int precision, void* hip_stream, yand_ctx** out) {
  if (!out) return YAND_ERR_ARG;
  *out = nullptr;
  if (!R || T < 2 || n < 2 || ldr < n) return YAND_ERR_ARG;
  if (precision < 0 || precision > 2) return YAND_ERR_ARG;
  if (n > max_pass_columns(precision)) return YAND_ERR_ARG;
  yand_ctx* ctx = new yand_ctx();
  ctx->stream = (hipStream_t)hip_stream;
  hipGetDevice(&ctx->device);
  ctx->precision = precision;
  ctx->T = T;
  ctx->n = n;
  ctx->Tp = round_up(T, kRowPad);
  ctx->lda = round_up(n, kColPad);
  ctx->nt = ctx->lda / kTile;
  ctx->esize = precision == 0 ? 8 : precision == 1 ? 4 : 2;
  const int64_t Tp = ctx->Tp, lda = ctx->lda;
  auto fail = [&](int rc) {
    yand_destroy(ctx);
    return rc;
  };
  int rc = YAND_OK;
  const size_t nb = (size_t)lda * sizeof(double), tb = (size_t)Tp * sizeof(double);
  if ((rc = alloc(&ctx->A, (size_t)Tp * lda * ctx->esize)) ||
      (rc = alloc((void**)&ctx->mu, nb)) ||
      (rc = alloc((void**)&ctx->Efix, 2 * nb)) ||
      (rc = alloc((void**)&ctx->AEfix, 2 * tb)) ||
      (rc = alloc((void**)&ctx->x, nb)) || (rc = alloc((void**)&ctx->g, nb)) ||
      (rc = alloc((void**)&ctx->d, nb)) || (rc = alloc((void**)&ctx->z, tb)) ||
      (rc = alloc((void**)&ctx->wv, tb)) || (rc = alloc((void**)&ctx->q, tb)) ||
      (rc = alloc((void**)&ctx->AE, 3 * tb)) ||
      (rc = alloc((void**)&ctx->E, 3 * nb)) ||
      (rc = alloc((void**)&ctx->W, 3 * nb)) ||
      (rc = alloc((void**)&ctx->t3, nb)) || (rc = alloc((void**)&ctx->r, nb)) ||
      (rc = alloc((void**)&ctx->y, nb)) || (rc = alloc((void**)&ctx->y2, nb)) ||
      (rc = alloc((void**)&ctx->hv, nb)) || (rc = alloc((void**)&ctx->s_t, tb)) ||
      (rc = alloc((void**)&ctx->pcg_s, nb)) ||
      (rc = alloc((void**)&ctx->pcg_res, nb)) ||
      (rc = alloc((void**)&ctx->pcg_p, nb)) ||
      (rc = alloc((void**)&ctx->pcg_u, nb)) ||
      (rc = alloc((void**)&ctx->part,
                  (size_t)kMaxPassGroups * lda * sizeof(double))) ||
      (rc = alloc((void**)&ctx->psums,
                  (size_t)kMaxPassGroups * kMaxSums * sizeof(double))) ||
      (rc = alloc((void**)&ctx->sums, kMaxSums * sizeof(double))) ||
      (rc = alloc((void**)&ctx->trpart,
                  (size_t)((n + 63) / 64) * n * sizeof(double))) ||
      (rc = alloc((void**)&ctx->sc, sizeof(DevScalars))))
    return fail(rc);
  hipStream_t st = ctx->stream;
  if (hipMemsetAsync(ctx->sc, 0, sizeof(DevScalars), st) != hipSuccess ||
      fill(ctx->z, Tp, 0.0, st) != hipSuccess ||
      fill(ctx->q, Tp, 0.0, st) != hipSuccess ||
      fill(ctx->AE, 3 * Tp, 0.0, st) != hipSuccess)
    return fail(YAND_ERR_HIP);
  double* colpart = nullptr;
  const int64_t nchunks = (T + 255) / 256;
  if ((rc = alloc((void**)&colpart, (size_t)nchunks * n * sizeof(double))))
    return fail(rc);
  hipError_t e = launch_center(R, T, n, ldr, precision, ctx->A, Tp, lda,
                               ctx->mu, colpart, &ctx->sc->nonfinite, st);
  if (e != hipSuccess) {
    hipFree(colpart);
    return fail(YAND_ERR_HIP);
  }
  // constraint frame and the fixed projections A e1, A e2
  int* has_e2 = (int*)&ctx->sc->pad;
  hipLaunchKernelGGL(efix_kernel, dim3(1), dim3(PT), 0, st, ctx->mu, n,
                     ctx->Efix, has_e2);
  for (int a = 0; a < 2; ++a) {
    PassArgs pa = pass_args(ctx, nullptr);
    pa.v = ctx->Efix + (int64_t)a * n;
    pa.tout = ctx->AEfix + (int64_t)a * Tp;
    int nwg;
    if (launch_pass(precision, PassKind::Dot, pa, st, &nwg) != hipSuccess) {
      hipFree(colpart);
      return fail(YAND_ERR_HIP);
    }
  }
  if (sync_scalars(ctx) != YAND_OK) {
    hipFree(colpart);
    return fail(YAND_ERR_HIP);
  }
  hipFree(colpart);
  if (ctx->hs.nonfinite) return fail(YAND_ERR_NONFINITE);
  ctx->have_e2 = ctx->hs.pad != 0;
  *out = ctx;
  return YAND_OK;
}

int yand_shape(yand_ctx* ctx, int64_t* T, int64_t* n, int* precision) {
  if (!ctx) return YAND_ERR_ARG;
  if (T) *T = ctx->T;
  if (n) *n = ctx->n;
  if (precision) *precision = ctx->precision;
  return YAND_OK;
}

int yand_get_mu(yand_ctx* ctx, double* mu_out) {
  if (!ctx || !mu_out) return YAND_ERR_ARG;
  HIPTRY(hipMemcpyAsync(mu_out, ctx->mu, ctx->n * sizeof(double),
                        hipMemcpyDeviceToDevice, ctx->stream));
  HIPTRY(hipStreamSynchronize(ctx->stream));
  return YAND_OK;
}

int yand_eval(yand_ctx* ctx, const double c[4], const double* w, double* f,
              double* grad, double mom[4]) {
  if (!ctx || !w) return YAND_ERR_ARG;
  TRY(check_c(c));
  TRY(oracle_at(ctx, c, w, grad != nullptr));
  if (grad)
    HIPTRY(hipMemcpyAsync(grad, ctx->g, ctx->n * sizeof(double),
                          hipMemcpyDeviceToDevice, ctx->stream));
  TRY(sync_scalars(ctx));
  if (f) *f = ctx->hs.f;
  if (mom)
    for (int i = 0; i < 4; ++i) mom[i] = ctx->hs.mom[i];
  flush_timed(ctx);
  return ctx->hs.nonfinite ? YAND_ERR_NONFINITE : YAND_OK;
}

int yand_hvp(yand_ctx* ctx, const double c[4], const double* w,
             const double* v, double* hv) {
  if (!ctx || !w || !v || !hv) return YAND_ERR_ARG;
  TRY(check_c(c));
  TRY(oracle_at(ctx, c, w, false));
  TRY(hvp_cached(ctx, c, v, hv, nullptr));
  HIPTRY(hipStreamSynchronize(ctx->stream));
  flush_timed(ctx);
  return YAND_OK;
}

int yand_linesearch_coeffs(yand_ctx* ctx, const double c[4], const double* w,
                           const double* d, double coef[5]) {
  if (!ctx || !w || !d || !coef) return YAND_ERR_ARG;
  TRY(check_c(c));
  TRY(oracle_at(ctx, c, w, false));
  HIPTRY(launch_dot(ctx->mu, d, ctx->n, &ctx->sc->mud, ctx->stream));
  TRY(line_at(ctx, c, d, 0));
  TRY(sync_scalars(ctx));
  for (int i = 0; i < 5; ++i) coef[i] = ctx->hs.coef[i];
  flush_timed(ctx);
  return YAND_OK;
}

int yand_select_step(yand_ctx* ctx, const double coef[5], double alpha_max,
                     double* alpha) {
  if (!ctx || !coef || !alpha) return YAND_ERR_ARG;
  if (std::isnan(alpha_max) || alpha_max < 0.0) return YAND_ERR_ARG;
  DevScalars hs = ctx->hs;
  for (int i = 0; i < 5; ++i) hs.coef[i] = coef[i];
  hs.amax = alpha_max;
  HIPTRY(hipMemcpyAsync(ctx->sc, &hs, sizeof(DevScalars),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPTRY(launch_select_step(ctx->sc, ctx->stream));
  TRY(sync_scalars(ctx));
  *alpha = ctx->hs.alpha;
  return ctx->hs.status == 0 ? YAND_OK : YAND_ERR_UNBOUNDED;
}

int yand_affine_normal(yand_ctx* ctx, const double c[4], const double* target,
                       const double* w, const yand_opts* opts, double* d_out,
                       double* gnorm) {
  if (!ctx || !w || !d_out) return YAND_ERR_ARG;
  TRY(check_c(c));
  int p0;
  TRY(setup_constraints(ctx, target, &p0));
  DirOpts o;
  if (opts) {
    o.solver = opts->solver;
    o.reg = opts->regularization;
    o.krylov_tol = opts->krylov_tol;
    o.krylov_maxit = opts->krylov_maxit;
    o.tau = opts->tau;
  }
  TRY(oracle_at(ctx, c, w, true));
  TRY(direction_at(ctx, c, p0, w, o, d_out, nullptr));
  TRY(sync_scalars(ctx));
  if (gnorm) *gnorm = ctx->hs.gn;
  flush_timed(ctx);
  return ctx->hs.nonfinite ? YAND_ERR_NONFINITE : YAND_OK;
}

int yand_mvsk_solve(yand_ctx* ctx, const double c[4], const double* target,
                    const double* w0, const yand_opts* opts_in,
                    double* w_out, yand_info* info) {
  if (!ctx || !w_out) return YAND_ERR_ARG;
  TRY(check_c(c));
  yand_opts opts;
  if (opts_in)
    opts = *opts_in;
  else
    yand_default_opts(&opts);
  if (opts.eps < 0.0 || opts.max_iter < 0 || opts.tau < 0.0)
    return YAND_ERR_ARG;
  if (target && !std::isfinite(*target)) return YAND_ERR_ARG;
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t st = ctx->stream;
  const int64_t n = ctx->n;
  int p0;
  TRY(setup_constraints(ctx, target, &p0));
  // starting point: w0 or equal weights, moved onto the constraints
  if (w0)
    HIPTRY(hipMemcpyAsync(ctx->x, w0, n * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
  else
    HIPTRY(fill(ctx->x, n, 1.0 / (double)n, st));
  {
    // right-hand sides in the orthonormal e-basis: e1^T x = 1/sqrt(n);
    // e2^T x = (r - mbar) / |mu - mbar| where mbar = mean(mu).
    std::vector<double> mu_h(n);
    HIPTRY(hipMemcpyAsync(mu_h.data(), ctx->mu, n * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    double mbar = 0.0, ss = 0.0;
    for (int64_t j = 0; j < n; ++j) mbar += mu_h[j];
    mbar /= (double)n;
    for (int64_t j = 0; j < n; ++j) ss += (mu_h[j] - mbar) * (mu_h[j] - mbar);
    const double b1 = 1.0 / std::sqrt((double)n);
    const double b2 = target ? (*target - mbar) / std::sqrt(ss) : 0.0;
    hipLaunchKernelGGL(feasible_kernel, dim3(1), dim3(PT), 0, st, ctx->x,
                       ctx->E, p0, n, b1, b2);
  }
  DirOpts o;
  o.reg = opts.regularization;
  o.krylov_tol = opts.krylov_tol;
  o.krylov_maxit = opts.krylov_maxit;
  o.tau = opts.tau;
  o.simplex = opts.feasible_set == YAND_SET_SIMPLEX;
  if (o.simplex) {
    // the start must lie in Delta(tau)
    std::vector<double> xh(n);
    HIPTRY(hipMemcpyAsync(xh.data(), ctx->x, n * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    for (int64_t j = 0; j < n; ++j)
      if (!(xh[j] >= opts.tau)) return YAND_ERR_ARG;
  }
  yand_info inf{};
  int status = YAND_WARN_MAXITER;
  int rc = YAND_OK;
  // phases: baseline, then (PCG with stall recovery) mild and aggressive
  struct Phase {
    int solver, kmax, max_iter;
    double reg;
  };
  std::vector<Phase> phases;
  phases.push_back({opts.solver, opts.krylov_maxit, opts.max_iter,
                    opts.solver == YAND_SOLVER_PCG ? opts.regularization
                                                   : 0.0});
  if (opts.solver == YAND_SOLVER_PCG && opts.stall_recovery) {
    phases.push_back({YAND_SOLVER_PCG, 2 * opts.krylov_maxit,
                      opts.restart_max_iter, opts.regularization});
    phases.push_back({YAND_SOLVER_DIRECT, 0, opts.restart_max_iter, 0.0});
  }
  bool converged = false;
  for (size_t ph = 0; ph < phases.size() && !converged && rc == YAND_OK;
       ++ph) {
    if (ph > 0) inf.restarts++;
    o.solver = phases[ph].solver;
    o.krylov_maxit = phases[ph].kmax;
    o.reg = phases[ph].reg;
    const auto t_phase = std::chrono::steady_clock::now();
    int small = 0;
    double f_prev = NAN;
    for (int it = 0;; ++it) {
      rc = oracle_at(ctx, c, ctx->x, true);
      if (rc) break;
      inf.oracle_passes++;
      rc = launch_grad_project(ctx->g, ctx->E, p0, n, ctx->sc, st) == hipSuccess
               ? YAND_OK
               : YAND_ERR_HIP;
      if (rc) break;
      if ((rc = sync_scalars(ctx))) break;
      inf.f = ctx->hs.f;
      inf.gnorm = ctx->hs.gn;
      if (ctx->hs.nonfinite) {
        rc = YAND_ERR_NONFINITE;
        break;
      }
      if (std::isnan(f_prev)) f_prev = ctx->hs.f;
      if (ctx->hs.gn <= opts.eps) {
        converged = true;
        break;
      }
      if (it >= phases[ph].max_iter) break;
      const double el = std::chrono::duration<double>(
                            std::chrono::steady_clock::now() - t_phase)
                            .count();
      if (opts.max_elapsed > 0.0 && el > opts.max_elapsed) break;
      DirStats ds;
      rc = direction_at(ctx, c, p0, ctx->x, o, ctx->d, &ds);
      if (rc) break;
      inf.dense_traces++;
      inf.third_passes++;
      inf.cg_iters += ds.cg;
      inf.hvp_passes += ds.cg;
      rc = line_at(ctx, c, ctx->d, 1);
      if (rc) break;
      inf.ls_passes++;
      if ((rc = sync_scalars(ctx))) break;
      inf.lambda_used = ctx->hs.lambda;
      if (ctx->hs.status != 0) {
        rc = YAND_ERR_UNBOUNDED;
        break;
      }
      HIPTRY(launch_axpy(ctx->x, ctx->d, n, ctx->sc, st));
      inf.iterations++;
      // stall: objective decrease below 1e-14 relative three times running
      const double a = ctx->hs.alpha, *A = ctx->hs.coef;
      const double dec = -(a * (A[1] + a * (A[2] + a * (A[3] + a * A[4]))));
      if (dec < 1e-14 * std::fabs(f_prev)) {
        if (++small >= 3) break;
      } else {
        small = 0;
      }
      f_prev = A[0] - dec;
    }
  }
  if (rc == YAND_OK) {
    if (converged)
      status = YAND_OK;
    else
      status = inf.restarts > 0 ? YAND_WARN_STALL : YAND_WARN_MAXITER;
    HIPTRY(hipMemcpyAsync(w_out, ctx->x, n * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
    HIPTRY(hipStreamSynchronize(st));
  } else {
    status = rc;
  }
  inf.status = status;
  inf.elapsed = std::chrono::duration<double>(
                    std::chrono::steady_clock::now() - t_start)
                    .count();
  if (info) *info = inf;
  flush_timed(ctx);
  return status;
}

int yand_mvsk_solve_R(const double* R, int64_t T, int64_t n, double c1,
                      double c2, double c3, double c4, const double* target,
                      double* w_out) {
  yand_ctx* ctx = nullptr;
  int rc = yand_create(R, T, n, n, YAND_FP64, nullptr, &ctx);
  if (rc) return rc;
  const double c[4] = {c1, c2, c3, c4};
  rc = yand_mvsk_solve(ctx, c, target, nullptr, nullptr, w_out, nullptr);
  yand_destroy(ctx);
  return rc;
}

// Per-kernel timing (instrumentation, not part of the method).
int yand_profile_enable(yand_ctx* ctx, int enable) {
  if (!ctx) return YAND_ERR_ARG;
  flush_timed(ctx);
  ctx->profiling = enable != 0;
  if (enable) ctx->prof.clear();
  return YAND_OK;
}

int yand_profile_read(yand_ctx* ctx, int index, char* name, int name_len,
                      double* total_ms, int64_t* count) {
  if (!ctx) return YAND_ERR_ARG;
  flush_timed(ctx);
  if (index < 0) return (int)ctx->prof.size();
  if (index >= (int)ctx->prof.size()) return YAND_ERR_ARG;
  const auto& p = ctx->prof[index];
  if (name && name_len > 0) {
    std::strncpy(name, p.first.c_str(), name_len - 1);
    name[name_len - 1] = 0;
  }
  if (total_ms) *total_ms = p.second.first;
  if (count) *count = p.second.second;
  return YAND_OK;
}

}  // extern "C"
