// libyand C-ABI: contexts, sample-oracle entry points, the YAND-MVSK outer
// loop (Algorithm 1) and the batched frontier solve, driving the HIP kernels
// of pass.hip, dense.hip and vec.hip.
//
// State is split in two.  Data (per context, immutable after creation) holds
// the centered matrix A at its storage precision, mu and the constraint frame.
// A Work (per solve lane) holds every per-iterate buffer, the device-resident
// scalars and a stream.  One outer iteration is enqueued as a fixed sequence
// of kernels with no host synchronisation: the stationarity test sets a device
// flag that makes the rest of the iteration return at once, and a failed
// factorisation forces a zero step.  The host reads the scalars of all lanes
// once per iteration and only then decides (stop, escalate the
// regularisation, freeze a lane).  The batched frontier captures one
// iteration of all lanes into a hipGraph and replays it.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/yand.h"
#include "common.h"
#include "kernels.h"
#include "mlp.h"
#include "vec.h"

using namespace yand;

namespace {

struct TimedLaunch {
  const char* name;
  hipEvent_t a, b;
};

struct Prof {
  bool on = false;
  std::vector<TimedLaunch> timed;
  std::vector<std::pair<std::string, std::pair<double, int64_t>>> acc;
};

struct Data {
  int device = 0;
  int precision = 0;
  int64_t T = 0, n = 0, Tp = 0, lda = 0, nt = 0;
  size_t esize = 8;
  void* A = nullptr;
  void* At = nullptr;       // A^T at the storage precision (FP32 / BF16 only)
  double* mu = nullptr;
  double* Efix = nullptr;   // 2 x n: e1 = 1/sqrt(n), e2 = unit centred mu
  double* AEfix = nullptr;  // 2 x Tp: A e1, A e2
  bool have_e2 = false;
  double mbar = 0.0, mnorm = 0.0;  // mean of mu and |mu - mbar|
  // launch shapes chosen by yand_autotune (0: built-in defaults)
  int pass_groups[6] = {0, 0, 0, 0, 0, 0};  // per PassKind
  int pass_rows[6] = {0, 0, 0, 0, 0, 0};    // rows per block, per PassKind
  int chol_group = 0;
  int chol_step_tm = 0;  // sub-block width of the in-group updates
  int chol_band = 0;     // band width of the panel step
  // XCD-aware tile order of the SYRK (device; null: plain order)
  int* syrk_order = nullptr;
  int64_t syrk_slots = 0;
  // balanced SYRK schedule over that order (device; null: not used)
  int* syrk_plan = nullptr;
  int syrk_wgs = 0, syrk_rounds = 0, syrk_ntile2 = 0, syrk_npieces = 0,
      syrk_nslots = 0;
};

struct Work {
  hipStream_t st = nullptr;
  bool own_stream = false;
  double *x = nullptr, *g = nullptr, *d = nullptr, *z = nullptr,
         *wv = nullptr, *q = nullptr, *AE = nullptr, *E = nullptr,
         *W = nullptr, *t3 = nullptr, *r = nullptr, *y = nullptr,
         *y2 = nullptr, *hv = nullptr, *s_t = nullptr;
  double *pcg_s = nullptr, *pcg_res = nullptr, *pcg_p = nullptr,
         *pcg_u = nullptr;
  double *part = nullptr, *psums = nullptr, *sums = nullptr,
         *trpart = nullptr;
  double *B = nullptr, *M = nullptr, *X = nullptr, *rn = nullptr;
  // FP32 / BF16 storage: s-scaled A^T and X rounded for the matrix cores
  void *SAt = nullptr, *Xl = nullptr;
  double *mask = nullptr, *ptmp = nullptr;  // face mask, projection scratch
  double* hold = nullptr;  // coordinates the face solver holds at the bound
  // T < n push-through trace: Gram partials, G, C, L^-1 of C, diag(B)
  double *tGp = nullptr, *tG = nullptr, *tC = nullptr, *tX = nullptr,
         *bdiag = nullptr, *tpart = nullptr;
  double* tW = nullptr;  // indefinite S: blocks of the signed factorisation
  // balanced SYRK: partial tiles and arrival counters
  double* syrk_ws = nullptr;
  int* syrk_cnt = nullptr;
  // probe estimate of the trace: signs and block products (Tp x 64), their
  // split partials, the block PCG vectors (64 x lda each) and per-column
  // scalars and flags
  double *pXi = nullptr, *pZ = nullptr, *pZp = nullptr, *pYp = nullptr,
         *pU = nullptr, *pY = nullptr, *pR = nullptr, *pW = nullptr,
         *pP = nullptr, *pHP = nullptr, *pAP = nullptr, *pcs = nullptr;
  int* pflags = nullptr;
  int tK = 0;
  int64_t tld = 0;
  DevScalars* sc = nullptr;
  bool own_sc = true;
  // lockstep lanes: B, M, X, rn and s_t point into the batch's strided
  // blocks (freed by the batch, not by the lane); with the PCG
  // configuration pcg_p and hv are rows of the batch's 64 x lda blocks
  bool shared_dense = false, shared_pcg = false;
  // the context's own workspace (single solves), as opposed to a batch lane
  // that shares the device with other lanes
  bool solo = false;
  DevScalars hs{};
  Prof* prof = nullptr;
};

}  // namespace

struct yand_ctx {
  Data d;
  Work w;
  Prof prof;
};

namespace {

// Device memory comes from hipMalloc, or, while an Arena is installed on the
// calling thread (the allocation-free entry point), from a bump allocator
// over the library's fixed scratch array: 256-byte aligned, never freed
// individually, YAND_ERR_TOO_LARGE once the array is exhausted.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
};
thread_local Arena* g_arena = nullptr;

int alloc(void** p, size_t bytes) {
  if (bytes < 256) bytes = 256;
  if (g_arena) {
    const size_t off = (g_arena->used + 255) & ~(size_t)255;
    if (off > g_arena->cap || bytes > g_arena->cap - off) {
      *p = nullptr;
      return YAND_ERR_TOO_LARGE;
    }
    *p = g_arena->base + off;
    g_arena->used = off + bytes;
    return YAND_OK;
  }
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return YAND_ERR_OOM;
  }
  return YAND_OK;
}

// Frees what alloc returned (arena memory is left to the arena).
void dfree(void* p) {
  if (!p) return;
  if (g_arena && (char*)p >= g_arena->base &&
      (char*)p < g_arena->base + g_arena->cap)
    return;
  (void)hipFree(p);
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

// ------------------------------------------------------------ profiling --

template <class F>
hipError_t timed(Work& w, const char* name, F fn) {
  if (!w.prof || !w.prof->on) return fn();
  TimedLaunch t{name, nullptr, nullptr};
  if (hipEventCreate(&t.a) != hipSuccess) return hipErrorOutOfMemory;
  if (hipEventCreate(&t.b) != hipSuccess) {
    (void)hipEventDestroy(t.a);
    return hipErrorOutOfMemory;
  }
  hipEventRecord(t.a, w.st);
  hipError_t e = fn();
  hipEventRecord(t.b, w.st);
  w.prof->timed.push_back(t);
  return e;
}

void flush_timed(Prof& p, hipStream_t st) {
  if (p.timed.empty()) return;
  (void)hipStreamSynchronize(st);
  for (auto& t : p.timed) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t.a, t.b);
    bool found = false;
    for (auto& a : p.acc)
      if (a.first == t.name) {
        a.second.first += ms;
        a.second.second += 1;
        found = true;
        break;
      }
    if (!found) p.acc.push_back({t.name, {(double)ms, 1}});
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  p.timed.clear();
}

// ------------------------------------------------------------ workspaces --

void free_work(Work& w) {
  if (w.shared_dense) w.B = w.M = w.X = w.rn = w.s_t = nullptr;
  if (w.shared_pcg) w.pcg_p = w.hv = nullptr;
  double* ptrs[] = {w.x,     w.g,      w.d,     w.z,      w.wv,   w.q,
                    w.AE,    w.E,      w.W,     w.t3,     w.r,    w.y,
                    w.y2,    w.hv,     w.s_t,   w.pcg_s,  w.pcg_res,
                    w.pcg_p, w.pcg_u,  w.part,  w.psums,  w.sums, w.trpart,
                    w.B,     w.M,      w.X,     w.rn,     w.mask, w.ptmp,
                    w.hold,  w.tGp,    w.tG,    w.tC,     w.tX,   w.bdiag,
                    w.tpart, w.tW};
  for (double* p : ptrs) dfree(p);
  dfree(w.SAt);
  dfree(w.Xl);
  double* pp[] = {w.pXi, w.pZ, w.pZp, w.pYp, w.pU, w.pY, w.pR, w.pW, w.pP,
                  w.pHP, w.pAP, w.pcs};
  for (double* q : pp) dfree(q);
  dfree(w.pflags);
  dfree(w.syrk_ws);
  dfree(w.syrk_cnt);
  if (w.sc && w.own_sc) dfree(w.sc);
  if (w.st && w.own_stream) (void)hipStreamDestroy(w.st);
  w = Work{};
}

int alloc_work(Work& w, const Data& D, DevScalars* sc_external) {
  const int64_t n = D.n, lda = D.lda, Tp = D.Tp;
  const size_t nb = (size_t)lda * sizeof(double), tb = (size_t)Tp * sizeof(double);
  int rc;
  if ((rc = alloc((void**)&w.x, nb)) || (rc = alloc((void**)&w.g, nb)) ||
      (rc = alloc((void**)&w.d, nb)) || (rc = alloc((void**)&w.z, tb)) ||
      (rc = alloc((void**)&w.wv, tb)) || (rc = alloc((void**)&w.q, tb)) ||
      (rc = alloc((void**)&w.AE, 3 * tb)) ||
      (rc = alloc((void**)&w.E, 3 * nb)) ||
      (rc = alloc((void**)&w.W, 3 * nb)) ||
      (rc = alloc((void**)&w.t3, nb)) || (rc = alloc((void**)&w.r, nb)) ||
      (rc = alloc((void**)&w.y, nb)) || (rc = alloc((void**)&w.y2, nb)) ||
      (rc = alloc((void**)&w.hv, nb)) || (rc = alloc((void**)&w.s_t, tb)) ||
      (rc = alloc((void**)&w.pcg_s, nb)) ||
      (rc = alloc((void**)&w.pcg_res, nb)) ||
      (rc = alloc((void**)&w.pcg_p, nb)) ||
      (rc = alloc((void**)&w.pcg_u, nb)) ||
      (rc = alloc((void**)&w.mask, nb)) || (rc = alloc((void**)&w.ptmp, nb)) ||
      (rc = alloc((void**)&w.hold, nb)) ||
      (rc = alloc((void**)&w.part,
                  (size_t)kMaxPassGroups * lda * sizeof(double))) ||
      (rc = alloc((void**)&w.psums,
                  (size_t)kMaxPassGroups * kMaxSums * sizeof(double))) ||
      (rc = alloc((void**)&w.sums, kMaxSums * sizeof(double))) ||
      (rc = alloc((void**)&w.trpart,
                  (size_t)((n + 63) / 64) * n * sizeof(double))))
    return rc;
  if (sc_external) {
    w.sc = sc_external;
    w.own_sc = false;
  } else {
    if ((rc = alloc((void**)&w.sc, sizeof(DevScalars)))) return rc;
    w.own_sc = true;
  }
  return YAND_OK;
}

// First contents of a workspace: zero scalars (when owned) and T-vectors.
int init_work(Work& w, const Data& D) {
  const int64_t Tp = D.Tp;
  static_assert(sizeof(DevScalars) % sizeof(double) == 0, "scalar block");
  if (w.own_sc)
    HIPTRY(launch_fill((double*)w.sc, sizeof(DevScalars) / sizeof(double), 0.0,
                       w.st));
  HIPTRY(launch_fill(w.z, Tp, 0.0, w.st));
  HIPTRY(launch_fill(w.q, Tp, 0.0, w.st));
  HIPTRY(launch_fill(w.AE, 3 * Tp, 0.0, w.st));
  HIPTRY(launch_fill(w.s_t, Tp, 0.0, w.st));
  return YAND_OK;
}

int ensure_bdiag(Work& w, const Data& D);

int ensure_thin(Work& w, const Data& D) {
  if (w.tG) return YAND_OK;
  w.tld = round_up(D.T, 128);
  w.tK = thin_splits(D.T);
  const size_t mm = (size_t)w.tld * w.tld * sizeof(double);
  TRY(alloc((void**)&w.tGp, mm * w.tK));
  TRY(alloc((void**)&w.tG, mm));
  TRY(alloc((void**)&w.tC, mm));
  TRY(alloc((void**)&w.tX, mm));
  return ensure_bdiag(w, D);
}

// bdiag and its partial rows (shared by the T < n and the probe routes)
int ensure_bdiag(Work& w, const Data& D) {
  if (!w.bdiag) TRY(alloc((void**)&w.bdiag, (size_t)D.lda * sizeof(double)));
  if (!w.tpart) {
    const int64_t tld = round_up(D.T, 128);
    const int64_t ldp = D.lda > tld ? D.lda : tld;
    TRY(alloc((void**)&w.tpart,
              (size_t)thin_part_rows(D.T) * ldp * sizeof(double)));
  }
  return YAND_OK;
}

int ensure_probe(Work& w, const Data& D) {
  if (w.pXi) return YAND_OK;
  TRY(ensure_bdiag(w, D));
  int sv = 1, sz = 1;
  block_splits(D.Tp, D.lda, &sv, &sz);
  const size_t tb = (size_t)D.Tp * kBlockWidth * sizeof(double);
  const size_t nb = (size_t)D.lda * kBlockWidth * sizeof(double);
  TRY(alloc((void**)&w.pXi, tb));
  TRY(alloc((void**)&w.pZ, tb));
  TRY(alloc((void**)&w.pZp, tb * sv));
  TRY(alloc((void**)&w.pYp, nb * sz));
  double** vecs[] = {&w.pU, &w.pY, &w.pR, &w.pW, &w.pP, &w.pHP, &w.pAP};
  for (double** v : vecs) TRY(alloc((void**)v, nb));
  TRY(alloc((void**)&w.pcs, (size_t)8 * kBlockWidth * sizeof(double)));
  TRY(alloc((void**)&w.pflags, 160 * sizeof(int)));
  return YAND_OK;
}

int ensure_dense(Work& w, const Data& D) {
  if (w.B) return YAND_OK;
  const size_t nn = (size_t)D.lda * D.lda * sizeof(double);
  TRY(alloc((void**)&w.B, nn));
  TRY(alloc((void**)&w.M, nn));
  TRY(alloc((void**)&w.X, nn));
  TRY(alloc((void**)&w.rn, (size_t)D.nt * D.Tp * sizeof(double)));
  if (D.precision != YAND_FP64) {
    // FP32: one rounded copy; BF16: high and low parts (4 bytes either way)
    TRY(alloc(&w.SAt, (size_t)D.lda * D.Tp * 4));
    TRY(alloc(&w.Xl, (size_t)D.lda * D.lda * 4));
  }
  return YAND_OK;
}

// Workspace of the balanced SYRK for `lanes` lanes (counters cleared once
// here; every launch leaves them at zero).
int alloc_syrk_ws(const Data& D, int lanes, hipStream_t st, double** ws,
                  int** cnt) {
  const size_t per = (size_t)std::max(D.syrk_nslots, 1) * kTile * kTile;
  const size_t cn = ((size_t)D.syrk_ntile2 + 1) / 2 * 2;
  TRY(alloc((void**)ws, per * lanes * sizeof(double)));
  TRY(alloc((void**)cnt, cn * lanes * sizeof(int)));
  HIPTRY(launch_fill((double*)*cnt, (int64_t)(cn * lanes / 2), 0.0, st));
  return YAND_OK;
}

int ensure_syrk_ws(Work& w, const Data& D) {
  if (!D.syrk_plan || w.syrk_ws) return YAND_OK;
  return alloc_syrk_ws(D, 1, w.st, &w.syrk_ws, &w.syrk_cnt);
}

SyrkSplit syrk_split(const Data& D, double* ws, int* cnt, int lanes_stride) {
  SyrkSplit p;
  if (!D.syrk_plan || !ws) return p;
  p.order = D.syrk_order;
  p.plan = D.syrk_plan;
  p.slots = D.syrk_wgs;
  p.rounds = D.syrk_rounds;
  p.ntile2 = D.syrk_ntile2;
  p.npieces = D.syrk_npieces;
  p.nslots = D.syrk_nslots;
  p.ws = ws;
  p.cnt = cnt;
  if (lanes_stride) {
    p.ws_lane = (int64_t)std::max(D.syrk_nslots, 1) * kTile * kTile;
    p.cnt_lane = ((int64_t)D.syrk_ntile2 + 1) / 2 * 2;
  }
  return p;
}

int sync_scalars(Work& w) {
  HIPTRY(hipMemcpyAsync(&w.hs, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost,
                        w.st));
  HIPTRY(hipStreamSynchronize(w.st));
  return YAND_OK;
}

// ----------------------------------------------------------- pipeline ----

PassArgs pass_args(const Data& D, const Work& w, const double c[4]) {
  PassArgs a{};
  a.A = D.A;
  a.lda = D.lda;
  a.Tp = D.Tp;
  a.n = D.n;
  a.part = w.part;
  a.psums = w.psums;
  a.c = c ? to_coef(c) : Coef{0, 0, 0, 0};
  a.invT = 1.0 / (double)D.T;
  a.skip = nullptr;
  return a;
}

int run_pass(const Data& D, Work& w, PassKind kind, const PassArgs& a,
             int* nwg, const char* name) {
  PassArgs b = a;
  b.groups = D.pass_groups[(int)kind];
  b.rows = D.pass_rows[(int)kind];
  HIPTRY(timed(w, name, [&] {
    return launch_pass(D.precision, kind, b, w.st, nwg);
  }));
  return YAND_OK;
}

// Oracle pass at x: z, g, f and the moments (device scalars).
int oracle_at(const Data& D, Work& w, const double c[4], const double* x,
              bool with_grad, const int* skip = nullptr) {
  PassArgs a = pass_args(D, w, c);
  a.v = x;
  a.tout = w.z;
  a.skip = skip;
  int nwg = 0;
  TRY(run_pass(D, w, with_grad ? PassKind::Oracle : PassKind::Value, a, &nwg,
               "oracle_pass"));
  HIPTRY(launch_reduce_sums(w.psums, nwg, 3, w.sums, w.st, skip));
  HIPTRY(launch_dot(D.mu, x, D.n, &w.sc->mux, w.st));
  HIPTRY(launch_objective(w.sums, a.invT, to_coef(c), w.sc, w.st));
  if (with_grad)
    HIPTRY(launch_reduce_partials(w.part, nwg, D.lda, D.n, 1.0, -c[0], D.mu,
                                  w.g, w.st, skip));
  return YAND_OK;
}

int hvp_cached(const Data& D, Work& w, const double c[4], const double* v,
               double* hv, double* tout, const int* skip = nullptr) {
  PassArgs a = pass_args(D, w, c);
  a.v = v;
  a.zc = w.z;
  a.tout = tout;
  a.skip = skip;
  int nwg = 0;
  TRY(run_pass(D, w, PassKind::Hvp, a, &nwg, "hvp_pass"));
  HIPTRY(launch_reduce_partials(w.part, nwg, D.lda, D.n, 1.0, 0.0, nullptr, hv,
                                w.st, skip));
  return YAND_OK;
}

// Line-search sums along d at the cached z; coefficients (and the step when
// select) in the device scalars.  mu^T d must already be in sc->mud.
int line_at(const Data& D, Work& w, const double c[4], const double* d,
            int select, const int* skip) {
  PassArgs a = pass_args(D, w, c);
  a.v = d;
  a.zc = w.z;
  a.tout = w.wv;
  a.skip = skip;
  int nwg = 0;
  TRY(run_pass(D, w, PassKind::Line, a, &nwg, "line_pass"));
  HIPTRY(launch_reduce_sums(w.psums, nwg, 9, w.sums, w.st, skip));
  HIPTRY(launch_coef_step(w.sums, a.invT, to_coef(c), select, w.sc, w.st,
                          skip));
  return YAND_OK;
}

__global__ void psi2_weight_kernel(const double* __restrict__ z, int64_t Tp,
                                   Coef c, double invT, double* __restrict__ s,
                                   const int* skip) {
  if (skip && *skip) return;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < Tp) s[t] = d2psi(c, z[t]) * invT;
}

__global__ void set_lambda_kernel(DevScalars* sc, double lam) {
  if (threadIdx.x == 0) {
    sc->lambda = lam;
    sc->fail = 0;
  }
}

struct DirOpts {
  int solver = YAND_SOLVER_DIRECT;
  double reg = 0.0;
  double krylov_tol = 1e-3;
  int krylov_maxit = 15;
  double tau = 1e-8;
  int simplex = 0;
  // simplex boundary block (budget hull only): face continuation and the
  // projected trial step with nominal step eta
  bool faces = false;
  double eta = 0.0;
  int select = 1;  // step rule for line_at: 1 exact quartic, 2 Armijo
  // FP32 / BF16 storage: products of the exact trace in FP64 instead of on
  // the storage precision's matrix cores
  bool dense64 = false;
  // PCG solver: probe estimate of the trace with `probes` sign vectors from
  // block `draw` of the counter stream keyed by `seed`
  bool probe = false;
  int probes = 64;
  uint64_t seed = 0, draw = 0;
};

const double* face_mask(const Work& w, const DirOpts& o) {
  return o.faces ? w.mask : nullptr;
}

// Line search of the iteration after the direction (and, on a face, the
// first part of the boundary block).  On a face: the projected segment left
// in w.ptmp is line-searched first (skipped unless it is a descent
// candidate) and taken when its step is usable; otherwise the raw
// direction's line search runs (skipped once the segment is taken).
int step_line(const Data& D, Work& w, const double c[4], const DirOpts& o,
              const int* skip) {
  if (!o.faces) return line_at(D, w, c, w.d, o.select, skip);
  PassArgs a = pass_args(D, w, c);
  a.v = w.ptmp;
  a.zc = w.z;
  a.tout = w.wv;
  a.skip = &w.sc->segskip;
  int nwg = 0;
  TRY(run_pass(D, w, PassKind::Line, a, &nwg, "line_pass"));
  HIPTRY(launch_reduce_sums(w.psums, nwg, 9, w.sums, w.st, &w.sc->segskip));
  HIPTRY(launch_segment_decide(w.sums, a.invT, to_coef(c), o.select, w.x,
                               D.n, o.tau, w.d, w.ptmp, w.mask, w.hold, w.sc,
                               w.st));
  return line_at(D, w, c, w.d, o.select, &w.sc->lsskip);
}

// Regularisation escalations (lambda <- max(10 lambda, 1e-12 scale)) before
// a direction gives up as indefinite: 16 reach 1e3 times the mean tangent
// curvature, so an indefinite tangent Hessian outside the convexity
// certificate still yields a (gradient-like) descent direction.
constexpr int kMaxEscalations = 16;

struct DirStats {
  int cg = 0;
  int escalations = 0;
  int probe_cg = 0;  // CG iterations of the probe solves (all columns)
  bool thin = false;  // the exact trace came from the T < n push-through
};

// Direction, first part: nu-projection (Aν), B = A^T diag(psi''/T) A,
// W_E = B E and the scales gamma, lambda.  Needs z, g and E[p0] = nu.
// A nu and the weights s_t = psi''(z_t) / T of the SYRK.
int dir_front_pre(const Data& D, Work& w, const double c[4], int p0,
                  const int* skip) {
  const int64_t n = D.n, Tp = D.Tp;
  {
    PassArgs a = pass_args(D, w, c);
    a.v = w.E + (int64_t)p0 * n;
    a.tout = w.AE + (int64_t)p0 * Tp;
    a.skip = skip;
    int nwg;
    TRY(run_pass(D, w, PassKind::Dot, a, &nwg, "dot_pass"));
  }
  hipLaunchKernelGGL(psi2_weight_kernel, dim3((unsigned)((Tp + 255) / 256)),
                     dim3(256), 0, w.st, w.z, Tp, to_coef(c),
                     1.0 / (double)D.T, w.s_t, skip);
  return YAND_OK;
}

// W_E = B E and the scales gamma, lambda (after the SYRK).
int dir_front_post(const Data& D, Work& w, int p0, const DirOpts& o,
                   const int* skip) {
  const int64_t n = D.n, np = D.lda;
  const int p = p0 + 1;
  HIPTRY(launch_symm_multi(w.B, np, n, w.E, p, w.W, w.st, skip));
  HIPTRY(launch_trace_scale(w.B, np, n, w.E, w.W, p, o.reg, w.sc, w.st,
                            face_mask(w, o)));
  return YAND_OK;
}

int dir_front(const Data& D, Work& w, const double c[4], int p0,
              const DirOpts& o, const int* skip) {
  TRY(ensure_dense(w, D));
  const int64_t np = D.lda, Tp = D.Tp;
  TRY(dir_front_pre(D, w, c, p0, skip));
  if (D.precision != YAND_FP64 && !o.dense64)
    HIPTRY(timed(w, "syrk", [&] {
      return launch_syrk_lp(D.precision, D.At, w.SAt, np, Tp, w.s_t, w.B,
                            w.st, skip, D.syrk_order, D.syrk_slots);
    }));
  else {
    TRY(ensure_syrk_ws(w, D));
    const SyrkSplit sp = syrk_split(D, w.syrk_ws, w.syrk_cnt, 0);
    HIPTRY(timed(w, "syrk", [&] {
      return launch_syrk(D.precision, D.A, D.lda, Tp, w.s_t, w.B, w.st, skip,
                         Lanes{}, 1, D.syrk_order, D.syrk_slots, &sp);
    }));
  }
  return dir_front_post(D, w, p0, o, skip);
}

// Projection of B into M and the factorisation M = L L^T, X = L^-1.
int dir_factor(const Data& D, Work& w, int p0, const int* skip,
               const double* mask = nullptr) {
  const int64_t n = D.n, np = D.lda;
  HIPTRY(launch_project(w.B, w.M, np, n, np, w.E, w.W, p0 + 1, w.sc, w.st,
                        mask));
  HIPTRY(timed(w, "potrf_trtri", [&] {
    return launch_potrf_trtri(w.M, w.X, np, &w.sc->fail, w.st, skip,
                              D.chol_group, Lanes{}, 1, w.solo,
                              D.chol_step_tm, D.chol_band);
  }));
  return YAND_OK;
}

int dir_trace_post(const Data& D, Work& w, const double c[4], int p0,
                   const int* skip, const double* mask);

// Exact trace q, third-order back-projection t3 and r = P_S(B nu - |G|/(m+1) t3).
int dir_trace(const Data& D, Work& w, const double c[4], int p0,
              const DirOpts& o, const int* skip,
              const double* mask = nullptr) {
  const int64_t n = D.n, np = D.lda, Tp = D.Tp;
  const int p = p0 + 1;
  if (D.precision != YAND_FP64 && !o.dense64)
    HIPTRY(timed(w, "trace_gemm", [&] {
      return launch_trace_lp(D.precision, D.A, D.lda, Tp, w.X, np, w.Xl, w.rn,
                             w.st, skip);
    }));
  else
    HIPTRY(timed(w, "trace_gemm", [&] {
      return launch_trace_gemm(D.precision, D.A, D.lda, Tp, w.X, np, w.rn,
                               w.st, skip);
    }));
  return dir_trace_post(D, w, c, p0, skip, mask);
}

// After the trace GEMM: the frame's A e_a, q, the third-order pass and the
// right-hand side r = P_S(B nu - |G|/(m+1) t3).
int dir_trace_post(const Data& D, Work& w, const double c[4], int p0,
                   const int* skip, const double* mask) {
  const int64_t n = D.n, Tp = D.Tp;
  const int p = p0 + 1;
  if (mask) {
    // the face's frame column E[0] = mask / sqrt(nfree): A E[0] afresh
    PassArgs a = pass_args(D, w, c);
    a.v = w.E;
    a.tout = w.AE;
    a.skip = skip;
    int nwg;
    TRY(run_pass(D, w, PassKind::Dot, a, &nwg, "dot_pass"));
  } else {
    HIPTRY(launch_copy(w.AE, D.AEfix, (int64_t)p0 * Tp, w.st, skip));
  }
  HIPTRY(launch_trace_weight(w.rn, (int)D.nt, Tp, w.AE, p, w.sc, w.q, w.st));
  {
    PassArgs a = pass_args(D, w, c);
    a.zc = w.z;
    a.q = w.q;
    a.skip = skip;
    int nwg;
    TRY(run_pass(D, w, PassKind::Third, a, &nwg, "third_pass"));
    HIPTRY(launch_reduce_partials(w.part, nwg, D.lda, n, 1.0, 0.0, nullptr,
                                  w.t3, w.st, skip));
  }
  const double mp1 = mask ? -1.0 : (double)(n - p0 + 1);
  HIPTRY(launch_rhs(w.W + (int64_t)p0 * n, w.t3, w.E, p, n, mp1, w.sc, w.r,
                    w.st, mask));
  return YAND_OK;
}

// d = K r - nu with K = P_S M^-1 P_S = P_S X^T X P_S (direct solve).
int dir_direct_solve(const Data& D, Work& w, int p0, const double* x,
                     const DirOpts& o, double* d, const int* skip) {
  const int64_t n = D.n, np = D.lda;
  HIPTRY(launch_trmv(w.X, np, n, w.r, w.y, w.trpart, false, w.st, skip));
  HIPTRY(launch_trmv(w.X, np, n, w.y, w.y2, w.trpart, true, w.st, skip));
  HIPTRY(launch_direction(w.y2, w.E, p0 + 1, n, x, D.mu, o.tau, o.simplex, d,
                          w.sc, w.st, face_mask(w, o)));
  if (o.faces)
    HIPTRY(launch_boundary(x, w.g, D.mu, n, o.tau, o.eta, d, w.ptmp, w.mask,
                           w.hold, w.sc, w.st));
  return YAND_OK;
}

// ------------------------------------------------------ projected PCG ----
constexpr int PT = 1024;
template <int K>
__device__ void bsum(double (&v)[K], double* sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) sh[k * 16 + wv] = s;
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

// Jacobi preconditioner diag(B) + lambda; the diagonal of B sits at
// bd[j * bs] (bs = ld + 1 for the dense B, 1 for a separate vector).
__device__ double precond_diag(const double* bd, int64_t bs, int64_t j,
                               double lam) {
  double dj = bd[j * bs] + lam;
  return dj > 0.0 ? dj : 1.0;
}

// Projected PCG on P_S (H + lambda) P_S s = r (s in S) with the Jacobi
// preconditioner P_S diag(B + lambda)^-1 P_S; r already in S.  Inner
// products with a projected vector come from the unprojected one and its
// frame components, x^T P_S y = x^T y - sum_a (e_a^T x)(e_a^T y) (with
// P_S = diag(mask) - E E^T and x, y zero off the face), so each CG step
// needs two block reductions.  Taking x^T y alone would be exact for x in S
// but lets the rounding residue of the residual outside S into the products
// once the residual itself is small.
// Operands of one projected PCG solve: right-hand side r, the diagonal of
// B at bd[j * bs], the frame E (p rows of n), iterate s, residual res,
// search direction pv, preconditioned residual u, scratch Ap, the product
// hp = B pv of the current step, the lane's scalars and face mask.
struct PcgLane {
  const double* r;
  const double* bd;
  int64_t bs;
  const double* E;
  int p;
  int64_t n;
  double *s, *res, *pv, *u, *Ap;
  const double* hp;
  DevScalars* sc;
  const double* mask;
};

// A lane already done at this iteration takes no step (cgdone, 0 steps).
__device__ void pcg_init_body(const PcgLane& L, double* sh) {
  const int tid = threadIdx.x;
  DevScalars* sc = L.sc;
  if (sc->done) {
    if (tid == 0) {
      sc->cgit = 0;
      sc->cgdone = 1;
    }
    return;
  }
  const double lam = sc->lambda;
  const int p = L.p;
  const int64_t n = L.n;
  const double *r = L.r, *E = L.E, *mask = L.mask;
  // E^T u (p), E^T r (p), r^T u, r^T r
  double dt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t j = tid; j < n; j += PT) {
    L.s[j] = 0.0;
    const double rj = r[j];
    const double uj =
        (mask ? mask[j] : 1.0) * rj / precond_diag(L.bd, L.bs, j, lam);
    L.u[j] = uj;
    for (int a = 0; a < p; ++a) {
      dt[a] += E[a * n + j] * uj;
      dt[3 + a] += E[a * n + j] * rj;
    }
    dt[6] += rj * uj;
    dt[7] += rj * rj;
  }
  bsum(dt, sh);
  double rz = dt[6];
  const double rr = dt[7];
  for (int a = 0; a < p; ++a) rz -= dt[3 + a] * dt[a];
  for (int64_t j = tid; j < n; j += PT) {
    double uj = L.u[j];
    for (int a = 0; a < p; ++a) uj -= dt[a] * E[a * n + j];
    L.u[j] = uj;
    L.pv[j] = uj;
    L.res[j] = r[j];
  }
  if (tid == 0) {
    sc->aux[0] = rz;
    sc->aux[1] = rr;
    sc->aux[2] = rr;
    sc->aux[3] = 0.0;
    sc->cgit = 0;
    sc->cgdone = rr > 0.0 ? 0 : 1;
  }
}

__device__ void pcg_update_body(const PcgLane& L, double tol, double* sh) {
  DevScalars* sc = L.sc;
  if (sc->cgdone) return;
  const int tid = threadIdx.x;
  const double lam = sc->lambda;
  const int p = L.p;
  const int64_t n = L.n;
  const double *E = L.E, *mask = L.mask, *Hp = L.hp;
  double *pv = L.pv, *Ap = L.Ap;
  // E^T Ap (p), E^T pv (p), pv^T Ap
  double d1[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t j = tid; j < n; j += PT) {
    const double a = (mask ? mask[j] : 1.0) * (Hp[j] + lam * pv[j]);
    Ap[j] = a;
    for (int k = 0; k < p; ++k) {
      d1[k] += E[k * n + j] * a;
      d1[3 + k] += E[k * n + j] * pv[j];
    }
    d1[6] += pv[j] * a;
  }
  bsum(d1, sh);
  double pap = d1[6];
  for (int k = 0; k < p; ++k) pap -= d1[3 + k] * d1[k];
  const double rz = sc->aux[0];
  const double al = pap > 0.0 ? rz / pap : 0.0;
  // E^T u (p), E^T res (p), res^T u, res^T res (new residual)
  double d2[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t j = tid; j < n; j += PT) {
    double a = Ap[j];
    for (int k = 0; k < p; ++k) a -= d1[k] * E[k * n + j];
    L.s[j] += al * pv[j];
    const double rj = L.res[j] - al * a;
    L.res[j] = rj;
    const double uj =
        (mask ? mask[j] : 1.0) * rj / precond_diag(L.bd, L.bs, j, lam);
    L.u[j] = uj;
    for (int k = 0; k < p; ++k) {
      d2[k] += E[k * n + j] * uj;
      d2[3 + k] += E[k * n + j] * rj;
    }
    d2[6] += rj * uj;
    d2[7] += rj * rj;
  }
  bsum(d2, sh);
  double rzn = d2[6];
  const double rr = d2[7];
  for (int k = 0; k < p; ++k) rzn -= d2[3 + k] * d2[k];
  const double beta = rz > 0.0 ? rzn / rz : 0.0;
  for (int64_t j = tid; j < n; j += PT) {
    double uj = L.u[j];
    for (int k = 0; k < p; ++k) uj -= d2[k] * E[k * n + j];
    L.u[j] = uj;
    pv[j] = uj + beta * pv[j];
  }
  if (tid == 0) {
    sc->aux[0] = rzn;
    sc->aux[1] = rr;
    if (!(pap > 0.0)) sc->aux[3] = 1.0;  // curvature breakdown
    sc->cgit += 1;
    // stop on |res| <= tol |r0| or a breakdown; later iterations are skipped
    if (sqrt(rr) <= tol * sqrt(sc->aux[2]) || !(pap > 0.0))
      sc->cgdone = 1;
  }
}

__global__ void __launch_bounds__(PT) pcg_init_kernel(PcgLane L) {
  __shared__ double sh[8 * 16];
  pcg_init_body(L, sh);
}

__global__ void __launch_bounds__(PT) pcg_update_kernel(PcgLane L,
                                                        double tol) {
  __shared__ double sh[8 * 16];
  pcg_update_body(L, tol, sh);
}

// Lane-batched forms: workgroup b runs lane b's solve.
__global__ void __launch_bounds__(PT)
pcg_init_lanes_kernel(const PcgLane* __restrict__ Ls) {
  __shared__ double sh[8 * 16];
  pcg_init_body(Ls[blockIdx.x], sh);
}

__global__ void __launch_bounds__(PT)
pcg_update_lanes_kernel(const PcgLane* __restrict__ Ls, double tol) {
  __shared__ double sh[8 * 16];
  pcg_update_body(Ls[blockIdx.x], tol, sh);
}

// *flag = 1 once every lane's solve has stopped (the block products of later
// steps are skipped).
__global__ void pcg_alldone_kernel(const PcgLane* __restrict__ Ls, int nl,
                                   int* flag) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int l = threadIdx.x; l < nl; l += blockDim.x)
    if (!Ls[l].sc->cgdone) atomicOr(&any, 1);
  __syncthreads();
  if (threadIdx.x == 0) *flag = any ? 0 : 1;
}

PcgLane pcg_lane(const Data& D, Work& w, int p0, const DirOpts& o,
                 const double* bd, int64_t bs) {
  PcgLane L;
  L.r = w.r;
  L.bd = bd;
  L.bs = bs;
  L.E = w.E;
  L.p = p0 + 1;
  L.n = D.n;
  L.s = w.pcg_s;
  L.res = w.pcg_res;
  L.pv = w.pcg_p;
  L.u = w.pcg_u;
  L.Ap = w.y;
  L.hp = w.hv;
  L.sc = w.sc;
  L.mask = face_mask(w, o);
  return L;
}

// The direction from the tangent solve s (and the boundary block's first
// part on a face).
int dir_from_solve(const Data& D, Work& w, int p0, const double* x,
                   const DirOpts& o, double* d) {
  HIPTRY(launch_direction(w.pcg_s, w.E, p0 + 1, D.n, x, D.mu, o.tau,
                          o.simplex, d, w.sc, w.st, face_mask(w, o)));
  if (o.faces)
    HIPTRY(launch_boundary(x, w.g, D.mu, D.n, o.tau, o.eta, d, w.ptmp, w.mask,
                           w.hold, w.sc, w.st));
  return YAND_OK;
}

// Projected PCG for the tangent system, krylov_maxit steps enqueued without
// host synchronisation: the update kernel raises cgdone at convergence or
// breakdown, and every later HVP pass and update returns at once.  The step
// count is left in sc->cgit.
int dir_pcg_enqueue(const Data& D, Work& w, const double c[4], int p0,
                    const double* x, const DirOpts& o, double* d,
                    const double* bd, int64_t bs) {
  const PcgLane L = pcg_lane(D, w, p0, o, bd, bs);
  hipLaunchKernelGGL(pcg_init_kernel, dim3(1), dim3(PT), 0, w.st, L);
  for (int it = 0; it < o.krylov_maxit; ++it) {
    TRY(hvp_cached(D, w, c, w.pcg_p, w.hv, nullptr, &w.sc->cgdone));
    hipLaunchKernelGGL(pcg_update_kernel, dim3(1), dim3(PT), 0, w.st, L,
                       o.krylov_tol);
  }
  return dir_from_solve(D, w, p0, x, o, d);
}

int dir_pcg_solve(const Data& D, Work& w, const double c[4], int p0,
                  const double* x, const DirOpts& o, double* d,
                  DirStats* stats, const double* bd, int64_t bs) {
  TRY(dir_pcg_enqueue(D, w, c, p0, x, o, d, bd, bs));
  TRY(sync_scalars(w));
  if (stats) stats->cg += w.hs.cgit;
  return YAND_OK;
}

// Exact trace by the T < n push-through (thin.hip): the frame's A e_a, the
// Gram matrix G of the rows of A P_S, then either (S > 0) C = S^1/2 G S^1/2
// + lambda I, its factor and inverse, or (some s_t < 0) the signed
// factorisation of W = lambda S^-1 + G, whose failure raises lambda as the
// dense route's does; q, the third-order pass and the right-hand side; also
// diag(B) for the preconditioner and W[p0] = B nu from one HVP pass.
// Returns with *ok = false (and the fail flag clear) when the identity does
// not apply at this iterate (some psi''(z_t) = 0) or C's factorisation
// fails.
int dir_thin(const Data& D, Work& w, const double c[4], int p0,
             const DirOpts& o, bool* ok) {
  TRY(ensure_thin(w, D));
  const int64_t n = D.n, Tp = D.Tp;
  const int p = p0 + 1;
  const double* mask = face_mask(w, o);
  hipLaunchKernelGGL(psi2_weight_kernel, dim3((unsigned)((Tp + 255) / 256)),
                     dim3(256), 0, w.st, w.z, Tp, to_coef(c),
                     1.0 / (double)D.T, w.s_t, nullptr);
  if (mask) {
    PassArgs a = pass_args(D, w, c);
    a.v = w.E;
    a.tout = w.AE;
    int nwg;
    TRY(run_pass(D, w, PassKind::Dot, a, &nwg, "dot_pass"));
  } else {
    HIPTRY(launch_copy(w.AE, D.AEfix, (int64_t)p0 * Tp, w.st));
  }
  // W[p0] = B nu and A nu in one HVP pass
  TRY(hvp_cached(D, w, c, w.E + (int64_t)p0 * n, w.W + (int64_t)p0 * n,
                 w.AE + (int64_t)p0 * Tp));
  HIPTRY(timed(w, "thin_gram", [&] {
    return launch_thin_gram(D.precision, D.A, D.lda, D.T, n, mask, w.tK,
                            w.tGp, w.tld, w.AE, Tp, p, w.tG, w.st);
  }));
  HIPTRY(launch_thin_factor_input(w.tG, w.tld, D.T, w.s_t, w.AE, Tp, p, n,
                                  o.reg, mask, w.sc, w.tC, w.st));
  TRY(sync_scalars(w));
  auto not_applicable = [&]() -> int {
    *ok = false;
    hipLaunchKernelGGL(set_lambda_kernel, dim3(1), dim3(64), 0, w.st, w.sc,
                       0.0);
    return YAND_OK;
  };
  if (w.hs.ptbad) return not_applicable();
  if (w.hs.sneg == 0) {
    HIPTRY(timed(w, "thin_potrf_trtri", [&] {
      return launch_potrf_trtri(w.tC, w.tX, w.tld, &w.sc->fail, w.st, nullptr,
                                0);
    }));
    TRY(sync_scalars(w));
    if (w.hs.fail) return not_applicable();
    HIPTRY(launch_thin_q(w.tX, w.tld, D.T, Tp, w.s_t, w.sc, w.tpart, w.q,
                         w.st));
  } else {
    if (!w.tW)
      TRY(alloc((void**)&w.tW,
                (size_t)thin_indef_doubles(D.T) * sizeof(double)));
    const int np_ = (int)D.T - w.hs.sneg;
    for (int attempt = 0;; ++attempt) {
      HIPTRY(timed(w, "thin_indef_factor", [&] {
        return launch_thin_indef_factor(w.tG, w.tld, D.T, w.s_t, np_, 0, w.sc,
                                        w.tW, w.st);
      }));
      TRY(sync_scalars(w));
      if (!w.hs.fail) break;
      if (attempt >= kMaxEscalations) return YAND_ERR_INDEFINITE;
      const double lam = std::max(10.0 * w.hs.lambda,
                                  1e-12 * w.hs.tang_scale);
      hipLaunchKernelGGL(set_lambda_kernel, dim3(1), dim3(64), 0, w.st, w.sc,
                         lam);
    }
    HIPTRY(launch_thin_indef_q(D.T, Tp, w.s_t, np_, w.sc, w.tW, w.q, w.st));
  }
  *ok = true;
  {
    PassArgs a = pass_args(D, w, c);
    a.zc = w.z;
    a.q = w.q;
    int nwg;
    TRY(run_pass(D, w, PassKind::Third, a, &nwg, "third_pass"));
    HIPTRY(launch_reduce_partials(w.part, nwg, D.lda, n, 1.0, 0.0, nullptr,
                                  w.t3, w.st));
  }
  const double mp1 = mask ? -1.0 : (double)(n - p0 + 1);
  HIPTRY(launch_rhs(w.W + (int64_t)p0 * n, w.t3, w.E, p, n, mp1, w.sc, w.r,
                    w.st, mask));
  HIPTRY(launch_bdiag(D.precision, D.A, D.lda, D.T, n, w.s_t, w.tpart,
                      w.bdiag, w.st));
  return YAND_OK;
}

// Probe estimate of the trace (probe.hip): frame products A e_a and one HVP
// pass (B nu, A nu), the Jacobi diagonal diag(B) and lambda, then k sign
// vectors Xi, U = A^T Xi, k projected PCG solves side by side whose Hessian
// products are block passes over A, Q = A Y, q_t = k^-1 sum_j Xi_tj Q_tj,
// the third-order pass and the right-hand side of the tangent solve.
int dir_probe(const Data& D, Work& w, const double c[4], int p0,
              const DirOpts& o, DirStats* stats) {
  TRY(ensure_probe(w, D));
  const int64_t n = D.n, Tp = D.Tp, ld = D.lda;
  const int p = p0 + 1;
  const double* mask = face_mask(w, o);
  hipLaunchKernelGGL(psi2_weight_kernel, dim3((unsigned)((Tp + 255) / 256)),
                     dim3(256), 0, w.st, w.z, Tp, to_coef(c),
                     1.0 / (double)D.T, w.s_t, nullptr);
  if (mask) {
    PassArgs a = pass_args(D, w, c);
    a.v = w.E;
    a.tout = w.AE;
    int nwg;
    TRY(run_pass(D, w, PassKind::Dot, a, &nwg, "dot_pass"));
  } else {
    HIPTRY(launch_copy(w.AE, D.AEfix, (int64_t)p0 * Tp, w.st));
  }
  TRY(hvp_cached(D, w, c, w.E + (int64_t)p0 * n, w.W + (int64_t)p0 * n,
                 w.AE + (int64_t)p0 * Tp));
  HIPTRY(launch_bdiag(D.precision, D.A, D.lda, D.T, n, w.s_t, w.tpart,
                      w.bdiag, w.st));
  HIPTRY(launch_probe_scale(w.bdiag, n, w.s_t, w.AE, D.T, Tp, p, o.reg, mask,
                            w.sc, w.st));
  const int k = o.probes;
  HIPTRY(launch_rademacher(o.seed, o.draw, D.T, Tp, k, w.pXi, w.st));
  HIPTRY(timed(w, "probe_block", [&] {
    return launch_block_atz(D.precision, D.A, ld, Tp, w.pXi, nullptr, w.pYp,
                            w.pU, w.st);
  }));
  HIPTRY(launch_bpcg_init(w.pU, w.bdiag, w.E, p, n, ld, k, w.pY, w.pR, w.pW,
                          w.pP, w.pcs, w.pflags, w.sc, mask, w.st));
  const int* alldone = w.pflags;
  for (int it = 0; it < o.krylov_maxit; ++it) {
    HIPTRY(timed(w, "probe_block", [&] {
      return launch_block_av(D.precision, D.A, ld, Tp, w.pP, w.pZp, w.pZ,
                             w.st, alldone);
    }));
    HIPTRY(timed(w, "probe_block", [&] {
      return launch_block_atz(D.precision, D.A, ld, Tp, w.pZ, w.s_t, w.pYp,
                              w.pHP, w.st, alldone);
    }));
    HIPTRY(launch_bpcg_update(w.pHP, w.bdiag, w.E, p, n, ld, w.pY, w.pR, w.pW,
                              w.pP, w.pAP, w.pcs, w.pflags, w.sc, mask,
                              o.krylov_tol, w.st));
  }
  HIPTRY(timed(w, "probe_block", [&] {
    return launch_block_av(D.precision, D.A, ld, Tp, w.pY, w.pZp, w.pZ, w.st);
  }));
  HIPTRY(launch_probe_q(w.pXi, w.pZ, D.T, Tp, k, w.q, w.st));
  if (stats) {
    int tot = 0;
    HIPTRY(hipMemcpyAsync(&tot, w.pflags + 129, sizeof(int),
                          hipMemcpyDeviceToHost, w.st));
    HIPTRY(hipStreamSynchronize(w.st));
    stats->probe_cg += tot;
  }
  {
    PassArgs a = pass_args(D, w, c);
    a.zc = w.z;
    a.q = w.q;
    int nwg;
    TRY(run_pass(D, w, PassKind::Third, a, &nwg, "third_pass"));
    HIPTRY(launch_reduce_partials(w.part, nwg, D.lda, n, 1.0, 0.0, nullptr,
                                  w.t3, w.st));
  }
  const double mp1 = mask ? -1.0 : (double)(n - p0 + 1);
  HIPTRY(launch_rhs(w.W + (int64_t)p0 * n, w.t3, w.E, p, n, mp1, w.sc, w.r,
                    w.st, mask));
  return YAND_OK;
}

// Eager direction with regularisation escalation (host reads the Cholesky
// flag) and either solver.  The oracle pass and the gradient projection must
// already have run at x with the done flag clear.  The PCG configuration
// with 2 T <= n takes the push-through trace when it applies.
int direction_eager(const Data& D, Work& w, const double c[4], int p0,
                    const double* x, const DirOpts& o, double* d,
                    DirStats* stats) {
  if (o.solver == YAND_SOLVER_PCG && o.probe) {
    TRY(dir_probe(D, w, c, p0, o, stats));
    return dir_pcg_solve(D, w, c, p0, x, o, d, stats, w.bdiag, 1);
  }
  if (o.solver == YAND_SOLVER_PCG && o.reg > 0.0 && 2 * D.T <= D.n) {
    bool ok = false;
    TRY(dir_thin(D, w, c, p0, o, &ok));
    if (ok) {
      if (stats) stats->thin = true;
      return dir_pcg_solve(D, w, c, p0, x, o, d, stats, w.bdiag, 1);
    }
  }
  TRY(dir_front(D, w, c, p0, o, nullptr));
  for (int attempt = 0;; ++attempt) {
    TRY(dir_factor(D, w, p0, nullptr, face_mask(w, o)));
    TRY(sync_scalars(w));
    if (!w.hs.fail) break;
    if (attempt >= kMaxEscalations) return YAND_ERR_INDEFINITE;
    const double lam = std::max(10.0 * w.hs.lambda, 1e-12 * w.hs.tang_scale);
    hipLaunchKernelGGL(set_lambda_kernel, dim3(1), dim3(64), 0, w.st, w.sc,
                       lam);
    if (stats) stats->escalations++;
  }
  TRY(dir_trace(D, w, c, p0, o, nullptr, face_mask(w, o)));
  if (o.solver == YAND_SOLVER_DIRECT)
    return dir_direct_solve(D, w, p0, x, o, d, nullptr);
  return dir_pcg_solve(D, w, c, p0, x, o, d, stats, w.B, D.lda + 1);
}

// One outer iteration of the direct configuration, enqueued with no host
// synchronisation: oracle, stationarity (sets done when |G| <= eps), exact-
// trace direction, line search, step, update.
// After the oracle pass at w.x: the face of Delta(tau) (boundary block),
// the projected gradient with the done test, and on the simplex the
// projected-KKT residual, which also ends the run at or below eps.
int stationarity(const Data& D, Work& w, const DirOpts& o, int p0,
                 double eps) {
  if (o.faces)
    HIPTRY(launch_face(w.x, w.g, D.n, o.tau, w.E, w.mask, w.hold, w.sc,
                       w.st));
  HIPTRY(launch_grad_project(w.g, w.E, p0, D.n, w.sc, w.st, eps,
                             face_mask(w, o)));
  if (o.simplex)
    HIPTRY(launch_kkt(w.x, w.g, D.n, o.tau, eps, w.ptmp, w.sc, w.st));
  return YAND_OK;
}

int enqueue_iteration(const Data& D, Work& w, const double c[4], int p0,
                      const DirOpts& o, double eps) {
  const int* skip = &w.sc->done;
  TRY(oracle_at(D, w, c, w.x, true, &w.sc->frozen));
  TRY(stationarity(D, w, o, p0, eps));
  TRY(dir_front(D, w, c, p0, o, skip));
  TRY(dir_factor(D, w, p0, skip, face_mask(w, o)));
  TRY(dir_trace(D, w, c, p0, o, skip, face_mask(w, o)));
  if (o.solver == YAND_SOLVER_PCG)
    TRY(dir_pcg_enqueue(D, w, c, p0, w.x, o, w.d, w.B, D.lda + 1));
  else
    TRY(dir_direct_solve(D, w, p0, w.x, o, w.d, skip));
  TRY(step_line(D, w, c, o, skip));
  HIPTRY(launch_axpy(w.x, w.d, D.n, w.sc, w.st));
  return YAND_OK;
}

// Lanes advancing in lockstep on one stream (a frontier on one context):
// the SYRK, the factorisation with its inverse and the trace GEMM of all
// lanes run as single grouped launches (blockIdx.y = lane) over strided
// per-lane blocks, so the lanes' tiles fill the GPU together; the passes
// and vector kernels run per lane in between.  With the PCG configuration
// the lanes' tangent solves also run together: their search directions are
// the rows of one 64 x lda block P, so each CG step is one pair of block
// products over A for every lane, HP = (A^T diag(s_l) A P)^T, between
// lane-batched init and update kernels.
struct Group {
  int nl = 0;
  Lanes ls;
  double *s = nullptr, *B = nullptr, *M = nullptr, *X = nullptr,
         *rn = nullptr;
  int *skip = nullptr, *fail = nullptr;
  // PCG: P and HP (64 x lda), Z and ZS (Tp x 64), split partials, the lanes'
  // operands (device array) and the all-stopped flag
  double *P = nullptr, *HP = nullptr, *Z = nullptr, *ZS = nullptr,
         *Zp = nullptr, *Yp = nullptr;
  PcgLane* pl = nullptr;
  int* cgall = nullptr;
  // balanced SYRK workspace, one per lane
  double* syrk_ws = nullptr;
  int* syrk_cnt = nullptr;
};

struct LaneRef {
  const Data* D;
  Work* w;
  const double* c;
  int p0;
};

int enqueue_group(const std::vector<LaneRef>& lanes, const DirOpts& o,
                  double eps, const Group& G, hipStream_t st) {
  const Data& D = *lanes[0].D;
  const int64_t np = D.lda, Tp = D.Tp;
  for (const auto& L : lanes) {
    Work& w = *L.w;
    TRY(oracle_at(D, w, L.c, w.x, true, &w.sc->frozen));
    TRY(stationarity(D, w, o, L.p0, eps));
    TRY(dir_front_pre(D, w, L.c, L.p0, &w.sc->done));
  }
  const SyrkSplit sp = syrk_split(D, G.syrk_ws, G.syrk_cnt, 1);
  HIPTRY(launch_syrk(D.precision, D.A, D.lda, Tp, G.s, G.B, st, G.skip, G.ls,
                     G.nl, D.syrk_order, D.syrk_slots, &sp));
  for (const auto& L : lanes) {
    Work& w = *L.w;
    TRY(dir_front_post(D, w, L.p0, o, &w.sc->done));
    HIPTRY(launch_project(w.B, w.M, np, D.n, np, w.E, w.W, L.p0 + 1, w.sc,
                          w.st, face_mask(w, o)));
  }
  HIPTRY(launch_potrf_trtri(G.M, G.X, np, G.fail, st, G.skip, D.chol_group,
                            G.ls, G.nl, true, D.chol_step_tm, D.chol_band));
  HIPTRY(launch_trace_gemm(D.precision, D.A, D.lda, Tp, G.X, np, G.rn, st,
                           G.skip, G.ls, G.nl));
  for (const auto& L : lanes) {
    Work& w = *L.w;
    const int* skip = &w.sc->done;
    TRY(dir_trace_post(D, w, L.c, L.p0, skip, face_mask(w, o)));
    if (o.solver != YAND_SOLVER_PCG)
      TRY(dir_direct_solve(D, w, L.p0, w.x, o, w.d, skip));
  }
  if (o.solver == YAND_SOLVER_PCG) {
    const unsigned nl = (unsigned)G.nl;
    hipLaunchKernelGGL(pcg_init_lanes_kernel, dim3(nl), dim3(PT), 0, st, G.pl);
    hipLaunchKernelGGL(pcg_alldone_kernel, dim3(1), dim3(64), 0, st, G.pl,
                       G.nl, G.cgall);
    for (int it = 0; it < o.krylov_maxit; ++it) {
      HIPTRY(launch_block_av(D.precision, D.A, D.lda, Tp, G.P, G.Zp, G.Z, st,
                             G.cgall));
      HIPTRY(launch_lane_scale(G.Z, G.s, G.ls.vec, G.nl, Tp, G.ZS, st,
                               G.cgall));
      HIPTRY(launch_block_atz(D.precision, D.A, D.lda, Tp, G.ZS, nullptr,
                              G.Yp, G.HP, st, G.cgall));
      hipLaunchKernelGGL(pcg_update_lanes_kernel, dim3(nl), dim3(PT), 0, st,
                         G.pl, o.krylov_tol);
      hipLaunchKernelGGL(pcg_alldone_kernel, dim3(1), dim3(64), 0, st, G.pl,
                         G.nl, G.cgall);
    }
    for (const auto& L : lanes)
      TRY(dir_from_solve(D, *L.w, L.p0, L.w->x, o, L.w->d));
  }
  for (const auto& L : lanes) {
    Work& w = *L.w;
    const int* skip = &w.sc->done;
    TRY(step_line(D, w, L.c, o, skip));
    HIPTRY(launch_axpy(w.x, w.d, D.n, w.sc, w.st));
  }
  return YAND_OK;
}

// ------------------------------------------------- constraints and start --

// x <- x + sum_a e_a (b_a - e_a^T x): minimum-norm move onto the budget (and
// target) constraint, expressed in the orthonormal frame e1, e2.
__global__ void __launch_bounds__(PT)
feasible_kernel(double* x, const double* E, int p0, int64_t n, double b1,
                double b2) {
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
            double* stats) {
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
  if (tid == 0) {
    stats[0] = mbar;
    stats[1] = nrm;
  }
}

__global__ void set_frozen_kernel(DevScalars* sc, int v) {
  if (threadIdx.x == 0) {
    sc->frozen = v;
    if (v) sc->done = 1;
  }
}
// Load the constraint frame into w.E and set w.x to the feasible start.
int setup_lane(const Data& D, Work& w, const double* target,
               const double* w0, int* p0) {
  *p0 = target ? 2 : 1;
  if (target && (!D.have_e2 || !std::isfinite(*target))) return YAND_ERR_ARG;
  hipLaunchKernelGGL(set_frozen_kernel, dim3(1), dim3(64), 0, w.st, w.sc, 0);
  HIPTRY(launch_reset_hold(w.hold, D.n, w.sc, w.st));
  HIPTRY(launch_copy(w.E, D.Efix, (int64_t)(*p0) * D.n, w.st));
  if (w0)
    HIPTRY(launch_copy(w.x, w0, D.n, w.st));
  else
    HIPTRY(launch_fill(w.x, D.n, 1.0 / (double)D.n, w.st));
  const double b1 = 1.0 / std::sqrt((double)D.n);
  const double b2 = target ? (*target - D.mbar) / D.mnorm : 0.0;
  hipLaunchKernelGGL(feasible_kernel, dim3(1), dim3(PT), 0, w.st, w.x, w.E,
                     *p0, D.n, b1, b2);
  return YAND_OK;
}

int check_simplex_start(const Data& D, Work& w, double tau) {
  std::vector<double> xh(D.n);
  HIPTRY(hipMemcpyAsync(xh.data(), w.x, D.n * sizeof(double),
                        hipMemcpyDeviceToHost, w.st));
  HIPTRY(hipStreamSynchronize(w.st));
  for (int64_t j = 0; j < D.n; ++j)
    if (!(xh[j] >= tau)) return YAND_ERR_ARG;
  return YAND_OK;
}

// ---------------------------------------------------- lanes (batch loop) --

struct Lane {
  const Data* D = nullptr;
  Work* w = nullptr;
  double c[4] = {0, 0, 0, 0};
  bool has_target = false;
  double target = 0.0;
  const double* w0 = nullptr;
  double* w_out = nullptr;
  int p0 = 1;
  // host state
  bool active = true, converged = false, frozen_set = false;
  bool stalled = false;  // the stall test ended the run
  int rc = YAND_OK;
  int small = 0;
  double f_prev = NAN;
  // stall-recovery phase of the lane and its iteration count when the phase
  // began (the phase's budget counts from there)
  int phase = 0, it0 = 0;
  yand_info info{};
};



// Apply the host decisions after reading a lane's scalars for one iteration
// (direct configuration).  Returns YAND_OK or a HIP error.
int after_iteration(Lane& L, const yand_opts& opts, const DirOpts& o) {
  Work& w = *L.w;
  const DevScalars& s = w.hs;
  L.info.oracle_passes++;
  L.info.f = s.f;
  L.info.gnorm = s.gn;
  L.info.kkt = o.simplex ? s.kkt : NAN;
  if (s.nonfinite) {
    L.rc = YAND_ERR_NONFINITE;
    L.active = false;
    return YAND_OK;
  }
  if (s.done) {
    L.converged = true;
    L.active = false;
    return YAND_OK;
  }
  if (s.fail) {
    // redo this iteration's direction with regularisation escalation; x did
    // not move, and z, g, nu of the iteration are still valid
    DirStats ds;
    int rc = direction_eager(*L.D, w, L.c, L.p0, w.x, o, w.d, &ds);
    if (rc != YAND_OK) {
      L.rc = rc;
      L.active = false;
      return YAND_OK;
    }
    TRY(step_line(*L.D, w, L.c, o, nullptr));
    HIPTRY(launch_axpy(w.x, w.d, L.D->n, w.sc, w.st));
    TRY(sync_scalars(w));
  }
  L.info.dense_traces++;
  L.info.third_passes++;
  L.info.ls_passes++;
  if (o.solver == YAND_SOLVER_PCG) {
    L.info.cg_iters += w.hs.cgit;
    L.info.hvp_passes += w.hs.cgit;
  }
  if (w.hs.projected) L.info.projected_steps++;
  L.info.lambda_used = w.hs.lambda;
  if (w.hs.status != 0) {
    L.rc = YAND_ERR_UNBOUNDED;
    L.active = false;
    return YAND_OK;
  }
  L.info.iterations++;
  const double a = w.hs.alpha, *A = w.hs.coef;
  const double dec = -(a * (A[1] + a * (A[2] + a * (A[3] + a * A[4]))));
  if (std::isnan(L.f_prev)) L.f_prev = A[0];
  // an iteration that adds holds changes the face: progress of the face
  // solver even when no weight moves
  if (dec < 1e-14 * std::fabs(L.f_prev) && w.hs.nhold <= w.hs.nhold0) {
    if (++L.small >= 3) {
      L.active = false;
      L.stalled = true;
    }
  } else {
    L.small = 0;
  }
  L.f_prev = A[0] - dec;
  const int pit = L.info.iterations - L.it0;
  L.info.phase_iterations[L.phase] = pit;
  if (pit >= opts.max_iter) L.active = false;
  return YAND_OK;
}

// Status of a lane that ran without error: converged, stalled (the stall
// test ended it, or restarts ran and it is still above eps) or the
// iteration / time budget ended it.
int finish_status(bool converged, bool stalled, int restarts) {
  if (converged) return YAND_OK;
  return (stalled || restarts > 0) ? YAND_WARN_STALL : YAND_WARN_MAXITER;
}

// Final stationarity check of a lane that stopped without converging.
int final_check(Lane& L, const yand_opts& opts, const DirOpts& o) {
  Work& w = *L.w;
  hipLaunchKernelGGL(set_frozen_kernel, dim3(1), dim3(64), 0, w.st, w.sc, 0);
  HIPTRY(launch_reset_hold(w.hold, L.D->n, w.sc, w.st));
  TRY(oracle_at(*L.D, w, L.c, w.x, true));
  TRY(stationarity(*L.D, w, o, L.p0, opts.eps));
  TRY(sync_scalars(w));
  L.info.f = w.hs.f;
  L.info.gnorm = w.hs.gn;
  L.info.kkt = o.simplex ? w.hs.kkt : NAN;
  L.info.oracle_passes++;
  if (w.hs.done) L.converged = true;
  return YAND_OK;
}

// Run the direct configuration on a set of lanes until each converges or
// stops.  Iteration 0 is enqueued eagerly; with use_graph, later iterations
// replay one captured graph of all lanes.  cs: control stream.  A single lane
// on the control stream itself needs no fork/join events.  opts.max_elapsed
// (> 0) stops every lane still running once that many seconds have passed
// since the call began, checked before each iteration.
int run_lanes(std::vector<Lane>& lanes, const yand_opts& opts,
              const DirOpts& o, hipStream_t cs, bool use_graph,
              DevScalars* host_sc, DevScalars* dev_sc,
              const Group* grp = nullptr) {
  const size_t nl = lanes.size();
  const auto t_start = std::chrono::steady_clock::now();
  HIPTRY(prepare_dense_kernels());
  const bool inline_lane =
      grp != nullptr || (nl == 1 && lanes[0].w->st == cs && !use_graph);
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join(inline_lane ? 0 : nl, nullptr);
  if (!inline_lane) {
    HIPTRY(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    for (auto& e : ev_join)
      HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  auto cleanup = [&]() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (auto& e : ev_join) (void)hipEventDestroy(e);
  };
  auto enqueue_all = [&]() -> int {
    if (grp) {
      std::vector<LaneRef> refs;
      for (auto& L : lanes) refs.push_back(LaneRef{L.D, L.w, L.c, L.p0});
      Group g = *grp;
      g.nl = (int)nl;
      return enqueue_group(refs, o, opts.eps, g, cs);
    }
    if (inline_lane) {
      Lane& L = lanes[0];
      return enqueue_iteration(*L.D, *L.w, L.c, L.p0, o, opts.eps);
    }
    HIPTRY(hipEventRecord(ev_fork, cs));
    for (size_t i = 0; i < nl; ++i) {
      Lane& L = lanes[i];
      HIPTRY(hipStreamWaitEvent(L.w->st, ev_fork, 0));
      TRY(enqueue_iteration(*L.D, *L.w, L.c, L.p0, o, opts.eps));
      HIPTRY(hipEventRecord(ev_join[i], L.w->st));
      HIPTRY(hipStreamWaitEvent(cs, ev_join[i], 0));
    }
    return YAND_OK;
  };
  auto read_all = [&]() -> int {
    if (dev_sc) {
      HIPTRY(hipMemcpyAsync(host_sc, dev_sc, nl * sizeof(DevScalars),
                            hipMemcpyDeviceToHost, cs));
      HIPTRY(hipStreamSynchronize(cs));
      for (size_t i = 0; i < nl; ++i) lanes[i].w->hs = host_sc[i];
    } else {
      for (auto& L : lanes) TRY(sync_scalars(*L.w));
      HIPTRY(hipStreamSynchronize(cs));
    }
    return YAND_OK;
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int rc = YAND_OK;
  for (int it = 0;; ++it) {
    if (opts.max_elapsed > 0.0 &&
        std::chrono::duration<double>(std::chrono::steady_clock::now() -
                                      t_start)
                .count() > opts.max_elapsed)
      for (auto& L : lanes) L.active = false;
    bool any = false;
    for (auto& L : lanes) any |= L.active;
    if (!any) break;
    // lanes that stopped must skip their work in replays
    for (auto& L : lanes)
      if (!L.active && !L.frozen_set) {
        hipLaunchKernelGGL(set_frozen_kernel, dim3(1), dim3(64), 0, cs,
                           L.w->sc, 1);
        L.frozen_set = true;
      }
    if (use_graph && it >= 1) {
      if (!exec) {
        // the frozen lanes' done flags were set on cs; make lane streams see it
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeGlobal) !=
            hipSuccess) {
          use_graph = false;
        } else {
          rc = enqueue_all();
          hipError_t e = hipStreamEndCapture(cs, &graph);
          if (rc != YAND_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            cleanup();
            return rc != YAND_OK ? rc : YAND_ERR_HIP;
          }
          if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) !=
              hipSuccess) {
            (void)hipGetLastError();
            (void)hipGraphDestroy(graph);
            graph = nullptr;
            exec = nullptr;
            use_graph = false;
          }
        }
      }
    }
    if (exec) {
      if (hipGraphLaunch(exec, cs) != hipSuccess) {
        rc = YAND_ERR_HIP;
        break;
      }
    } else {
      rc = enqueue_all();
      if (rc) break;
    }
    if ((rc = read_all())) break;
    for (auto& L : lanes) {
      if (!L.active) continue;
      if ((rc = after_iteration(L, opts, o))) break;
    }
    if (rc) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  cleanup();
  if (rc) return rc;
  for (auto& L : lanes) {
    if (L.rc == YAND_OK && !L.converged) TRY(final_check(L, opts, o));
    // holds belong to one solve: later calls on the work start without them
    HIPTRY(launch_reset_hold(L.w->hold, L.D->n, L.w->sc, L.w->st));
  }
  return YAND_OK;
}

}  // namespace

// ===================================================================== ABI ==

// ------------------------------------------------------- warm start --

namespace {

constexpr int kWsF = YAND_WS_FEATURES;

// Moments m1..m4 of the equal-weight portfolio (one value pass).
int equal_weight_moments(yand_ctx* ctx, double mom[4]) {
  const Data& D = ctx->d;
  Work& w = ctx->w;
  const double c1[4] = {1.0, 1.0, 1.0, 1.0};
  HIPTRY(launch_fill(w.x, D.n, 1.0 / (double)D.n, w.st));
  TRY(oracle_at(D, w, c1, w.x, false));
  TRY(sync_scalars(w));
  if (w.hs.nonfinite) return YAND_ERR_NONFINITE;
  for (int i = 0; i < 4; ++i) mom[i] = w.hs.mom[i];
  return YAND_OK;
}

void instance_features(const Data& D, const double mom[4], const double c[4],
                       const double* target, double* F) {
  const double tiny = 1e-300;
  const double m2 = std::max(mom[1], tiny);
  for (int k = 0; k < 4; ++k) F[k] = std::log1p(c[k]);
  F[4] = target ? 1.0 : 0.0;
  F[5] = (target && D.mnorm > 0.0) ? (*target - D.mbar) / D.mnorm : 0.0;
  F[6] = std::log(m2);
  F[7] = mom[2] / std::pow(m2, 1.5);
  F[8] = std::log(std::max(mom[3], tiny) / (m2 * m2));
  F[9] = D.mbar / std::sqrt(m2);
  F[10] = D.mnorm / std::sqrt((double)D.n * m2);
}

int all_features(yand_ctx* ctx, int64_t N, const double* C4,
                 const double* targets, std::vector<double>& F) {
  if (!ctx || N < 1 || !C4) return YAND_ERR_ARG;
  for (int64_t b = 0; b < N; ++b) {
    TRY(check_c(C4 + 4 * b));
    if (targets && (!std::isfinite(targets[b]) || !ctx->d.have_e2))
      return YAND_ERR_ARG;
  }
  double mom[4];
  TRY(equal_weight_moments(ctx, mom));
  F.assign((size_t)N * kWsF, 0.0);
  for (int64_t b = 0; b < N; ++b)
    instance_features(ctx->d, mom, C4 + 4 * b, targets ? targets + b : nullptr,
                      F.data() + b * kWsF);
  return YAND_OK;
}

// Standardised FP32 features on the device (caller frees *Xd).
int upload_features(const yand_mlp& h, const std::vector<double>& F,
                    int64_t N, hipStream_t st, float** Xd) {
  std::vector<float> xf((size_t)N * kWsF);
  for (int64_t b = 0; b < N; ++b)
    for (int k = 0; k < kWsF; ++k)
      xf[b * kWsF + k] =
          (float)((F[b * kWsF + k] - h.fmean[k]) / h.fscale[k]);
  TRY(alloc((void**)Xd, xf.size() * sizeof(float)));
  HIPTRY(hipMemcpyAsync(*Xd, xf.data(), xf.size() * sizeof(float),
                        hipMemcpyHostToDevice, st));
  HIPTRY(hipStreamSynchronize(st));
  return YAND_OK;
}

// Reduced-gradient norm at the start setup_lane builds from w0 (nullable);
// the start itself stays in w.x.
int start_gnorm(const Data& D, Work& w, const double c[4],
                const double* target, const double* w0, double* gn) {
  int p0 = 1;
  TRY(setup_lane(D, w, target, w0, &p0));
  TRY(oracle_at(D, w, c, w.x, true));
  HIPTRY(launch_grad_project(w.g, w.E, p0, D.n, w.sc, w.st, -1.0));
  TRY(sync_scalars(w));
  *gn = w.hs.nonfinite ? NAN : w.hs.gn;
  return YAND_OK;
}

struct DevBufs {
  std::vector<void*> p;
  ~DevBufs() {
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
  template <class T>
  int get(T** out, size_t bytes) {
    void* q = nullptr;
    TRY(alloc(&q, bytes));
    p.push_back(q);
    *out = (T*)q;
    return YAND_OK;
  }
};

}  // namespace

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
  o->eta = 0.05;
  o->linesearch = YAND_LS_EXACT;
  o->dense_fp64 = 0;
  o->trace_mode = YAND_TRACE_EXACT;
  o->probes = 64;
  o->probe_seed = 0;
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
  flush_timed(ctx->prof, ctx->w.st);
  free_work(ctx->w);
  void* ptrs[] = {ctx->d.A,    ctx->d.At,         ctx->d.mu,
                  ctx->d.Efix, ctx->d.AEfix,      ctx->d.syrk_order,
                  ctx->d.syrk_plan};
  for (void* p : ptrs) dfree(p);
  delete ctx;
  return YAND_OK;
}

}  // extern "C"

// Context creation.  All device memory is taken before the first kernel, so
// an allocation failure leaves nothing enqueued; with dense_upfront the n x n
// buffers of the direct configuration are taken here too instead of at the
// first direction.  Memory taken from an arena is cleared first (it holds
// the previous call's contents).
static int create_ctx(const double* R, int64_t T, int64_t n, int64_t ldr,
                      int precision, void* hip_stream, bool dense_upfront,
                      yand_ctx** out) {
  if (!out) return YAND_ERR_ARG;
  *out = nullptr;
  if (!R || T < 2 || n < 2 || ldr < n) return YAND_ERR_ARG;
  if (precision < 0 || precision > 2) return YAND_ERR_ARG;
  if (n > max_pass_columns(precision)) return YAND_ERR_ARG;
  yand_ctx* ctx = new yand_ctx();
  Data& D = ctx->d;
  Work& w = ctx->w;
  w.st = (hipStream_t)hip_stream;
  w.own_stream = false;
  w.prof = &ctx->prof;
  (void)hipGetDevice(&D.device);
  D.precision = precision;
  D.T = T;
  D.n = n;
  D.Tp = round_up(T, kRowPad);
  D.lda = round_up(n, kColPad);
  D.nt = D.lda / kTile;
  D.esize = precision == 0 ? 8 : precision == 1 ? 4 : 2;
  auto fail = [&](int rc) {
    yand_destroy(ctx);
    return rc;
  };
  int rc;
  const size_t nb = (size_t)D.lda * sizeof(double),
               tb = (size_t)D.Tp * sizeof(double);
  if ((rc = alloc(&D.A, (size_t)D.Tp * D.lda * D.esize)) ||
      (precision != YAND_FP64 &&
       (rc = alloc(&D.At, (size_t)D.Tp * D.lda * D.esize))) ||
      (rc = alloc((void**)&D.mu, nb)) ||
      (rc = alloc((void**)&D.Efix, 2 * nb)) ||
      (rc = alloc((void**)&D.AEfix, 2 * tb)))
    return fail(rc);
  if ((rc = alloc_work(w, D, nullptr))) return fail(rc);
  w.solo = true;
  hipStream_t st = w.st;
  double* colpart = nullptr;
  const int64_t nchunks = (T + 255) / 256;
  if ((rc = alloc((void**)&colpart, (size_t)nchunks * n * sizeof(double))))
    return fail(rc);
  // the SYRK's tile order and balanced schedule (not in the allocation-free
  // entry point, whose context uses the plain order)
  if (!g_arena) {
    const std::vector<int> ord = syrk_tile_order((int)D.nt);
    if (!ord.empty()) {
      if ((rc = alloc((void**)&D.syrk_order, ord.size() * sizeof(int))))
        return fail(rc);
      if (hipMemcpy(D.syrk_order, ord.data(), ord.size() * sizeof(int),
                    hipMemcpyHostToDevice) != hipSuccess)
        return fail(YAND_ERR_HIP);
      D.syrk_slots = (int64_t)ord.size() / 2;
      SyrkPlan plan;
      if (syrk_split_plan((int)D.nt, D.Tp / kSlice, syrk_split_slots(),
                          &plan)) {
        if ((rc = alloc((void**)&D.syrk_plan, plan.plan.size() * sizeof(int))))
          return fail(rc);
        if (hipMemcpy(D.syrk_plan, plan.plan.data(),
                      plan.plan.size() * sizeof(int),
                      hipMemcpyHostToDevice) != hipSuccess)
          return fail(YAND_ERR_HIP);
        D.syrk_wgs = plan.slots;
        D.syrk_rounds = plan.rounds;
        D.syrk_ntile2 = plan.ntile2;
        D.syrk_npieces = plan.npieces;
        D.syrk_nslots = plan.nslots;
      }
    }
  }
  if (dense_upfront && (rc = ensure_dense(w, D))) return fail(rc);
  if (dense_upfront && D.precision == YAND_FP64 &&
      (rc = ensure_syrk_ws(w, D)))
    return fail(rc);
  if (g_arena &&
      launch_fill((double*)g_arena->base, (int64_t)(g_arena->used / 8), 0.0,
                  st) != hipSuccess)
    return fail(YAND_ERR_HIP);
  if (init_work(w, D) != YAND_OK) return fail(YAND_ERR_HIP);
  hipError_t e = launch_center(R, T, n, ldr, precision, D.A, D.Tp, D.lda,
                               D.mu, colpart, &w.sc->nonfinite, st);
  if (e == hipSuccess && precision != YAND_FP64)
    e = launch_transpose_lp(precision, D.A, D.lda, D.Tp, D.At, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(efix_kernel, dim3(1), dim3(PT), 0, st, D.mu, n, D.Efix,
                       w.sums);
    for (int a = 0; a < 2 && e == hipSuccess; ++a) {
      PassArgs pa = pass_args(D, w, nullptr);
      pa.v = D.Efix + (int64_t)a * n;
      pa.tout = D.AEfix + (int64_t)a * D.Tp;
      int nwg;
      e = launch_pass(precision, PassKind::Dot, pa, st, &nwg);
    }
  }
  double stats[2] = {0.0, 0.0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(stats, w.sums, 2 * sizeof(double),
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&w.hs, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost,
                       st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(colpart);
  if (e != hipSuccess) return fail(YAND_ERR_HIP);
  if (w.hs.nonfinite) return fail(YAND_ERR_NONFINITE);
  D.mbar = stats[0];
  D.mnorm = stats[1];
  D.have_e2 = stats[1] > 1e-300;
  *out = ctx;
  return YAND_OK;
}

extern "C" {

int yand_create(const double* R, int64_t T, int64_t n, int64_t ldr,
                int precision, void* hip_stream, yand_ctx** out) {
  return create_ctx(R, T, n, ldr, precision, hip_stream, false, out);
}

int yand_shape(yand_ctx* ctx, int64_t* T, int64_t* n, int* precision) {
  if (!ctx) return YAND_ERR_ARG;
  if (T) *T = ctx->d.T;
  if (n) *n = ctx->d.n;
  if (precision) *precision = ctx->d.precision;
  return YAND_OK;
}

int yand_get_mu(yand_ctx* ctx, double* mu_out) {
  if (!ctx || !mu_out) return YAND_ERR_ARG;
  HIPTRY(hipMemcpyAsync(mu_out, ctx->d.mu, ctx->d.n * sizeof(double),
                        hipMemcpyDeviceToDevice, ctx->w.st));
  HIPTRY(hipStreamSynchronize(ctx->w.st));
  return YAND_OK;
}

int yand_eval(yand_ctx* ctx, const double c[4], const double* w, double* f,
              double* grad, double mom[4]) {
  if (!ctx || !w) return YAND_ERR_ARG;
  TRY(check_c(c));
  Work& W = ctx->w;
  TRY(oracle_at(ctx->d, W, c, w, grad != nullptr));
  if (grad)
    HIPTRY(hipMemcpyAsync(grad, W.g, ctx->d.n * sizeof(double),
                          hipMemcpyDeviceToDevice, W.st));
  TRY(sync_scalars(W));
  if (f) *f = W.hs.f;
  if (mom)
    for (int i = 0; i < 4; ++i) mom[i] = W.hs.mom[i];
  flush_timed(ctx->prof, W.st);
  return W.hs.nonfinite ? YAND_ERR_NONFINITE : YAND_OK;
}

int yand_hvp(yand_ctx* ctx, const double c[4], const double* w,
             const double* v, double* hv) {
  if (!ctx || !w || !v || !hv) return YAND_ERR_ARG;
  TRY(check_c(c));
  TRY(oracle_at(ctx->d, ctx->w, c, w, false));
  TRY(hvp_cached(ctx->d, ctx->w, c, v, hv, nullptr));
  HIPTRY(hipStreamSynchronize(ctx->w.st));
  flush_timed(ctx->prof, ctx->w.st);
  return YAND_OK;
}

int yand_linesearch_coeffs(yand_ctx* ctx, const double c[4], const double* w,
                           const double* d, double coef[5]) {
  if (!ctx || !w || !d || !coef) return YAND_ERR_ARG;
  TRY(check_c(c));
  Work& W = ctx->w;
  TRY(oracle_at(ctx->d, W, c, w, false));
  HIPTRY(launch_dot(ctx->d.mu, d, ctx->d.n, &W.sc->mud, W.st));
  TRY(line_at(ctx->d, W, c, d, 0, nullptr));
  TRY(sync_scalars(W));
  for (int i = 0; i < 5; ++i) coef[i] = W.hs.coef[i];
  flush_timed(ctx->prof, W.st);
  return YAND_OK;
}

int yand_select_step(yand_ctx* ctx, const double coef[5], double alpha_max,
                     double* alpha) {
  if (!ctx || !coef || !alpha) return YAND_ERR_ARG;
  if (std::isnan(alpha_max) || alpha_max < 0.0) return YAND_ERR_ARG;
  Work& W = ctx->w;
  TRY(sync_scalars(W));
  DevScalars hs = W.hs;
  for (int i = 0; i < 5; ++i) hs.coef[i] = coef[i];
  hs.amax = alpha_max;
  HIPTRY(hipMemcpyAsync(W.sc, &hs, sizeof(DevScalars), hipMemcpyHostToDevice,
                        W.st));
  HIPTRY(launch_select_step(W.sc, W.st));
  TRY(sync_scalars(W));
  *alpha = W.hs.alpha;
  return W.hs.status == 0 ? YAND_OK : YAND_ERR_UNBOUNDED;
}

int yand_affine_normal(yand_ctx* ctx, const double c[4], const double* target,
                       const double* w, const yand_opts* opts, double* d_out,
                       double* gnorm) {
  if (!ctx || !w || !d_out) return YAND_ERR_ARG;
  TRY(check_c(c));
  Work& W = ctx->w;
  int p0 = target ? 2 : 1;
  if (target && (!ctx->d.have_e2 || !std::isfinite(*target))) return YAND_ERR_ARG;
  HIPTRY(launch_copy(W.E, ctx->d.Efix, (int64_t)p0 * ctx->d.n, W.st));
  if (opts && (opts->trace_mode < YAND_TRACE_EXACT ||
               opts->trace_mode > YAND_TRACE_PROBE || opts->probes < 1 ||
               opts->probes > kBlockWidth || !(opts->krylov_tol > 0.0)))
    return YAND_ERR_ARG;
  DirOpts o;
  if (opts) {
    o.solver = opts->solver;
    o.reg = opts->regularization;
    o.krylov_tol = opts->krylov_tol;
    o.krylov_maxit = opts->krylov_maxit;
    o.tau = opts->tau;
    o.dense64 = opts->dense_fp64 != 0;
    o.probe = opts->trace_mode == YAND_TRACE_PROBE;
    o.probes = opts->probes;
    o.seed = opts->probe_seed;
  }
  TRY(oracle_at(ctx->d, W, c, w, true));
  HIPTRY(launch_grad_project(W.g, W.E, p0, ctx->d.n, W.sc, W.st));
  TRY(direction_eager(ctx->d, W, c, p0, w, o, d_out, nullptr));
  TRY(sync_scalars(W));
  if (gnorm) *gnorm = W.hs.gn;
  flush_timed(ctx->prof, W.st);
  return W.hs.nonfinite ? YAND_ERR_NONFINITE : YAND_OK;
}

int yand_project_simplex(const double* y, int64_t n, double tau, double* x) {
  if (!y || !x || n < 1 || !(tau >= 0.0) || !(tau * (double)n < 1.0))
    return YAND_ERR_ARG;
  HIPTRY(launch_project_simplex(y, n, tau, x, nullptr));
  HIPTRY(hipStreamSynchronize(nullptr));
  return YAND_OK;
}

int yand_kkt_residual(yand_ctx* ctx, const double c[4], const double* w,
                      double tau, double* kkt) {
  if (!ctx || !w || !kkt || !(tau >= 0.0) || !(tau * (double)ctx->d.n < 1.0))
    return YAND_ERR_ARG;
  TRY(check_c(c));
  Work& W = ctx->w;
  hipLaunchKernelGGL(set_frozen_kernel, dim3(1), dim3(64), 0, W.st, W.sc, 0);
  TRY(oracle_at(ctx->d, W, c, w, true));
  HIPTRY(launch_kkt(w, W.g, ctx->d.n, tau, -1.0, W.ptmp, W.sc, W.st));
  TRY(sync_scalars(W));
  *kkt = W.hs.kkt;
  return W.hs.nonfinite ? YAND_ERR_NONFINITE : YAND_OK;
}

// PCG configuration with stall recovery (eager; the Krylov test is on the host).
static int solve_pcg(yand_ctx* ctx, const double c[4], int p0,
                     const yand_opts& opts, yand_info& inf, bool* converged,
                     bool* stalled) {
  const Data& D = ctx->d;
  Work& w = ctx->w;
  DirOpts o;
  o.krylov_tol = opts.krylov_tol;
  o.probe = opts.trace_mode == YAND_TRACE_PROBE;
  o.probes = opts.probes;
  o.seed = opts.probe_seed;
  o.tau = opts.tau;
  o.dense64 = opts.dense_fp64 != 0;
  o.simplex = opts.feasible_set == YAND_SET_SIMPLEX;
  o.faces = o.simplex && opts.eta > 0.0 && p0 == 1;
  o.select = opts.linesearch == YAND_LS_ARMIJO ? 2 : 1;
  struct Phase {
    int solver, kmax, max_iter;
    double reg, eta;
  };
  // stall recovery: budget set, twice the Krylov budget then the direct
  // solve; simplex boundary block, the projected trial steps 0.045 then
  // 0.02 (Appendix D, Table "YAND-MVSK parameter settings")
  std::vector<Phase> phases;
  phases.push_back({YAND_SOLVER_PCG, opts.krylov_maxit, opts.max_iter,
                    opts.regularization, opts.eta});
  if (opts.stall_recovery) {
    if (o.faces) {
      phases.push_back({YAND_SOLVER_PCG, opts.krylov_maxit,
                        opts.restart_max_iter, opts.regularization, 0.045});
      phases.push_back({YAND_SOLVER_PCG, opts.krylov_maxit,
                        opts.restart_max_iter, opts.regularization, 0.02});
    } else {
      phases.push_back({YAND_SOLVER_PCG, 2 * opts.krylov_maxit,
                        opts.restart_max_iter, opts.regularization, opts.eta});
      phases.push_back({YAND_SOLVER_DIRECT, 0, opts.restart_max_iter, 0.0,
                        opts.eta});
    }
  }
  *converged = false;
  for (size_t ph = 0; ph < phases.size() && !*converged; ++ph) {
    if (ph > 0) inf.restarts++;
    *stalled = false;
    const int it_phase0 = inf.iterations;
    o.solver = phases[ph].solver;
    o.krylov_maxit = phases[ph].kmax;
    o.reg = phases[ph].reg;
    o.eta = phases[ph].eta;
    const auto t_phase = std::chrono::steady_clock::now();
    int small = 0;
    double f_prev = NAN;
    HIPTRY(launch_reset_hold(w.hold, D.n, w.sc, w.st));
    for (int it = 0;; ++it) {
      TRY(oracle_at(D, w, c, w.x, true));
      inf.oracle_passes++;
      TRY(stationarity(D, w, o, p0, opts.eps));
      TRY(sync_scalars(w));
      inf.f = w.hs.f;
      inf.gnorm = w.hs.gn;
      inf.kkt = o.simplex ? w.hs.kkt : NAN;
      if (w.hs.nonfinite) return YAND_ERR_NONFINITE;
      if (std::isnan(f_prev)) f_prev = w.hs.f;
      if (w.hs.done) {
        *converged = true;
        break;
      }
      if (it >= phases[ph].max_iter) break;
      const double el = std::chrono::duration<double>(
                            std::chrono::steady_clock::now() - t_phase)
                            .count();
      if (opts.max_elapsed > 0.0 && el > opts.max_elapsed) break;
      DirStats ds;
      // the probe block of this direction: the solve's direction count
      o.draw = (uint64_t)(inf.dense_traces + inf.probe_traces);
      TRY(direction_eager(D, w, c, p0, w.x, o, w.d, &ds));
      if (o.probe && o.solver == YAND_SOLVER_PCG)
        inf.probe_traces++;
      else
        inf.dense_traces++;
      if (ds.thin) inf.thin_traces++;
      inf.third_passes++;
      inf.cg_iters += ds.cg;
      inf.hvp_passes += ds.cg;
      inf.probe_cg_iters += ds.probe_cg;
      TRY(step_line(D, w, c, o, nullptr));
      inf.ls_passes++;
      TRY(sync_scalars(w));
      inf.lambda_used = w.hs.lambda;
      if (w.hs.projected) inf.projected_steps++;
      if (w.hs.status != 0) return YAND_ERR_UNBOUNDED;
      HIPTRY(launch_axpy(w.x, w.d, D.n, w.sc, w.st));
      inf.iterations++;
      const double a = w.hs.alpha, *A = w.hs.coef;
      const double dec = -(a * (A[1] + a * (A[2] + a * (A[3] + a * A[4]))));
      inf.phase_iterations[ph] = inf.iterations - it_phase0;
      if (dec < 1e-14 * std::fabs(f_prev) && w.hs.nhold <= w.hs.nhold0) {
        if (++small >= 3) {
          *stalled = true;
          break;
        }
      } else {
        small = 0;
      }
      f_prev = A[0] - dec;
    }
    if (!*converged) {
      // budget spent or stalled: the phase's state is that of x on its own
      // face, without the face solver's holds
      HIPTRY(launch_reset_hold(w.hold, D.n, w.sc, w.st));
      TRY(oracle_at(D, w, c, w.x, true));
      TRY(stationarity(D, w, o, p0, opts.eps));
      TRY(sync_scalars(w));
      inf.f = w.hs.f;
      inf.gnorm = w.hs.gn;
      inf.kkt = o.simplex ? w.hs.kkt : NAN;
      if (w.hs.nonfinite) return YAND_ERR_NONFINITE;
      *converged = w.hs.done != 0;
    }
  }
  HIPTRY(launch_reset_hold(w.hold, D.n, w.sc, w.st));
  return YAND_OK;
}

static bool valid_opts(const yand_opts& o) {
  return o.eps >= 0.0 && o.max_iter >= 0 && o.tau >= 0.0 &&
         (o.trace_mode == YAND_TRACE_EXACT ||
          o.trace_mode == YAND_TRACE_PROBE) &&
         o.probes >= 1 && o.probes <= kBlockWidth &&
         o.krylov_tol > 0.0 && std::isfinite(o.krylov_tol) &&
         !std::isnan(o.max_elapsed) &&
         (o.solver == YAND_SOLVER_DIRECT || o.solver == YAND_SOLVER_PCG) &&
         (o.feasible_set == YAND_SET_BUDGET ||
          o.feasible_set == YAND_SET_SIMPLEX) &&
         o.krylov_maxit >= 0 && o.restart_max_iter >= 0 && o.eta >= 0.0 &&
         std::isfinite(o.eta) &&
         (o.linesearch == YAND_LS_EXACT || o.linesearch == YAND_LS_ARMIJO);
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
  if (!valid_opts(opts)) return YAND_ERR_ARG;
  const auto t_start = std::chrono::steady_clock::now();
  const Data& D = ctx->d;
  Work& w = ctx->w;
  int p0;
  TRY(setup_lane(D, w, target, w0, &p0));
  if (opts.feasible_set == YAND_SET_SIMPLEX)
    TRY(check_simplex_start(D, w, opts.tau));
  yand_info inf{};
  int rc = YAND_OK;
  bool converged = false, stalled = false;
  if (opts.solver == YAND_SOLVER_PCG) {
    rc = solve_pcg(ctx, c, p0, opts, inf, &converged, &stalled);
  } else {
    DirOpts o;
    o.tau = opts.tau;
    o.dense64 = opts.dense_fp64 != 0;
    o.simplex = opts.feasible_set == YAND_SET_SIMPLEX;
    o.faces = o.simplex && opts.eta > 0.0 && p0 == 1;
    o.eta = opts.eta;
    o.select = opts.linesearch == YAND_LS_ARMIJO ? 2 : 1;
    std::vector<Lane> lanes(1);
    Lane& L = lanes[0];
    L.D = &D;
    L.w = &w;
    for (int i = 0; i < 4; ++i) L.c[i] = c[i];
    L.p0 = p0;
    L.active = opts.max_iter > 0;
    rc = run_lanes(lanes, opts, o, w.st, false, nullptr, nullptr);
    if (rc == YAND_OK) {
      inf = L.info;
      converged = L.converged;
      stalled = L.stalled;
      if (L.rc != YAND_OK) rc = L.rc;
    }
  }
  int status;
  if (rc == YAND_OK) {
    status = finish_status(converged, stalled, inf.restarts);
    HIPTRY(hipMemcpyAsync(w_out, w.x, D.n * sizeof(double),
                          hipMemcpyDeviceToDevice, w.st));
    HIPTRY(hipStreamSynchronize(w.st));
  } else {
    status = rc;
  }
  inf.status = status;
  inf.elapsed = std::chrono::duration<double>(
                    std::chrono::steady_clock::now() - t_start)
                    .count();
  if (info) *info = inf;
  flush_timed(ctx->prof, w.st);
  return status;
}

// Batched solve: each instance b runs on contexts[b] (one shared context for
// a frontier, or different ones for universes of different n).  Instances are
// processed in waves of at most `lanes` solves that advance together.
static int batch_solve(int64_t B, yand_ctx* const* ctxs, const double* C4,
                       const double* targets, const double* const* W0,
                       const yand_opts* opts_in, double* const* W_out,
                       yand_info* infos, int max_lanes, int use_graph,
                       bool group_lanes) {
  if (B <= 0 || !ctxs || !C4 || !W_out) return YAND_ERR_ARG;
  yand_opts opts;
  if (opts_in)
    opts = *opts_in;
  else
    yand_default_opts(&opts);
  if (!valid_opts(opts)) return YAND_ERR_ARG;
  // the probe estimate of the trace runs in single solves only
  if (opts.solver == YAND_SOLVER_PCG && opts.trace_mode != YAND_TRACE_EXACT)
    return YAND_ERR_ARG;
  for (int64_t b = 0; b < B; ++b) {
    if (!ctxs[b] || !W_out[b]) return YAND_ERR_ARG;
    TRY(check_c(C4 + 4 * b));
    if (ctxs[b]->d.device != ctxs[0]->d.device) return YAND_ERR_ARG;
  }
  const auto t_start = std::chrono::steady_clock::now();
  // Own control stream (graph capture is not allowed on the legacy default
  // stream), ordered after the caller's stream and joined back at the end.
  hipStream_t caller = ctxs[0]->w.st;
  hipStream_t cs = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  HIPTRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  HIPTRY(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
  HIPTRY(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
  HIPTRY(hipEventRecord(ev_in, caller));
  HIPTRY(hipStreamWaitEvent(cs, ev_in, 0));
  DirOpts o;
  o.tau = opts.tau;
  o.dense64 = opts.dense_fp64 != 0;
  o.simplex = opts.feasible_set == YAND_SET_SIMPLEX;
  o.faces = o.simplex && opts.eta > 0.0 && !targets;
  o.eta = opts.eta;
  o.select = opts.linesearch == YAND_LS_ARMIJO ? 2 : 1;
  o.solver = opts.solver;
  o.krylov_tol = opts.krylov_tol;
  o.krylov_maxit = opts.krylov_maxit;
  o.reg = opts.solver == YAND_SOLVER_PCG ? opts.regularization : 0.0;
  const bool pcg = opts.solver == YAND_SOLVER_PCG;
  // lane count: bounded by max_lanes and by free device memory
  size_t freeb = 0, totalb = 0;
  (void)hipMemGetInfo(&freeb, &totalb);
  size_t per_lane = 0;
  for (int64_t b = 0; b < B; ++b) {
    const Data& D = ctxs[b]->d;
    size_t need = 3 * (size_t)D.lda * D.lda * 8 + (size_t)D.nt * D.Tp * 8 +
                  (size_t)kMaxPassGroups * D.lda * 8 + 12 * (size_t)D.Tp * 8 +
                  24 * (size_t)D.lda * 8 + (size_t)((D.n + 63) / 64) * D.n * 8;
    if (D.precision != YAND_FP64)
      need += ((size_t)D.Tp + D.lda) * D.lda * 4;
    per_lane = std::max(per_lane, need);
  }
  int64_t nl = std::min<int64_t>(B, max_lanes > 0 ? max_lanes : 64);
  const int64_t mem_lanes = (int64_t)((freeb / 2) / std::max<size_t>(per_lane, 1));
  nl = std::max<int64_t>(1, std::min(nl, mem_lanes));
  // workspaces with their own streams and one contiguous scalar block
  DevScalars* dev_sc = nullptr;
  if (alloc((void**)&dev_sc, (size_t)nl * sizeof(DevScalars)) != YAND_OK) {
    (void)hipStreamDestroy(cs);
    (void)hipEventDestroy(ev_in);
    (void)hipEventDestroy(ev_out);
    return YAND_ERR_OOM;
  }
  HIPTRY(hipMemsetAsync(dev_sc, 0, (size_t)nl * sizeof(DevScalars), cs));
  std::vector<DevScalars> host_sc(nl);
  std::vector<Work> works(nl);
  // every workspace is sized for the largest instance it may serve
  Data big = ctxs[0]->d;
  for (int64_t b = 0; b < B; ++b) {
    const Data& D = ctxs[b]->d;
    big.n = std::max(big.n, D.n);
    big.lda = std::max(big.lda, D.lda);
    big.Tp = std::max(big.Tp, D.Tp);
    big.nt = std::max(big.nt, D.nt);
    // matrix-core scratch for any FP32 / BF16 context, sized for the widest
    if (D.precision != YAND_FP64 &&
        (big.precision == YAND_FP64 || D.esize > big.esize)) {
      big.precision = D.precision;
      big.esize = D.esize;
    }
  }
  int rc = YAND_OK;
  // lockstep lanes: instances on one context whose exact-trace products are
  // FP64 share grouped launches; their dense buffers live in strided blocks
  bool lockstep = nl > 1 && group_lanes;
  for (int64_t b = 1; b < B && lockstep; ++b)
    lockstep = ctxs[b] == ctxs[0];
  lockstep = lockstep && (big.precision == YAND_FP64 || opts.dense_fp64);
  Group grp;
  double* gblk[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double* pblk[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  if (lockstep && pcg) {
    // batched tangent solves: P, HP, Z, ZS and the split partials
    int sv = 1, sz = 1;
    block_splits(big.Tp, big.lda, &sv, &sz);
    const int64_t bw = kBlockWidth;
    const int64_t sizes[6] = {bw * big.lda, bw * big.lda, big.Tp * bw,
                              big.Tp * bw, sv * big.Tp * bw,
                              sz * bw * big.lda};
    for (int q = 0; q < 6 && rc == YAND_OK; ++q)
      rc = alloc((void**)&pblk[q], (size_t)sizes[q] * sizeof(double));
    if (rc == YAND_OK)
      rc = alloc((void**)&grp.pl, kBlockWidth * sizeof(PcgLane));
    if (rc == YAND_OK) rc = alloc((void**)&grp.cgall, sizeof(int));
    // rows of P past the lanes (and past n) stay zero for the products
    if (rc == YAND_OK &&
        hipMemsetAsync(pblk[0], 0, (size_t)sizes[0] * sizeof(double), cs) !=
            hipSuccess)
      rc = YAND_ERR_HIP;
    grp.P = pblk[0];
    grp.HP = pblk[1];
    grp.Z = pblk[2];
    grp.ZS = pblk[3];
    grp.Zp = pblk[4];
    grp.Yp = pblk[5];
  }
  if (lockstep) {
    const int64_t mat = big.lda * big.lda, rnl = big.nt * big.Tp;
    const int64_t sizes[5] = {mat, mat, mat, rnl, big.Tp};
    for (int q = 0; q < 5 && rc == YAND_OK; ++q)
      rc = alloc((void**)&gblk[q], (size_t)sizes[q] * nl * sizeof(double));
    grp.B = gblk[0];
    grp.M = gblk[1];
    grp.X = gblk[2];
    grp.rn = gblk[3];
    grp.s = gblk[4];
    grp.ls.mat = mat;
    grp.ls.rn = rnl;
    grp.ls.vec = big.Tp;
    grp.ls.flag = (int64_t)(sizeof(DevScalars) / sizeof(int));
    grp.skip = &dev_sc[0].done;
    grp.fail = &dev_sc[0].fail;
    if (rc == YAND_OK && big.syrk_plan)
      rc = alloc_syrk_ws(big, (int)nl, cs, &grp.syrk_ws, &grp.syrk_cnt);
  }
  for (int64_t i = 0; i < nl && rc == YAND_OK; ++i) {
    Work& w = works[i];
    if (lockstep) {
      w.st = cs;
      w.own_stream = false;
    } else {
      if (hipStreamCreateWithFlags(&w.st, hipStreamNonBlocking) !=
          hipSuccess) {
        rc = YAND_ERR_HIP;
        break;
      }
      w.own_stream = true;
      if (hipStreamWaitEvent(w.st, ev_in, 0) != hipSuccess) {
        rc = YAND_ERR_HIP;
        break;
      }
    }
    rc = alloc_work(w, big, dev_sc + i);
    if (rc == YAND_OK && lockstep) {
      dfree(w.s_t);
      w.s_t = grp.s + i * grp.ls.vec;
      w.B = grp.B + i * grp.ls.mat;
      w.M = grp.M + i * grp.ls.mat;
      w.X = grp.X + i * grp.ls.mat;
      w.rn = grp.rn + i * grp.ls.rn;
      w.shared_dense = true;
      if (pcg) {
        dfree(w.pcg_p);
        dfree(w.hv);
        w.pcg_p = grp.P + i * big.lda;
        w.hv = grp.HP + i * big.lda;
        w.shared_pcg = true;
      }
    }
    if (rc == YAND_OK) rc = ensure_dense(w, big);
    if (rc == YAND_OK && (big.precision == YAND_FP64 || opts.dense_fp64))
      rc = ensure_syrk_ws(w, big);
    if (rc == YAND_OK) rc = init_work(w, big);
  }
  for (int64_t start = 0; start < B && rc == YAND_OK; start += nl) {
    const int64_t cnt = std::min(nl, B - start);
    std::vector<Lane> lanes(cnt);
    for (int64_t i = 0; i < cnt && rc == YAND_OK; ++i) {
      const int64_t b = start + i;
      Lane& L = lanes[i];
      L.D = &ctxs[b]->d;
      L.w = &works[i];
      for (int k = 0; k < 4; ++k) L.c[k] = C4[4 * b + k];
      L.has_target = targets != nullptr;
      if (targets) L.target = targets[b];
      L.w_out = W_out[b];
      L.w0 = W0 ? W0[b] : nullptr;
      L.active = opts.max_iter > 0;
      rc = setup_lane(*L.D, *L.w, targets ? &L.target : nullptr, L.w0,
                      &L.p0);
      if (rc == YAND_OK && o.simplex)
        rc = check_simplex_start(*L.D, *L.w, opts.tau);
    }
    for (auto& w : works) {
      if (rc != YAND_OK) break;
      if (hipStreamSynchronize(w.st) != hipSuccess) rc = YAND_ERR_HIP;
    }
    if (rc != YAND_OK) break;
    // the lanes' solve operands for the batched tangent solves (per phase:
    // the face mask and the preconditioner source depend on it)
    auto upload_pcg = [&](const DirOpts& od) -> int {
      if (!(lockstep && od.solver == YAND_SOLVER_PCG)) return YAND_OK;
      std::vector<PcgLane> pl(cnt);
      for (int64_t i = 0; i < cnt; ++i)
        pl[i] = pcg_lane(*lanes[i].D, *lanes[i].w, lanes[i].p0, od,
                         lanes[i].w->B, lanes[i].D->lda + 1);
      HIPTRY(hipMemcpyAsync(grp.pl, pl.data(), cnt * sizeof(PcgLane),
                            hipMemcpyHostToDevice, cs));
      HIPTRY(hipStreamSynchronize(cs));
      return YAND_OK;
    };
    rc = upload_pcg(o);
    if (rc == YAND_OK)
      rc = run_lanes(lanes, opts, o, cs, use_graph != 0, host_sc.data(),
                     dev_sc, lockstep ? &grp : nullptr);
    // stall recovery of the PCG configuration, as in a single solve: the
    // lanes that neither converged nor failed continue from where they
    // stopped, with twice the Krylov budget, then with the direct solve
    // (budget set), or with the projected trial steps 0.045 then 0.02 (the
    // simplex boundary block)
    if (pcg && opts.stall_recovery) {
      struct Phase {
        int solver, kmax;
        double reg, eta;
      };
      std::vector<Phase> phases;
      if (o.faces) {
        phases.push_back({YAND_SOLVER_PCG, opts.krylov_maxit,
                          opts.regularization, 0.045});
        phases.push_back({YAND_SOLVER_PCG, opts.krylov_maxit,
                          opts.regularization, 0.02});
      } else {
        phases.push_back({YAND_SOLVER_PCG, 2 * opts.krylov_maxit,
                          opts.regularization, opts.eta});
        phases.push_back({YAND_SOLVER_DIRECT, 0, 0.0, opts.eta});
      }
      for (size_t ph = 0; ph < phases.size() && rc == YAND_OK; ++ph) {
        bool any = false;
        for (auto& L : lanes) {
          L.active = false;
          if (L.converged || L.rc != YAND_OK) continue;
          L.active = opts.restart_max_iter > 0;
          L.stalled = false;
          L.small = 0;
          L.f_prev = NAN;
          L.frozen_set = false;
          L.info.restarts++;
          L.phase = (int)ph + 1;
          L.it0 = L.info.iterations;
          any = true;
        }
        if (!any) break;
        yand_opts op = opts;
        op.max_iter = opts.restart_max_iter;
        DirOpts od = o;
        od.solver = phases[ph].solver;
        od.krylov_maxit = phases[ph].kmax;
        od.reg = phases[ph].reg;
        od.eta = phases[ph].eta;
        rc = upload_pcg(od);
        if (rc == YAND_OK)
          rc = run_lanes(lanes, op, od, cs, use_graph != 0, host_sc.data(),
                         dev_sc, lockstep ? &grp : nullptr);
      }
    }
    for (int64_t i = 0; i < cnt && rc == YAND_OK; ++i) {
      Lane& L = lanes[i];
      const int64_t b = start + i;
      int st = L.rc != YAND_OK
                   ? L.rc
                   : finish_status(L.converged, L.stalled, L.info.restarts);
      L.info.status = st;
      if (hipMemcpyAsync(L.w_out, L.w->x, L.D->n * sizeof(double),
                         hipMemcpyDeviceToDevice, cs) != hipSuccess)
        rc = YAND_ERR_HIP;
      L.info.elapsed = std::chrono::duration<double>(
                           std::chrono::steady_clock::now() - t_start)
                           .count();
      if (infos) infos[b] = L.info;
    }
  }
  if (hipStreamSynchronize(cs) != hipSuccess && rc == YAND_OK)
    rc = YAND_ERR_HIP;
  for (auto& w : works) free_work(w);
  for (double* q : gblk) dfree(q);
  dfree(grp.syrk_ws);
  dfree(grp.syrk_cnt);
  for (double* q : pblk) dfree(q);
  dfree(grp.pl);
  dfree(grp.cgall);
  (void)hipFree(dev_sc);
  (void)hipEventRecord(ev_out, cs);
  (void)hipStreamWaitEvent(caller, ev_out, 0);
  (void)hipStreamSynchronize(caller);
  (void)hipEventDestroy(ev_in);
  (void)hipEventDestroy(ev_out);
  (void)hipStreamDestroy(cs);
  return rc;
}

int yand_frontier_solve(yand_ctx* ctx, int64_t B, const double* C4,
                        const double* targets, const double* W0,
                        const yand_opts* opts, double* W_out,
                        yand_info* infos) {
  if (!ctx || !W_out || B <= 0) return YAND_ERR_ARG;
  std::vector<yand_ctx*> ctxs(B, ctx);
  std::vector<double*> outs(B);
  std::vector<const double*> starts(B);
  for (int64_t b = 0; b < B; ++b) {
    outs[b] = W_out + b * ctx->d.n;
    starts[b] = W0 ? W0 + b * ctx->d.n : nullptr;
  }
  return batch_solve(B, ctxs.data(), C4, targets, W0 ? starts.data() : nullptr,
                     opts, outs.data(), infos, 64, 1, true);
}

int yand_batch_solve(int64_t B, yand_ctx* const* ctxs, const double* C4,
                     const double* targets, const double* const* W0,
                     const yand_opts* opts, double* const* W_out,
                     yand_info* infos, int max_lanes, int use_graph) {
  return batch_solve(B, ctxs, C4, targets, W0, opts, W_out, infos, max_lanes,
                     use_graph & 1, (use_graph & 2) == 0);
}

int yand_warmstart_features(yand_ctx* ctx, int64_t N, const double* C4,
                            const double* targets, double* F) {
  if (!F) return YAND_ERR_ARG;
  std::vector<double> f;
  TRY(all_features(ctx, N, C4, targets, f));
  std::memcpy(F, f.data(), f.size() * sizeof(double));
  return YAND_OK;
}

int yand_warmstart_train(yand_ctx* ctx, int64_t N, const double* C4,
                         const double* targets, const double* W_solved,
                         const yand_mlp_opts* opts_in, yand_mlp** out,
                         double* final_loss) {
  if (!out) return YAND_ERR_ARG;
  *out = nullptr;
  if (!ctx || !W_solved || N < 1 || N > (1 << 20)) return YAND_ERR_ARG;
  yand_mlp_opts o;
  if (opts_in)
    o = *opts_in;
  else
    yand_default_mlp_opts(&o);
  if (o.epochs < 0 || !(o.lr > 0.0) || o.hidden < 1 || o.layers < 2)
    return YAND_ERR_ARG;
  std::vector<double> F;
  TRY(all_features(ctx, N, C4, targets, F));
  const Data& D = ctx->d;
  hipStream_t st = ctx->w.st;
  const int64_t m = D.n - 1;
  yand_mlp* h = nullptr;
  TRY(yand_mlp_create(kWsF, m, o.hidden, o.layers, o.seed, st, &h));
  std::unique_ptr<yand_mlp, int (*)(yand_mlp*)> guard(h, yand_mlp_destroy);
  // feature standardisation (per column; constant columns map to zero)
  h->fmean.assign(kWsF, 0.0);
  h->fscale.assign(kWsF, 1.0);
  for (int k = 0; k < kWsF; ++k) {
    double s = 0.0, q = 0.0;
    for (int64_t b = 0; b < N; ++b) s += F[b * kWsF + k];
    const double mean = s / (double)N;
    for (int64_t b = 0; b < N; ++b) {
      const double d = F[b * kWsF + k] - mean;
      q += d * d;
    }
    const double sd = std::sqrt(q / (double)N);
    h->fmean[k] = mean;
    h->fscale[k] = sd > 1e-12 * std::max(1.0, std::fabs(mean)) ? sd : 1.0;
  }
  DevBufs bufs;
  float* Xd = nullptr;
  TRY(upload_features(*h, F, N, st, &Xd));
  bufs.p.push_back(Xd);
  // targets: reduced coordinates, centred per column, one global scale
  double *Y = nullptr, *ss = nullptr;
  float* Z = nullptr;
  TRY(bufs.get(&Y, (size_t)N * m * sizeof(double)));
  TRY(bufs.get(&ss, (size_t)m * sizeof(double)));
  TRY(bufs.get(&Z, (size_t)N * m * sizeof(float)));
  TRY(alloc((void**)&h->ybar, (size_t)m * sizeof(double)));
  HIPTRY(launch_to_reduced(W_solved, N, D.n, Y, st));
  HIPTRY(launch_col_stats(Y, N, m, h->ybar, ss, st));
  std::vector<double> hs(m);
  HIPTRY(hipMemcpyAsync(hs.data(), ss, m * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  double tot = 0.0;
  for (double x : hs) tot += x;
  if (!std::isfinite(tot)) return YAND_ERR_NONFINITE;
  const double scale = std::sqrt(tot / ((double)N * (double)m));
  h->yscale = scale > 0.0 ? scale : 1.0;
  HIPTRY(launch_standardize(Y, h->ybar, h->yscale, N, m, Z, st));
  h->n = D.n;
  double loss = NAN;
  for (int e = 0; e < o.epochs; ++e) {
    TRY(h->net.loss_grad(N, Xd, Z, e + 1 == o.epochs ? &loss : nullptr));
    h->t += 1;
    TRY(h->net.adam(h->net.grads, o.lr, h->t));
  }
  HIPTRY(hipStreamSynchronize(st));
  if (final_loss) *final_loss = loss;
  *out = guard.release();
  return YAND_OK;
}

int yand_warmstart_predict(yand_ctx* ctx, yand_mlp* mlp, int64_t B,
                           const double* C4, const double* targets,
                           double* W0_out, int* used_mlp, double* gnorms) {
  if (!ctx || !mlp || !W0_out || B < 1 || B > (1 << 20)) return YAND_ERR_ARG;
  const Data& D = ctx->d;
  if (mlp->n != D.n || !mlp->ybar || (int64_t)mlp->fmean.size() != kWsF)
    return YAND_ERR_ARG;
  std::vector<double> F;
  TRY(all_features(ctx, B, C4, targets, F));
  Work& w = ctx->w;
  hipStream_t st = w.st;
  // the network runs on this context's stream
  HIPTRY(hipStreamSynchronize(mlp->stream));
  mlp->net.stream = st;
  mlp->stream = st;
  DevBufs bufs;
  float* Xd = nullptr;
  TRY(upload_features(*mlp, F, B, st, &Xd));
  bufs.p.push_back(Xd);
  float* O = nullptr;
  TRY(bufs.get(&O, (size_t)B * (D.n - 1) * sizeof(float)));
  TRY(mlp->net.forward(B, Xd, O));
  HIPTRY(launch_from_reduced_f32(O, mlp->ybar, mlp->yscale, B, D.n, W0_out,
                                 st));
  for (int64_t b = 0; b < B; ++b) {
    const double* c = C4 + 4 * b;
    const double* tg = targets ? targets + b : nullptr;
    double* row = W0_out + b * D.n;
    double g_mlp = NAN, g_plain = NAN;
    TRY(start_gnorm(D, w, c, tg, row, &g_mlp));
    HIPTRY(launch_copy(row, w.x, D.n, st));
    TRY(start_gnorm(D, w, c, tg, nullptr, &g_plain));
    const bool use = g_mlp < g_plain;  // false when the proposal is NaN
    if (!use) HIPTRY(launch_copy(row, w.x, D.n, st));
    if (used_mlp) used_mlp[b] = use ? 1 : 0;
    if (gnorms) {
      gnorms[2 * b] = g_mlp;
      gnorms[2 * b + 1] = g_plain;
    }
  }
  HIPTRY(hipStreamSynchronize(st));
  flush_timed(ctx->prof, st);
  return YAND_OK;
}

// ------------------------------------------------ return-floor protocol --

namespace {

// Linear interpolation between order statistics at (n - 1) q.
double percentile(std::vector<double> v, double q) {
  std::sort(v.begin(), v.end());
  const double h = (double)(v.size() - 1) * q;
  const size_t lo = (size_t)std::floor(h);
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (h - (double)lo) * (v[hi] - v[lo]);
}

struct DeviceVec {
  double* p = nullptr;
  ~DeviceVec() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

int yand_return_floor(yand_ctx* ctx, const double profile[3], double q,
                      const yand_opts* opts_in, int max_rounds,
                      double c_out[4], double* floor_out, double* ret_out,
                      double* w_out, yand_info* info, int* solves_out) {
  if (!ctx || !profile || !w_out || !(q >= 0.0 && q <= 1.0) ||
      max_rounds < 0)
    return YAND_ERR_ARG;
  for (int k = 0; k < 3; ++k)
    if (!(profile[k] >= 0.0) || !std::isfinite(profile[k]))
      return YAND_ERR_ARG;
  yand_opts opts;
  if (opts_in) {
    opts = *opts_in;
  } else {
    yand_default_opts(&opts);
    opts.feasible_set = YAND_SET_SIMPLEX;
  }
  if (opts.feasible_set != YAND_SET_SIMPLEX || !valid_opts(opts))
    return YAND_ERR_ARG;
  const Data& D = ctx->d;
  const int64_t n = D.n;

  double mom[4];
  TRY(equal_weight_moments(ctx, mom));
  double base[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < 3; ++k) {
    if (profile[k] == 0.0) continue;
    if (mom[k + 1] == 0.0) return YAND_ERR_ARG;
    base[k + 1] = profile[k] / std::fabs(mom[k + 1]);
  }
  std::vector<double> mu(n), x(n);
  HIPTRY(hipMemcpyAsync(mu.data(), D.mu, n * sizeof(double),
                        hipMemcpyDeviceToHost, ctx->w.st));
  HIPTRY(hipStreamSynchronize(ctx->w.st));
  const double floor_v = percentile(mu, q);
  const auto mm = std::minmax_element(mu.begin(), mu.end());
  const double spread = *mm.second - *mm.first;
  const double tol = 1e-9 * spread;

  DeviceVec cur;
  HIPTRY(hipMalloc((void**)&cur.p, n * sizeof(double)));

  struct Pt {
    double ret, c1;
  };
  Pt best{0.0, -1.0};
  bool have_best = false;
  yand_info best_info{};
  int solves = 0;

  // One solve from equal weights at the mean coefficient c1; the closest
  // solve so far (ties to the larger c1) is kept in w_out.
  auto run = [&](double c1, Pt* out) -> int {
    double c[4] = {c1, base[1], base[2], base[3]};
    yand_info inf{};
    const int rc = yand_mvsk_solve(ctx, c, nullptr, nullptr, &opts, cur.p,
                                   &inf);
    ++solves;
    if (rc < 0) return rc;
    HIPTRY(hipMemcpy(x.data(), cur.p, n * sizeof(double),
                     hipMemcpyDeviceToHost));
    double r = 0.0;
    for (int64_t i = 0; i < n; ++i) r += mu[i] * x[i];
    out->ret = r;
    out->c1 = c1;
    const double e = std::fabs(r - floor_v), eb = std::fabs(best.ret - floor_v);
    if (!have_best || e < eb || (e == eb && c1 > best.c1)) {
      best = *out;
      best_info = inf;
      have_best = true;
      HIPTRY(hipMemcpy(w_out, cur.p, n * sizeof(double),
                       hipMemcpyDeviceToDevice));
    }
    return YAND_OK;
  };

  Pt lo, hi, mid;
  TRY(run(0.0, &lo));
  if (lo.ret < floor_v && spread > 0.0) {
    TRY(run(1.0 / spread, &hi));
    for (int k = 0; hi.ret < floor_v && k < max_rounds; ++k) {
      lo = hi;
      TRY(run(4.0 * hi.c1, &hi));
    }
    for (int k = 0; hi.ret >= floor_v && std::fabs(best.ret - floor_v) > tol &&
                    k < max_rounds;
         ++k) {
      TRY(run(lo.c1 == 0.0 ? 0.5 * hi.c1 : std::sqrt(lo.c1 * hi.c1), &mid));
      if (mid.ret >= floor_v)
        hi = mid;
      else
        lo = mid;
    }
  }
  if (c_out) {
    c_out[0] = best.c1;
    for (int k = 1; k < 4; ++k) c_out[k] = base[k];
  }
  if (floor_out) *floor_out = floor_v;
  if (ret_out) *ret_out = best.ret;
  if (info) *info = best_info;
  if (solves_out) *solves_out = solves;
  return best_info.status;
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

// ----------------------------------------------------------- autotuner --

int yand_autotune(yand_ctx* ctx, double* report) {
  if (!ctx) return YAND_ERR_ARG;
  Data& D = ctx->d;
  Work& w = ctx->w;
  const hipStream_t st = w.st;
  const double c[4] = {1.0, 5.0, 2.0, 10.0};
  int p0 = 1;
  TRY(setup_lane(D, w, nullptr, nullptr, &p0));
  TRY(oracle_at(D, w, c, w.x, true));
  HIPTRY(launch_grad_project(w.g, w.E, p0, D.n, w.sc, st, -1.0));
  struct Ev {
    hipEvent_t a = nullptr, b = nullptr;
    ~Ev() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } guard;
  HIPTRY(hipEventCreate(&guard.a));
  HIPTRY(hipEventCreate(&guard.b));
  const hipEvent_t e0 = guard.a, e1 = guard.b;
  // mean milliseconds of reps calls of fn on st, after one warm-up call
  auto time_ms = [&](auto&& fn, int reps, double* ms) -> int {
    HIPTRY(fn());
    HIPTRY(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) HIPTRY(fn());
    HIPTRY(hipEventRecord(e1, st));
    HIPTRY(hipEventSynchronize(e1));
    float t = 0.f;
    HIPTRY(hipEventElapsedTime(&t, e0, e1));
    *ms = (double)t / reps;
    return YAND_OK;
  };
  // workgroups per pass: a band of rows per workgroup; more groups hide
  // more latency, fewer write fewer partial rows.  Then the rows per block
  // at that count: taller blocks share one reduction, shorter ones hold
  // fewer registers.
  static const int kCands[] = {256, 384, 512, 768, 1024};
  static const int kRows[] = {1, 2, 4};
  static const PassKind kKinds[6] = {PassKind::Oracle, PassKind::Value,
                                     PassKind::Hvp,    PassKind::Line,
                                     PassKind::Dot,    PassKind::Third};
  double best_ms[7];
  for (int k = 0; k < 6; ++k) {
    PassArgs a = pass_args(D, w, c);
    a.v = w.x;
    switch (kKinds[k]) {
      case PassKind::Oracle:
      case PassKind::Value: a.tout = w.z; break;
      case PassKind::Hvp: a.zc = w.z; break;
      case PassKind::Line: a.zc = w.z; a.tout = w.wv; break;
      case PassKind::Dot: a.tout = w.wv; break;
      case PassKind::Third: a.zc = w.z; a.q = w.q; break;
    }
    best_ms[k] = 1e30;
    D.pass_rows[k] = 0;
    for (int g : kCands) {
      a.groups = g;
      int nwg = 0;
      double ms = 0.0;
      TRY(time_ms([&] { return launch_pass(D.precision, kKinds[k], a, st, &nwg); },
                  5, &ms));
      if (ms < best_ms[k]) {
        best_ms[k] = ms;
        D.pass_groups[k] = g;
      }
    }
    a.groups = D.pass_groups[k];
    const int cap = pass_rows_cap(D.precision, D.lda);
    for (int r : kRows) {
      if (r > cap) break;
      a.rows = r;
      int nwg = 0;
      double ms = 0.0;
      TRY(time_ms([&] { return launch_pass(D.precision, kKinds[k], a, st, &nwg); },
                  5, &ms));
      if (ms < best_ms[k]) {
        best_ms[k] = ms;
        D.pass_rows[k] = r;
      }
    }
  }
  // blocks per group of the two-level Cholesky: deeper group updates touch
  // the trailing matrix less often, shallower groups shorten the steps; then
  // the widths of the in-group update sub-blocks and the panel bands at that
  // group size (narrower pieces spread a short step over more CUs)
  DirOpts o;
  TRY(dir_front(D, w, c, p0, o, nullptr));
  const int64_t n = D.n, np = D.lda;
  auto time_factor = [&](int grp, int tm, int band, double* ms) -> int {
    double total = 0.0;
    for (int rep = 0; rep < 2; ++rep) {
      HIPTRY(launch_project(w.B, w.M, np, n, np, w.E, w.W, p0 + 1, w.sc, st));
      HIPTRY(hipEventRecord(e0, st));
      HIPTRY(launch_potrf_trtri(w.M, w.X, np, &w.sc->fail, st, nullptr, grp,
                                Lanes{}, 1, true, tm, band));
      HIPTRY(hipEventRecord(e1, st));
      HIPTRY(hipEventSynchronize(e1));
      float t = 0.f;
      HIPTRY(hipEventElapsedTime(&t, e0, e1));
      if (rep > 0) total += t;
    }
    *ms = total;
    return YAND_OK;
  };
  best_ms[6] = 1e30;
  D.chol_step_tm = 0;
  D.chol_band = 0;
  for (int grp : {2, 3, 4, 5, 6, 8}) {
    double ms = 0.0;
    TRY(time_factor(grp, 0, 0, &ms));
    if (ms < best_ms[6]) {
      best_ms[6] = ms;
      D.chol_group = grp;
    }
  }
  for (int tm : {32, 64})
    for (int band : {32, 64}) {
      double ms = 0.0;
      TRY(time_factor(D.chol_group, tm, band, &ms));
      if (ms < best_ms[6]) {
        best_ms[6] = ms;
        D.chol_step_tm = tm;
        D.chol_band = band;
      }
    }
  HIPTRY(hipStreamSynchronize(st));
  if (report) {
    int rec[YAND_TUNING_INTS];
    TRY(yand_tuning(ctx, nullptr, rec));
    for (int k = 0; k < YAND_TUNING_INTS; ++k) report[k] = rec[k];
    for (int k = 0; k < 7; ++k) report[YAND_TUNING_INTS + k] = best_ms[k];
  }
  return YAND_OK;
}

int yand_tuning(yand_ctx* ctx, const int* set, int* get) {
  if (!ctx) return YAND_ERR_ARG;
  Data& D = ctx->d;
  if (set) {
    for (int k = 0; k < 6; ++k) {
      if (set[k] < 0 || set[k] > kMaxPassGroups) return YAND_ERR_ARG;
      const int r = set[7 + k];
      if (r != 0 && r != 1 && r != 2 && r != 4) return YAND_ERR_ARG;
    }
    if (set[6] < 0 || set[6] > 64) return YAND_ERR_ARG;
    for (int k = 13; k < 15; ++k)
      if (set[k] != 0 && set[k] != 32 && set[k] != 64) return YAND_ERR_ARG;
    for (int k = 0; k < 6; ++k) {
      D.pass_groups[k] = set[k];
      D.pass_rows[k] = set[7 + k];
    }
    D.chol_group = set[6];
    D.chol_step_tm = set[13];
    D.chol_band = set[14];
  }
  if (get) {
    for (int k = 0; k < 6; ++k) {
      get[k] = D.pass_groups[k];
      get[7 + k] = D.pass_rows[k];
    }
    get[6] = D.chol_group;
    get[13] = D.chol_step_tm;
    get[14] = D.chol_band;
  }
  return YAND_OK;
}

// ------------------------------------------------ allocation-free solve --

}  // extern "C"

namespace {

// Device workspace of yand_mvsk_solve_R_noalloc: one fixed array per device,
// held until the process ends.  Host code never uses the array's name as an
// address: each device's copy is looked up once with hipGetSymbolAddress.
constexpr size_t kScratchBytes = (size_t)256 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_ptr(void** out) {
  int dev = 0;
  HIPTRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return YAND_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPTRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return YAND_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return YAND_OK;
}

// Bytes create_ctx (FP64, n x n buffers up front) takes from an arena: the
// same requests in the same order, each rounded up to 256 bytes.
size_t noalloc_need(int64_t T, int64_t n) {
  const size_t Tp = (size_t)round_up(T, kRowPad),
               lda = (size_t)round_up(n, kColPad), nt = lda / kTile;
  const size_t nb = lda * 8, tb = Tp * 8;
  size_t used = 0;
  auto take = [&](size_t b, int k = 1) {
    for (int i = 0; i < k; ++i)
      used = ((used + 255) & ~(size_t)255) + (b < 256 ? 256 : b);
  };
  take(Tp * lda * 8);                    // A
  take(nb);                              // mu
  take(2 * nb);                          // Efix
  take(2 * tb);                          // AEfix
  take(nb, 3);                           // x, g, d
  take(tb, 3);                           // z, wv, q
  take(3 * tb);                          // AE
  take(3 * nb, 2);                       // E, W
  take(nb, 5);                           // t3, r, y, y2, hv
  take(tb);                              // s_t
  take(nb, 4);                           // PCG vectors
  take(nb, 3);                           // mask, ptmp, hold
  take((size_t)kMaxPassGroups * lda * 8);       // pass partials
  take((size_t)kMaxPassGroups * kMaxSums * 8);  // scalar partials
  take((size_t)kMaxSums * 8);                   // sums
  take((size_t)((n + 63) / 64) * n * 8);        // trmv partials
  take(sizeof(DevScalars));
  take((size_t)((T + 255) / 256) * n * 8);      // column-sum partials
  take(lda * lda * 8, 3);                       // B, M, X
  take(nt * Tp * 8);                            // trace row norms
  return used;
}

struct ArenaScope {
  explicit ArenaScope(Arena* a) { g_arena = a; }
  ~ArenaScope() { g_arena = nullptr; }
};

}  // namespace

extern "C" {

int yand_mvsk_solve_R_noalloc(const double* R, int64_t T, int64_t n,
                              double c1, double c2, double c3, double c4,
                              const double* target, double* w_out) {
  if (!R || !w_out || T < 2 || n < 2) return YAND_ERR_ARG;
  if (n > max_pass_columns(YAND_FP64) ||
      noalloc_need(T, n) > kScratchBytes) {
    fprintf(stderr,
            "libyand: yand_mvsk_solve_R_noalloc: T=%lld n=%lld needs %zu "
            "bytes of workspace; the scratch array holds %zu\n",
            (long long)T, (long long)n,
            n > max_pass_columns(YAND_FP64) ? (size_t)0 : noalloc_need(T, n),
            kScratchBytes);
    return YAND_ERR_TOO_LARGE;
  }
  void* base = nullptr;
  TRY(scratch_ptr(&base));
  Arena arena;
  arena.base = (char*)base;
  arena.cap = kScratchBytes;
  ArenaScope scope(&arena);
  yand_ctx* ctx = nullptr;
  int rc = create_ctx(R, T, n, n, YAND_FP64, nullptr, true, &ctx);
  if (rc) return rc;
  const double c[4] = {c1, c2, c3, c4};
  rc = yand_mvsk_solve(ctx, c, target, nullptr, nullptr, w_out, nullptr);
  yand_destroy(ctx);
  return rc;
}

int yand_profile_enable(yand_ctx* ctx, int enable) {
  if (!ctx) return YAND_ERR_ARG;
  flush_timed(ctx->prof, ctx->w.st);
  ctx->prof.on = enable != 0;
  if (enable) ctx->prof.acc.clear();
  return YAND_OK;
}

int yand_profile_read(yand_ctx* ctx, int index, char* name, int name_len,
                      double* total_ms, int64_t* count) {
  if (!ctx) return YAND_ERR_ARG;
  flush_timed(ctx->prof, ctx->w.st);
  if (index < 0) return (int)ctx->prof.acc.size();
  if (index >= (int)ctx->prof.acc.size()) return YAND_ERR_ARG;
  const auto& p = ctx->prof.acc[index];
  if (name && name_len > 0) {
    std::strncpy(name, p.first.c_str(), name_len - 1);
    name[name_len - 1] = 0;
  }
  if (total_ms) *total_ms = p.second.first;
  if (count) *count = p.second.second;
  return YAND_OK;
}

}  // extern "C"
