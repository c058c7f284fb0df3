// Kernel launchers of libyand (internal).
#pragma once

#include <vector>

#include "common.h"

namespace yand {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename S> struct Vec16;
template <> struct Vec16<double> { static constexpr int N = 2; };
template <> struct Vec16<float> { static constexpr int N = 4; };
template <> struct Vec16<bf16_t> { static constexpr int N = 8; };

template <typename S>
__device__ __forceinline__ void unpack16(const u32x4& raw,
                                         double (&out)[Vec16<S>::N]);
template <>
__device__ __forceinline__ void unpack16<double>(const u32x4& raw,
                                                 double (&out)[2]) {
  out[0] = __hiloint2double((int)raw.y, (int)raw.x);
  out[1] = __hiloint2double((int)raw.w, (int)raw.z);
}
template <>
__device__ __forceinline__ void unpack16<float>(const u32x4& raw,
                                                double (&out)[4]) {
  out[0] = (double)__uint_as_float(raw.x);
  out[1] = (double)__uint_as_float(raw.y);
  out[2] = (double)__uint_as_float(raw.z);
  out[3] = (double)__uint_as_float(raw.w);
}
template <>
__device__ __forceinline__ void unpack16<bf16_t>(const u32x4& raw,
                                                 double (&out)[8]) {
  const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    out[2 * i] = (double)__uint_as_float(w[i] << 16);
    out[2 * i + 1] = (double)__uint_as_float(w[i] & 0xffff0000u);
  }
}

constexpr int kMaxSums = 16;       // scalar partial sums per pass workgroup
constexpr int kMaxPassChunks = 8;  // 16-byte chunks per thread per row

enum class PassKind { Oracle, Value, Hvp, Line, Dot, Third };

struct PassArgs {
  const void* A;        // Tp x lda, storage precision
  int64_t lda;
  int64_t Tp;
  int64_t n;
  int64_t rows_per_wg;  // set by the launcher
  const double* v;      // dot operand (n)
  const double* zc;     // cached z = Ax (Tp)
  const double* q;      // per-row input (Tp)
  double* tout;         // per-row output (Tp), may be null for Hvp/Line
  double* part;         // [nwg][lda] back-projection partials
  double* psums;        // [nwg][kMaxSums] scalar partials
  Coef c;
  double invT;
  const int* skip;      // nonzero: every workgroup returns at once
  int groups;           // workgroups to launch (0: the shape's default)
  int rows;             // rows per block: 1, 2 or 4, capped at the shape's
                        // register budget (0: the shape's default)
};

int pass_groups(int64_t Tp, int R, int groups, int64_t* rows_per_wg);
int64_t max_pass_columns(int precision);
// Largest block height a pass over rows of lda entries runs at (its
// register budget); a larger request runs at this one.
int pass_rows_cap(int precision, int64_t lda);
hipError_t launch_pass(int precision, PassKind kind, const PassArgs& a,
                       hipStream_t st, int* nwg);
hipError_t launch_reduce_partials(const double* part, int nwg, int64_t lda,
                                  int64_t n, double alpha, double beta,
                                  const double* y, double* out,
                                  hipStream_t st, const int* skip = nullptr);
hipError_t launch_reduce_sums(const double* psums, int nwg, int nsum,
                              double* out, hipStream_t st,
                              const int* skip = nullptr);
hipError_t launch_center(const double* R, int64_t T, int64_t n, int64_t ldr,
                         int precision, void* A, int64_t Tp, int64_t lda,
                         double* mu, double* scratch, int* nonfinite,
                         hipStream_t st);

// ---- dense FP64 MFMA kernels (dense.hip) ----------------------------------
constexpr int kTile = 128;  // output tile and Cholesky block size
constexpr int kSlice = 16;  // K depth of one pipelined slice of the products

// Lanes of a grouped launch (blockIdx.y = lane): element strides between
// the lanes' n x n matrices (B, M, X), T-vectors (s), row-norm arrays (rn)
// and int strides between their flags (skip, fail).  All zero with one lane.
struct Lanes {
  int64_t mat = 0, vec = 0, rn = 0, flag = 0;
};

// Balanced SYRK schedule (syrk_split_plan) and its per-lane workspace.
// order: the first rounds x slots (I, J) pairs of syrk_tile_order; plan:
// per workgroup (first piece, piece count), then npieces pieces of
// kSplitPieceInts ints (tile, first and end slice, index of the piece in
// its tile), then ntile2 tiles of kSplitTileInts ints (I, J, pieces, first
// workspace slot; a tile's pieces take consecutive slots) (device, both).
// ws: nslots partial tiles of kTile x kTile doubles per lane (ws_lane
// doubles apart); cnt: ntile2 arrival counters per lane (cnt_lane ints
// apart), zero before the first launch and left at zero by every launch.
constexpr int kSplitPieceInts = 4;
constexpr int kSplitTileInts = 4;
struct SyrkSplit {
  const int* order = nullptr;
  const int* plan = nullptr;
  int slots = 0, rounds = 0, ntile2 = 0, npieces = 0, nslots = 0;
  double* ws = nullptr;
  int64_t ws_lane = 0;
  int* cnt = nullptr;
  int64_t cnt_lane = 0;
};
// Host tables of the balanced schedule (see syrk_split_plan).
struct SyrkPlan {
  std::vector<int> order, plan;
  int slots = 0, rounds = 0, ntile2 = 0, npieces = 0, nslots = 0;
};

// B = A^T diag(s) A (full symmetric n x n, ldb = lda), s length Tp, non-null.
// order (device, nullable): the XCD-aware tile order of syrk_tile_order for
// this lda / kTile, order_slots workgroups (its length / 2).  split
// (nullable, with a workspace): the balanced schedule instead, on
// split->slots workgroups per lane.
hipError_t launch_syrk(int precision, const void* A, int64_t lda, int64_t Tp,
                       const double* s, double* B, hipStream_t st,
                       const int* skip = nullptr, Lanes ls = Lanes{},
                       int nlanes = 1, const int* order = nullptr,
                       int64_t order_slots = 0,
                       const SyrkSplit* split = nullptr);
// (I, J) pairs of the SYRK's lower tiles per workgroup for nt x nt tiles,
// grouped by XCD (-1 for idle slots); empty below 16 tiles (plain order).
std::vector<int> syrk_tile_order(int nt);
// Balanced schedule of the SYRK for nt x nt tiles and ns kSlice-deep
// slices per tile on `slots` resident workgroups (a multiple of the 8
// XCDs): whole tiles of syrk_tile_order for as many full rounds as every
// XCD's list fills; then each XCD's m remaining tiles are shared equally by
// its U workgroups: the first m take the tiles' leading slices (all at the
// same K at the same time, as in a whole round), the other U - m the rest
// of every tile, concatenated.  False when it does not apply (fewer than
// 16 tiles, shares under 16 slices).

bool syrk_split_plan(int nt, int64_t ns, int slots, SyrkPlan* out);
// Resident workgroups of the balanced SYRK kernel on the current device.
int syrk_split_slots();
// In-place Cholesky of the lower triangle of M (np x np, np multiple of
// kTile) and X = L^-1 (lower triangle and the diagonal blocks' upper zeros;
// the tiles above the diagonal blocks are left untouched).  *fail != 0 on exit
// when a pivot was not positive.  fill: the diagonal-block launches also
// carry most of the previous group update on the CUs they leave idle, shared
// equally among the lanes (the same results; meant for a stream that has the
// device to itself, since those launches then take every CU).  step_tm: sub-
// block width of the in-group updates, fin_band: band width of the panel
// step (32 or 64 each, 0: 32); every choice gives bit-identical L and X,
// since each entry is the same product over the same reduction order.
hipError_t launch_potrf_trtri(double* M, double* X, int64_t np, int* fail,
                              hipStream_t st, const int* skip = nullptr,
                              int group = 0, Lanes ls = Lanes{},
                              int nlanes = 1, bool fill = false,
                              int step_tm = 0, int fin_band = 0);
// Sets the LDS attribute of the diagonal-block kernel (call before capture).
hipError_t prepare_dense_kernels();
// rn[J][t] = sum_{j in tile J} (sum_k A[t][k] X[j][k])^2  (X lower)
hipError_t launch_trace_gemm(int precision, const void* A, int64_t lda,
                             int64_t Tp, const double* X, int64_t np,
                             double* rn, hipStream_t st,
                             const int* skip = nullptr, Lanes ls = Lanes{},
                             int nlanes = 1);
// ---- FP32 / BF16 matrix-core variants (lowp.hip), precision 1 or 2 ------
// At (lda x Tp) = A^T at the storage precision.
hipError_t launch_transpose_lp(int precision, const void* A, int64_t lda,
                               int64_t Tp, void* At, hipStream_t st);
// B = A^T diag(s) A from At: SAt (np x Tp x 4 bytes scratch) = s-scaled At
// (BF16: high and low parts), then FP32-accumulated products; B (np x np,
// FP64) exactly symmetric.  order (device, nullable): the XCD-aware tile
// order of syrk_tile_order, order_slots workgroups.
hipError_t launch_syrk_lp(int precision, const void* At, void* SAt,
                          int64_t np, int64_t Tp, const double* s, double* B,
                          hipStream_t st, const int* skip = nullptr,
                          const int* order = nullptr,
                          int64_t order_slots = 0);
// rn as launch_trace_gemm from X rounded into Xl (np x np x 4 bytes
// scratch; BF16: high and low parts).
hipError_t launch_trace_lp(int precision, const void* A, int64_t lda,
                           int64_t Tp, const double* X, int64_t np, void* Xl,
                           double* rn, hipStream_t st,
                           const int* skip = nullptr);
// ---- block passes (dense.hip): kb <= 64 vectors at once -----------------
constexpr int kBlockWidth = 64;
// Split counts of the two block products for this shape: *sv splits of the
// n-side reduction of Z = A V, *sz of the T-side one of A^T Z.  Partial
// slabs: sv x Tp x 64 and sz x 64 x lda doubles.
int block_splits(int64_t Tp, int64_t lda, int* sv, int* sz);
// Z (Tp x 64, row-major) = A V, V 64 x lda (row j = vector j); Zp partials.
hipError_t launch_block_av(int precision, const void* A, int64_t lda,
                           int64_t Tp, const double* V, double* Zp, double* Z,
                           hipStream_t st, const int* skip = nullptr);
// Y (64 x lda, row j = vector j) = (A^T diag(s) Z)^T (s nullable = 1).
hipError_t launch_block_atz(int precision, const void* A, int64_t lda,
                            int64_t Tp, const double* Z, const double* s,
                            double* Yp, double* Y, hipStream_t st,
                            const int* skip = nullptr);
// ---- probe estimate of the trace (probe.hip) -----------------------------
struct DevScalars;
// Xi (Tp x 64): SplitMix64 signs for t < T, j < k; zero elsewhere.
hipError_t launch_rademacher(uint64_t seed, uint64_t draw, int64_t T,
                             int64_t Tp, int k, double* Xi, hipStream_t st);
// sc->lambda = reg * tangent trace of B / (free coordinates - p).
hipError_t launch_probe_scale(const double* bd, int64_t n, const double* s,
                              const double* AE, int64_t T, int64_t Tp, int p,
                              double reg, const double* mask, DevScalars* sc,
                              hipStream_t st);
// Block PCG over the 64 columns (rows of the 64 x ld arrays); columns >= k
// are done at once.  flags: [0] all done, [1 + j] done, [65 + j]
// iterations, [129] total iterations; cs: 8 doubles per column.
hipError_t launch_bpcg_init(const double* U, const double* bd, const double* E,
                            int p, int64_t n, int64_t ld, int k, double* Y,
                            double* Rr, double* Z, double* P, double* cs,
                            int* flags, const DevScalars* sc,
                            const double* mask, hipStream_t st);
hipError_t launch_bpcg_update(const double* HP, const double* bd,
                              const double* E, int p, int64_t n, int64_t ld,
                              double* Y, double* Rr, double* Z, double* P,
                              double* AP, double* cs, int* flags,
                              const DevScalars* sc, const double* mask,
                              double tol, hipStream_t st);
// C = alpha op(A) op(B) + beta C in FP64 on the matrix cores (C: M x N,
// row-major, ldc); op(A) is M x K (A row-major, or its transpose when at),
// op(B) K x N (B row-major, or its transpose when bt).  M and N must be
// multiples of 128 and K of 16 (invalid value otherwise); beta = 0 does not
// read C.
hipError_t launch_gemm64(const double* A, int64_t lda, bool at,
                         const double* B, int64_t ldb, bool bt, double* C,
                         int64_t ldc, int64_t M, int64_t N, int64_t K,
                         double alpha, double beta, hipStream_t st);
// ZS[t][l] = Z[t][l] * s[l * vec + t] for l < nl, 0 for nl <= l < 64
// (Z, ZS: Tp x 64 row-major): per-lane row weights of a batched Hessian
// product.  nl outside [1, 64] is an invalid value.
hipError_t launch_lane_scale(const double* Z, const double* s, int64_t vec,
                             int nl, int64_t Tp, double* ZS, hipStream_t st,
                             const int* skip = nullptr);
// q_t = k^-1 sum_j Xi_tj Q_tj (zero for t >= T).
hipError_t launch_probe_q(const double* Xi, const double* Q, int64_t T,
                          int64_t Tp, int k, double* q, hipStream_t st);
// y = X v (lower), y = X^T v (transposed); X is np x np, 16-byte aligned
// with np even (rows are read two entries at a time).  part holds
// ceil(n/64) * n doubles of partial sums for the transposed product.
hipError_t launch_trmv(const double* X, int64_t np, int64_t n,
                       const double* v, double* y, double* part, bool trans,
                       hipStream_t st, const int* skip = nullptr);
// W[:, a] = B E[:, a] for a < p <= 3 (E is n x p column-major with ld n;
// B 16-byte aligned with ldb even).
hipError_t launch_symm_multi(const double* B, int64_t ldb, int64_t n,
                             const double* E, int p, double* W,
                             hipStream_t st, const int* skip = nullptr);


// ---- T < n push-through of the exact trace (thin.hip) ----
struct DevScalars;
// Column splits of the Gram kernel for T rows (1..64, partials <= 64 MiB).
int thin_splits(int64_t T);
// Workspace (doubles) of the indefinite push-through factorisation for T.
int64_t thin_indef_doubles(int64_t T);
// Indefinite S (np_ bars with s > 0, T - np_ >= 1 with s < 0): the signed
// factorisation of W = lambda S^-1 + G (G lower, ld ldg) with lambda from
// sc; sc->fail is raised when it does not exist (B_m not positive
// definite).  ws: thin_indef_doubles(T) doubles, kept for launch_thin_indef_q.
hipError_t launch_thin_indef_factor(const double* G, int64_t ldg, int64_t T,
                                    const double* s, int np_, int chol_group,
                                    DevScalars* sc, double* ws,
                                    hipStream_t st);
// q (Tp, zero padding) from that factorisation.
hipError_t launch_thin_indef_q(int64_t T, int64_t Tp, const double* s,
                               int np_, const DevScalars* sc, double* ws,
                               double* q, hipStream_t st);
// Rows of the partial-sum scratch (each ld long) that launch_thin_q
// (ld = ldg) and launch_bdiag (ld = lda) need for T rows.
int64_t thin_part_rows(int64_t T);
// G = A diag(mask) A^T - sum_{a<p} (A e_a)(A e_a)^T, lower triangle of the
// T x T leading block of G (ld ldg); Gp holds K x ldg x ldg partials.
hipError_t launch_thin_gram(int precision, const void* A, int64_t lda,
                            int64_t T, int64_t n, const double* mask, int K,
                            double* Gp, int64_t ldg, const double* AE,
                            int64_t Tp, int p, double* G, hipStream_t st);
// Scales (lambda, gamma, trace, ptbad) into sc and the lower triangle of
// C = S^1/2 G S^1/2 + lambda I (identity padding to ldg).
hipError_t launch_thin_factor_input(const double* G, int64_t ldg, int64_t T,
                                    const double* s, const double* AE,
                                    int64_t Tp, int p, int64_t n, double reg,
                                    const double* mask, DevScalars* sc,
                                    double* C, hipStream_t st);
// q_t = (1 - lambda (C^-1)_tt) / s_t from X = L^-1 (ld ldg); 0 for t >= T.
// part: thin_part_rows(T) x ldg scratch.
hipError_t launch_thin_q(const double* X, int64_t ldg, int64_t T, int64_t Tp,
                         const double* s, const DevScalars* sc, double* part,
                         double* q, hipStream_t st);
// bd_j = sum_t s_t A_tj^2.  part: thin_part_rows(T) x lda scratch.
hipError_t launch_bdiag(int precision, const void* A, int64_t lda, int64_t T,
                        int64_t n, const double* s, double* part, double* bd,
                        hipStream_t st);

}  // namespace yand
