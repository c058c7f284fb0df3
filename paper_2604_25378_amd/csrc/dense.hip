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
#include <algorithm>
#include <array>

#include "common.h"
#include "kernels.h"

namespace yand {
namespace {

constexpr int BM = kTile;
constexpr int BKK = kSlice;
constexpr int NT = 256;
// Output tiles are TM x TN (128 x 128, or 64-wide for the short launches on
// the critical path of the factorisation).
// LDS row pitch of the k-major slices: TM + 16 doubles, so the four k-rows
// one MFMA operand read touches start 32 banks apart and each half-wave
// reads 64 distinct banks.
template <int TM>
constexpr int ldp() { return TM + 16; }
constexpr int LDP = ldp<BM>();

// LDS layouts of one BKK-deep slice of a 128-wide operand:
//  - operand contiguous in m in memory (KC = false): k-major, s[k * LDP + m];
//  - operand contiguous in k (KC = true): m-major, s[m * LDK + k] with
//    LDK = BKK + 1, which keeps both the 16-byte row stores and the MFMA
//    operand reads (16 rows x 4 k per instruction) spread over the banks.
constexpr int LDK = BKK + 1;
// one k-slice of one operand, in either layout
template <int TM>
constexpr int stage_size() {
  return TM * LDK > BKK * ldp<TM>() ? TM * LDK : BKK * ldp<TM>();
}
constexpr int kStage = stage_size<BM>();

template <bool KC, int TM = BM>
__device__ __forceinline__ int lds_at(int m, int k) {
  return KC ? m * LDK + k : k * ldp<TM>() + m;
}

// One BKK-deep slice of one operand, moved global -> registers -> LDS in
// 16-byte chunks (PER per thread).  KC: element (m, k) at base[m * ld + k];
// otherwise at base[k * ld + m].  SC: the operand is scaled by scale[k]
// (KC = false only); each chunk's factor is fetched with the chunk.
template <typename T, bool KC, int TM = BM, bool SC = false>
struct Stage {
  static_assert(!(SC && KC), "scaled operands are stored k-major");
  static constexpr int VEC = Vec16<T>::N;
  static constexpr int PER = TM * BKK / VEC / NT;
  static_assert(PER >= 1, "slice smaller than the workgroup");
  u32x4 r[PER];
  double sc[PER];

  __device__ __forceinline__ void chunk_at(int i, int tid, int* m, int* k) const {
    const int idx = tid + i * NT;
    if constexpr (KC) {
      constexpr int CPR = BKK / VEC;
      *m = idx / CPR;
      *k = (idx % CPR) * VEC;
    } else {
      constexpr int CPR = TM / VEC;
      *k = idx / CPR;
      *m = (idx % CPR) * VEC;
    }
  }

  __device__ __forceinline__ void load1(int i, const T* base, int64_t ld,
                                        int64_t k0, const double* scale,
                                        int tid) {
    int m, k;
    chunk_at(i, tid, &m, &k);
    const T* p = KC ? base + (int64_t)m * ld + k0 + k : base + (k0 + k) * ld + m;
    r[i] = *(const u32x4*)p;
    if constexpr (SC) sc[i] = scale[k0 + k];
  }

  __device__ __forceinline__ void store1(int i, double* s, int tid) const {
    int m, k;
    chunk_at(i, tid, &m, &k);
    double x[VEC];
    unpack16<T>(r[i], x);
    if constexpr (KC) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) s[lds_at<true, TM>(m, k + e)] = x[e];
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        s[lds_at<false, TM>(m + e, k)] = SC ? x[e] * sc[i] : x[e];
    }
  }

  __device__ __forceinline__ void load(const T* base, int64_t ld, int64_t k0,
                                       const double* scale, int tid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) load1(i, base, ld, k0, scale, tid);
  }
  __device__ __forceinline__ void store(double* s, int tid) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) store1(i, s, tid);
  }
};

// The memory operations of one slice of the pipeline, in issue order:
// chunk c of A to LDS, chunk c of B to LDS, then the next-but-one slice's
// chunk c of A and of B into the freed registers.  Operation q runs after
// MFMA group q * G / NOPS, so every chunk waits a full slice between its
// load and its store.
template <int PA, int PB>
struct PipeOps {
  static constexpr int N = 2 * PA + 2 * PB;
  // kind: 0 store A, 1 store B, 2 load A, 3 load B; chunk index in *c
  static constexpr int kind(int q, int* c) {
    int o = 0;
    for (int ch = 0; ch < (PA > PB ? PA : PB); ++ch)
      for (int kd = 0; kd < 4; ++kd) {
        const bool isA = kd == 0 || kd == 2;
        if (ch >= (isA ? PA : PB)) continue;
        if (o == q) {
          *c = ch;
          return kd;
        }
        ++o;
      }
    return -1;
  }
};

// One slice: MFMAs on the LDS buffers (rA, rB), the next k-step's fragments
// read while the current ones are multiplied; STORE writes the slice held in
// registers to (wA, wB), LOAD fetches the slice at kl into the registers.
// Each group of NB MFMAs (one A fragment) is followed by the memory
// operations that fall on it; scheduling barriers keep that interleaving.
template <bool STORE, bool LOAD, typename TA, bool AKC, typename TB, bool BKC,
          int TM, int TN, bool BS>
__device__ __forceinline__ void core_slice(
    const double* rA, const double* rB, double* wA, double* wB,
    Stage<TA, AKC, TM>& sa, Stage<TB, BKC, TN, BS>& sb, const TA* Ab,
    int64_t lda, const TB* Bb, int64_t ldb, const double* bscale, int64_t kl,
    f64x4 (&acc)[TM / 32][TN / 32], int wm, int wn, int lane, int tid) {
  constexpr int MB = TM / 32, NB = TN / 32, G = 4 * MB;
  using Ops = PipeOps<Stage<TA, AKC, TM>::PER, Stage<TB, BKC, TN, BS>::PER>;
  const int c = lane & 15, kq = lane >> 4;
  double a[MB], b[NB];
#pragma unroll
  for (int i = 0; i < MB; ++i) a[i] = rA[lds_at<AKC, TM>(wm + i * 16 + c, kq)];
#pragma unroll
  for (int j = 0; j < NB; ++j) b[j] = rB[lds_at<BKC, TN>(wn + j * 16 + c, kq)];
#pragma unroll
  for (int t = 0; t < BKK / 4; ++t) {
    double an[MB], bn[NB];
    if (t + 1 < BKK / 4) {
      const int kr = 4 * (t + 1) + kq;
#pragma unroll
      for (int i = 0; i < MB; ++i) an[i] = rA[lds_at<AKC, TM>(wm + i * 16 + c, kr)];
#pragma unroll
      for (int j = 0; j < NB; ++j) bn[j] = rB[lds_at<BKC, TN>(wn + j * 16 + c, kr)];
    }
#pragma unroll
    for (int i = 0; i < MB; ++i) {
#pragma unroll
      for (int j = 0; j < NB; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j],
                                                         0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      const int g = t * MB + i;
#pragma unroll
      for (int q = 0; q < Ops::N; ++q) {
        if (q * G / Ops::N != g) continue;
        int ch = 0;
        const int kd = Ops::kind(q, &ch);
        if (STORE && kd == 0) sa.store1(ch, wA, tid);
        if (STORE && kd == 1) sb.store1(ch, wB, tid);
        if (LOAD && kd == 2) sa.load1(ch, Ab, lda, kl, nullptr, tid);
        if (LOAD && kd == 3) sb.load1(ch, Bb, ldb, kl, bscale, tid);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (t + 1 < BKK / 4) {
#pragma unroll
      for (int i = 0; i < MB; ++i) a[i] = an[i];
#pragma unroll
      for (int j = 0; j < NB; ++j) b[j] = bn[j];
    }
  }
}

// acc (this wave's TM/2 x TN/2 block) = sum_{k in [kbeg, kend)} opA(m,k) opB(k,n),
// opB scaled by bscale[k] when BS.  kend - kbeg must be a multiple of BKK.
// sA, sB hold two k-slices each (double buffer): slice s is multiplied from
// buffer s % 2 while slice s + 1 moves from registers into the other buffer
// and slice s + 2 is fetched into the registers, both interleaved with the
// MFMAs; one barrier per slice.  LDS is free again on return.
template <typename TA, bool AKC, typename TB, bool BKC, int TM = BM,
          int TN = TM, bool BS = false>
__device__ void gemm_core(const TA* Ab, int64_t lda, const TB* Bb,
                          int64_t ldb, const double* bscale, int64_t kbeg,
                          int64_t kend, f64x4 (&acc)[TM / 32][TN / 32],
                          double* sA, double* sB,
                          int tid = (int)threadIdx.x) {
  constexpr int MB = TM / 32, NB = TN / 32;
  constexpr int STA = stage_size<TM>(), STB = stage_size<TN>();
  const int lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * (TM / 2), wn = (w & 1) * (TN / 2);
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (kbeg >= kend) return;
  const int64_t ns = (kend - kbeg) / BKK;
  Stage<TA, AKC, TM> sa;
  Stage<TB, BKC, TN, BS> sb;
  sa.load(Ab, lda, kbeg, nullptr, tid);
  sb.load(Bb, ldb, kbeg, bscale, tid);
  sa.store(sA, tid);
  sb.store(sB, tid);
  if (ns > 1) {
    // same chunk order as the loads inside the loop, so that the wait
    // counts the compiler derives at the loop head stay exact
    using Ops = PipeOps<Stage<TA, AKC, TM>::PER, Stage<TB, BKC, TN, BS>::PER>;
#pragma unroll
    for (int q = 0; q < Ops::N; ++q) {
      int ch = 0;
      const int kd = Ops::kind(q, &ch);
      if (kd == 2) sa.load1(ch, Ab, lda, kbeg + BKK, nullptr, tid);
      if (kd == 3) sb.load1(ch, Bb, ldb, kbeg + BKK, bscale, tid);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();
  int64_t si = 0;
  for (; si + 2 < ns; ++si) {
    const int b = (int)(si & 1);
    const int64_t k0 = kbeg + si * BKK;
    core_slice<true, true>(sA + b * STA, sB + b * STB, sA + (b ^ 1) * STA,
                           sB + (b ^ 1) * STB, sa, sb, Ab, lda, Bb, ldb, bscale,
                           k0 + 2 * BKK, acc, wm, wn, lane, tid);
    __syncthreads();
  }
  if (si + 1 < ns) {
    const int b = (int)(si & 1);
    const int64_t k0 = kbeg + si * BKK;
    core_slice<true, false>(sA + b * STA, sB + b * STB, sA + (b ^ 1) * STA,
                            sB + (b ^ 1) * STB, sa, sb, Ab, lda, Bb, ldb,
                            bscale, 0, acc, wm, wn, lane, tid);
    __syncthreads();
    ++si;
  }
  {
    const int b = (int)(si & 1);
    core_slice<false, false>(sA + b * STA, sB + b * STB, nullptr, nullptr, sa,
                             sb, Ab, lda, Bb, ldb, bscale, 0, acc, wm, wn, lane,
                             tid);
    __syncthreads();
  }
}

// Visit this wave's accumulator entries as (row, col) inside the TM x TN
// tile: D[row][col] of 16x16x4 f64 MFMA block (i, j) is held by lane l in
// register r with row = l / 16 + 4 r and col = l % 16 (gfx950 layout).
template <int TM = BM, int TN = TM, class F>
__device__ __forceinline__ void for_each_acc(
    const f64x4 (&acc)[TM / 32][TN / 32], F f) {
  constexpr int MB = TM / 32, NB = TN / 32;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * (TM / 2), wn = (w & 1) * (TN / 2);
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
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
// Tile (I, J) of B and, off the diagonal, its mirror (J, I).
__device__ __forceinline__ void syrk_store(double* B, int64_t ld, int I, int J,
                                           const f64x4 (&acc)[4][4]) {
  double* Bij = B + (int64_t)I * BM * ld + (int64_t)J * BM;
  double* Bji = B + (int64_t)J * BM * ld + (int64_t)I * BM;
  const bool mirror = I != J;
  for_each_acc(acc, [&](int r, int c, double v) {
    Bij[(int64_t)r * ld + c] = v;
    if (mirror) Bji[(int64_t)c * ld + r] = v;
  });
}

// B = A^T diag(s) A, lower tiles computed, written to both triangles.
template <typename S>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
syrk_kernel(const S* __restrict__ A, int64_t lda, int64_t Tp,
            const double* __restrict__ s, double* __restrict__ B,
            const int* skip, Lanes ls, const int* __restrict__ order) {
  const int ln = blockIdx.y;
  s += ln * ls.vec;
  B += ln * ls.mat;
  if (skip) skip += ln * ls.flag;
  if (skip && *skip) return;
  __shared__ double sA[2 * kStage], sB[2 * kStage];
  int I, J;
  if (order) {
    I = order[2 * blockIdx.x];
    J = order[2 * blockIdx.x + 1];
    if (I < 0) return;
  } else {
    lower_tile(blockIdx.x, &I, &J);
  }
  f64x4 acc[4][4];
  gemm_core<S, false, S, false, BM, BM, true>(
      A + (int64_t)I * BM, lda, A + (int64_t)J * BM, lda, s, 0, Tp, acc, sA, sB);
  syrk_store(B, lda, I, J, acc);
}

// Balanced SYRK (stream-K).  The grid holds one workgroup per resident slot
// (blockIdx.x = slot, slot % 8 its XCD).  Each workgroup first computes
// `rounds` whole tiles of the XCD-aware order, then its pieces of the tiles
// left on its XCD (see syrk_split_plan).  A tile cut into several pieces is
// completed by the workgroup whose piece arrives last (arrival counter):
// every piece is published to the workspace, and the last one adds them
// all up from there in piece order (ascending K), so the sum does not
// depend on the order of arrival, and resets the counter for the next
// launch.  Nothing waits on another workgroup.
template <typename S>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
syrk_split_kernel(const S* __restrict__ A, int64_t lda, int64_t Tp,
                  const double* __restrict__ s, double* __restrict__ B,
                  const int* skip, Lanes ls, const int* __restrict__ order,
                  int rounds, const int* __restrict__ plan, int npieces,
                  double* ws, int64_t ws_lane, int* cnt, int64_t cnt_lane) {
  const int ln = blockIdx.y;
  s += ln * ls.vec;
  B += ln * ls.mat;
  ws += ln * ws_lane;
  cnt += ln * cnt_lane;
  if (skip) skip += ln * ls.flag;
  if (skip && *skip) return;
  __shared__ double sA[2 * kStage], sB[2 * kStage];
  __shared__ int last;
  const int wg = blockIdx.x, slots = gridDim.x, tid = threadIdx.x;
  const int first = plan[2 * wg], count = plan[2 * wg + 1];
  const int* pieces = plan + 2 * slots;
  const int* tiles = pieces + npieces * kSplitPieceInts;
  constexpr int64_t kTileD = (int64_t)BM * BM;
  f64x4 acc[4][4];
  // jobs [0, rounds): whole tiles; then this workgroup's pieces
  for (int job = 0; job < rounds + count; ++job) {
    int I, J, np = 1, t = 0;
    int64_t kb = 0, ke = Tp;
    const int* tt = nullptr;
    const int* pc = nullptr;
    if (job < rounds) {
      I = order[2 * (job * slots + wg)];
      J = order[2 * (job * slots + wg) + 1];
      if (I < 0) continue;
    } else {
      pc = pieces + (first + job - rounds) * kSplitPieceInts;
      t = pc[0];
      tt = tiles + t * kSplitTileInts;
      I = tt[0];
      J = tt[1];
      np = tt[2];
      kb = (int64_t)pc[1] * BKK;
      ke = (int64_t)pc[2] * BKK;
    }
    // the thread index made opaque per job, so that the products' index
    // arithmetic is not hoisted out of the loop (it would stay live across
    // the jobs and spill)
    int tj = tid;
    asm volatile("" : "+v"(tj));
    gemm_core<S, false, S, false, BM, BM, true>(A + (int64_t)I * BM, lda,
                                                A + (int64_t)J * BM, lda, s,
                                                kb, ke, acc, sA, sB, tj);
    if (np > 1) {
      // publish this piece, thread-major (coalesced for writer and reader)
      double* mine = ws + (int64_t)(tt[3] + pc[3]) * kTileD;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            mine[(int64_t)((i * 4 + j) * 4 + r) * NT + tid] = acc[i][j][r];
      __threadfence();
      __syncthreads();
      if (tid == 0) last = atomicAdd(cnt + t, 1) == np - 1;
      __syncthreads();
      if (!last) continue;
      __threadfence();
      // the tile's entries, each summed over the pieces in piece order;
      // EB entries at a time so that their loads are in flight together
      // (a wait for loads also waits for the stores issued before them)
      const int lane = tid & 63, w = tid >> 6;
      const int wm = (w >> 1) * (BM / 2), wn = (w & 1) * (BM / 2);
      double* Bij = B + (int64_t)I * BM * lda + (int64_t)J * BM;
      double* Bji = B + (int64_t)J * BM * lda + (int64_t)I * BM;
      const double* w0 = ws + (int64_t)tt[3] * kTileD + tid;
      constexpr int EB = 16;
#pragma unroll 1
      for (int e0 = 0; e0 < 64; e0 += EB) {
        double v[EB];
#pragma unroll
        for (int u = 0; u < EB; ++u) v[u] = w0[(int64_t)(e0 + u) * NT];
#pragma unroll 1
        for (int p = 1; p < np; ++p) {
          const double* wp = w0 + (int64_t)p * kTileD;
          double x[EB];
#pragma unroll
          for (int u = 0; u < EB; ++u) x[u] = wp[(int64_t)(e0 + u) * NT];
#pragma unroll
          for (int u = 0; u < EB; ++u) v[u] += x[u];
        }
#pragma unroll
        for (int u = 0; u < EB; ++u) {
          const int e = e0 + u;
          const int rr = wm + (e >> 4) * 16 + (lane >> 4) + 4 * (e & 3);
          const int cc = wn + ((e >> 2) & 3) * 16 + (lane & 15);
          Bij[(int64_t)rr * lda + cc] = v[u];
          if (I != J) Bji[(int64_t)cc * lda + rr] = v[u];
        }
      }
      if (tid == 0) cnt[t] = 0;
      continue;
    }
    syrk_store(B, lda, I, J, acc);
  }
}

// ------------------------------------------------------- trace row norms --
// rn[J][t] = sum_{j in tile J} (sum_k A[t][k] X[j][k])^2 for X lower.
template <typename S>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
trace_gemm_kernel(const S* __restrict__ A, int64_t lda, int64_t Tp,
                  const double* __restrict__ X, int64_t ldx,
                  double* __restrict__ rn, const int* skip, Lanes ls) {
  const int ln = blockIdx.y;
  X += ln * ls.mat;
  rn += ln * ls.rn;
  if (skip) skip += ln * ls.flag;
  if (skip && *skip) return;
  __shared__ double sA[2 * kStage], sB[2 * kStage];
  __shared__ double rows[2][BM];
  // Longest reductions first (J descending), so the short ones fill the
  // tail.  The row-tile count is padded to a multiple of 8 so that row tile
  // t always lands on XCD t mod 8 (workgroups go round-robin over the 8
  // XCDs): the column tiles sharing rows of A then share one L2.
  const int ntt = (int)(Tp / BM), ntp = (ntt + 7) / 8 * 8;
  const int nJ = gridDim.x / ntp;
  const int ti = (int)blockIdx.x % ntp;
  if (ti >= ntt) return;
  const int J = nJ - 1 - (int)blockIdx.x / ntp;
  const int64_t t0 = (int64_t)ti * BM;
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

// ------------------------------------------------- block passes over A --
// Products of A with a block of kb <= 64 vectors at once (the probe solves
// of the trace estimate): Z = A V and Y = A^T diag(s) Z as two FP64 MFMA
// GEMMs with 128 x 64 output tiles.  A has few 128-row tiles along the output
// side of each product, so the reduction dimension is split over
// workgroups; every split writes its own partial slab and a second kernel
// sums the slabs in split order (deterministic).
//  V and Y: 64 x lda, column j of the block contiguous (row j of the array);
//  Z: Tp x 64 row-major (bar t's 64 values contiguous).
constexpr int BW = 64;  // block width

template <typename S>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
block_av_kernel(const S* __restrict__ A, int64_t lda, const double* __restrict__ V,
                int64_t kchunk, double* __restrict__ Zp, int64_t Tp,
                const int* skip) {
  if (skip && *skip) return;
  __shared__ double sA[2 * stage_size<BM>()], sB[2 * stage_size<BW>()];
  const int ntt = (int)(Tp / BM);
  const int ti = (int)blockIdx.x % ntt, sp = (int)blockIdx.x / ntt;
  const int64_t t0 = (int64_t)ti * BM, k0 = (int64_t)sp * kchunk;
  const int64_t k1 = k0 + kchunk < lda ? k0 + kchunk : lda;
  f64x4 acc[BM / 32][BW / 32];
  gemm_core<S, true, double, true, BM, BW>(A + t0 * lda, lda, V, lda, nullptr,
                                           k0, k1, acc, sA, sB);
  double* out = Zp + (int64_t)sp * Tp * BW + t0 * BW;
  for_each_acc<BM, BW>(acc, [&](int r, int c, double v) {
    out[(int64_t)r * BW + c] = v;
  });
}

template <typename S, bool SCALE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
block_atz_kernel(const S* __restrict__ A, int64_t lda, int64_t Tp,
                 const double* __restrict__ Z, const double* __restrict__ s,
                 int64_t tchunk, double* __restrict__ Yp, const int* skip) {
  if (skip && *skip) return;
  __shared__ double sA[2 * stage_size<BM>()], sB[2 * stage_size<BW>()];
  const int njt = (int)(lda / BM);
  const int jt = (int)blockIdx.x % njt, sp = (int)blockIdx.x / njt;
  const int64_t j0 = (int64_t)jt * BM, k0 = (int64_t)sp * tchunk;
  const int64_t k1 = k0 + tchunk < Tp ? k0 + tchunk : Tp;
  f64x4 acc[BM / 32][BW / 32];
  gemm_core<S, false, double, false, BM, BW, SCALE>(A + j0, lda, Z, BW, s, k0,
                                                    k1, acc, sA, sB);
  double* out = Yp + (int64_t)sp * BW * lda + j0;
  for_each_acc<BM, BW>(acc, [&](int r, int c, double v) {
    out[(int64_t)c * lda + r] = v;
  });
}

// out[i] = sum_{p < parts} part[p * len + i], parts summed in order.
__global__ void sum_slabs_kernel(const double* __restrict__ part, int parts,
                                 int64_t len, double* __restrict__ out,
                                 const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int p = 0; p < parts; ++p) v += part[(int64_t)p * len + i];
    out[i] = v;
  }
}

// General FP64 product C = alpha op(A) op(B) + beta C in 128 x 128 tiles
// (one per workgroup): op(A)(m, k) = A[m * lda + k], or A[k * lda + m] when
// transposed (AKC false); op(B)(k, n) = B[k * ldb + n], or B[n * ldb + k]
// when transposed (BKC true).  M, N multiples of 128, K of 16.
template <bool AKC, bool BKC>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
gemm64_kernel(const double* __restrict__ A, int64_t lda,
              const double* __restrict__ B, int64_t ldb, double* C,
              int64_t ldc, int64_t K, int ntn, double alpha, double beta) {
  __shared__ double sA[2 * stage_size<BM>()], sB[2 * stage_size<BM>()];
  const int64_t m0 = (int64_t)(blockIdx.x / ntn) * BM;
  const int64_t n0 = (int64_t)(blockIdx.x % ntn) * BM;
  const double* Ab = AKC ? A + m0 * lda : A + m0;
  const double* Bb = BKC ? B + n0 * ldb : B + n0;
  f64x4 acc[BM / 32][BM / 32];
  gemm_core<double, AKC, double, BKC, BM, BM>(Ab, lda, Bb, ldb, nullptr, 0, K,
                                              acc, sA, sB);
  if (beta == 0.0) {
    for_each_acc<BM, BM>(acc, [&](int r, int c, double v) {
      C[(m0 + r) * ldc + n0 + c] = alpha * v;
    });
    return;
  }
  // with beta: each 16-row block's reads before its writes (a wait for a
  // load also waits for the stores before it)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * (BM / 2), wn = (w & 1) * (BM / 2);
#pragma unroll
  for (int i = 0; i < BM / 32; ++i) {
    double old[BM / 32][4];
#pragma unroll
    for (int j = 0; j < BM / 32; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        old[j][r] = C[(m0 + wm + i * 16 + (lane >> 4) + 4 * r) * ldc + n0 +
                      wn + j * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < BM / 32; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        C[(m0 + wm + i * 16 + (lane >> 4) + 4 * r) * ldc + n0 + wn + j * 16 +
          (lane & 15)] = alpha * acc[i][j][r] + beta * old[j][r];
  }
}

// ZS[t][l] = Z[t][l] s_l[t] for lanes l < nl (s_l at s + l * vec), 0 for
// the block's unused columns: the per-lane weights of a batched Hessian
// product A^T diag(s_l) A v_l.
__global__ void lane_scale_kernel(const double* __restrict__ Z,
                                  const double* __restrict__ s, int64_t vec,
                                  int nl, int64_t Tp, double* __restrict__ ZS,
                                  const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
       i < Tp * BW; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = i / BW;
    const int l = (int)(i % BW);
    ZS[i] = l < nl ? Z[i] * s[(int64_t)l * vec + t] : 0.0;
  }
}

// ------------------------------------------------------ blocked Cholesky --
// Diagonal block k: Cholesky factor L_kk of the 128 x 128 block and its
// inverse X_kk = L_kk^-1, computed in LDS by one workgroup of 8 waves.
//
// LDS layout (128 rows of LDD doubles): L in the lower triangle (diagonal
// included); the strictly lower part of X stored transposed in the strict
// upper triangle (X[i][j], i > j, at row j, column i); 1/L_ii in rdiag.
//
// Factorisation: right-looking in 16-column steps.  Waves 0 and 1 factor
// each panel (the 16 columns from the diagonal down) in registers, 64 rows
// below the leaf each, the leaf's values moving between lanes by DPP row
// broadcasts.  The trailing update A22 -= L21 L21^T runs on the FP64 matrix
// cores: first the next panel's blocks, one per wave, then the rest on the
// other waves while the panel is factored.
// Inverse: the eight leaves in parallel (one wave each), then recursive
// doubling, X21 = -X22 (L21 X11), for half sizes 16, 32 and 64 on the matrix
// cores.
constexpr int DT = 512;      // threads of the diagonal-block kernel
constexpr int SB = 16;       // leaf width
// padded LDS row: 130 doubles = 4 banks mod 64, so the 16 rows x 4 k of an
// MFMA operand read (16 lanes down a column, 4 k across) hit 64 distinct
// banks
constexpr int LDD = BM + 2;
// BM x LDD tile, rdiag (BM), a zero (padded to 16 bytes)
constexpr size_t kDiagLds = ((size_t)BM * LDD + BM + 2) * sizeof(double);

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// One 16 x 16 output block: sum_{k in [kb, kb + 16 NC)} fa(r0 + i, k)
// fb(k, c0 + j).  Every operand is read from LDS before the first MFMA (one
// round trip instead of one per MFMA), and two accumulators alternate.
// Lane l holds (r0 + l/16 + 4 r, c0 + l%16) in component r of the result.
template <int NC, class FA, class FB>
__device__ __forceinline__ f64x4 mfma_block_n(FA fa, FB fb, int r0, int c0,
                                              int kb, int lane) {
  const int lr = lane & 15, lk = lane >> 4;
  double a[4 * NC], b[4 * NC];
#pragma unroll
  for (int q = 0; q < 4 * NC; ++q) {
    a[q] = fa(r0 + lr, kb + 4 * q + lk);
    b[q] = fb(kb + 4 * q + lk, c0 + lr);
  }
  f64x4 acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
  for (int q = 0; q < 4 * NC; ++q)
    acc[q & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc[q & 1],
                                                      0, 0, 0);
  return acc[0] + acc[1];
}

// The same for ke - kb in {16, 32, 48, 64} (uniform).
template <class FA, class FB>
__device__ __forceinline__ f64x4 mfma_block(FA fa, FB fb, int r0, int c0,
                                            int kb, int ke, int lane) {
  switch ((ke - kb) / 16) {
    case 1: return mfma_block_n<1>(fa, fb, r0, c0, kb, lane);
    case 2: return mfma_block_n<2>(fa, fb, r0, c0, kb, lane);
    case 3: return mfma_block_n<3>(fa, fb, r0, c0, kb, lane);
    default: return mfma_block_n<4>(fa, fb, r0, c0, kb, lane);
  }
}

// 1 / sqrt(p) for p > 0: hardware estimate refined by one Newton-Raphson
// step y <- y + y (1 - p y^2) / 2 (relative error of the estimate squares).
__device__ __forceinline__ double rsqrt_nr(double p) {
  const double y = __builtin_amdgcn_rsq(p);
  const double r = fma(-p * y, y, 1.0);
  return fma(0.5 * y, r, y);
}

// 1 / p for p > 0: hardware estimate refined by one Newton-Raphson step
// r <- r + r (1 - p r) (relative error of the estimate squares).
__device__ __forceinline__ double rcp_nr(double p) {
  const double r = __builtin_amdgcn_rcp(p);
  return fma(r, fma(-p, r, 1.0), r);
}

// Value of v in lane n of this lane's row of 16 (DPP row broadcast).  Every
// lane has a valid source lane, so bound_ctrl changes no value; it lets the
// compiler drop the initialisation of the destination.
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + N, 0xF, 0xF, true);
}

// Columns C >= J + 2 of every slot: A[r][C] -= u_r A[C][J] + v_r A[C][J+1],
// two columns at a time so that four independent FMA chains interleave.
template <int J, int C, int NS>
__device__ __forceinline__ void panel_update(double (&a)[2][SB],
                                             const double (&u)[NS],
                                             const double (&v)[NS]) {
  if constexpr (C + 1 < SB) {
    const double l0 = row_bcast<C>(a[0][J]), l1 = row_bcast<C>(a[0][J + 1]);
    const double m0 = row_bcast<C + 1>(a[0][J]);
    const double m1 = row_bcast<C + 1>(a[0][J + 1]);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      a[s][C] = fma(-u[s], l0, a[s][C]);
      a[s][C + 1] = fma(-u[s], m0, a[s][C + 1]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      a[s][C] = fma(-v[s], l1, a[s][C]);
      a[s][C + 1] = fma(-v[s], m1, a[s][C + 1]);
      // keep the update here: sunk to its first use it would hold every
      // broadcast value live until the end of the panel
      asm volatile("" : "+v"(a[s][C]), "+v"(a[s][C + 1]));
    }
    panel_update<J, C + 2, NS>(a, u, v);
  } else if constexpr (C < SB) {
    const double l0 = row_bcast<C>(a[0][J]), l1 = row_bcast<C>(a[0][J + 1]);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      a[s][C] = fma(-v[s], l1, fma(-u[s], l0, a[s][C]));
      asm volatile("" : "+v"(a[s][C]));
    }
  }
}

// Elimination of the column pair (J, J + 1) of the panel (see panel_chol)
// with its 2 x 2 pivot block B = [[b11, b21], [b21, b22]], then the pairs
// after it.  The rows' pair entries P = [A[r][J], A[r][J+1]] stay as they
// are; the columns after the pair lose P B^-1 P^T.  B^-1 comes from the
// determinant in closed form, one reciprocal per pair on the serial chain.
template <int J, int NS>
__device__ __forceinline__ void panel_pairs(double (&a)[2][SB],
                                            double (&bb)[SB / 2][3],
                                            bool& bad) {
  if constexpr (J < SB) {
    double b11 = row_bcast<J>(a[0][J]);
    double b21 = row_bcast<J + 1>(a[0][J]);
    double b22 = row_bcast<J + 1>(a[0][J + 1]);
    double det = fma(b11, b22, -b21 * b21);
    const bool ok = b11 > 0.0 && b11 < INFINITY && det > 0.0 && det < INFINITY;
    bad = bad || !ok;
    b11 = ok ? b11 : 1.0;
    b21 = ok ? b21 : 0.0;
    b22 = ok ? b22 : 1.0;
    det = ok ? det : 1.0;
    bb[J / 2][0] = b11;
    bb[J / 2][1] = b21;
    bb[J / 2][2] = det;
    const double rdet = rcp_nr(det);
    const double w11 = b22 * rdet, w21 = -b21 * rdet, w22 = b11 * rdet;
    double u[NS], v[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      u[s] = fma(a[s][J], w11, a[s][J + 1] * w21);
      v[s] = fma(a[s][J], w21, a[s][J + 1] * w22);
    }
    panel_update<J, J + 2, NS>(a, u, v);
    panel_pairs<J + 2, NS>(a, bb, bad);
  }
}

// Rows of the panel at c0 into a (see panel_chol); rows past the block read
// the zero *zs.  Selecting the address rather than the value keeps every
// read unconditional: a select of loaded values is turned into branches,
// each paying a full LDS round trip.
template <int NS>
__device__ __forceinline__ void panel_load(const double* S, const double* zs,
                                           int c0, int r1, int lane,
                                           double (&a)[2][SB]) {
  const int row[2] = {c0 + (lane & 15), r1 + lane};
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const bool in = row[s] < BM;
#pragma unroll
    for (int j = 0; j < SB; ++j)
      a[s][j] = *(in ? S + row[s] * LDD + c0 + j : zs);
  }
}

// One wave: Cholesky factor of the panel S[c0:BM, c0:c0+SB], whose trailing
// updates are complete.  Slot 0 of lane l holds leaf row c0 + l % 16 (each
// row of 16 lanes a copy of the leaf, so that the leaf's entries reach every
// lane by a row broadcast); slot 1 holds row r1 + l below the leaf (NS slots
// in use).  Two waves may share a panel, each with its own rows below and its
// own copy of the leaf's elimination; only the leaf owner stores the leaf and
// reports a failed pivot.  Block elimination with 2 x 2 pivots leaves, per
// column pair, the pair entries P of each row and the pivot block B (kept as
// b11, b21, det); afterwards L_B = chol(B) and the rows' factor entries
// P L_B^-T are formed off the serial chain.  Stores L (on and below the
// diagonal) and 1 / L_jj in rd.  Leaf entries right of the diagonal are
// updated too but never broadcast nor stored.
template <int NS>
__device__ __forceinline__ void panel_chol(double* S, double* rd, int c0,
                                           int r1, bool owner, int lane,
                                           int* fail, double (&a)[2][SB]) {
  const int row[2] = {c0 + (lane & 15), r1 + lane};
  double bb[SB / 2][3];
  bool bad = false;
  panel_pairs<0, NS>(a, bb, bad);
  if (bad && owner && lane == 0) atomicOr(fail, 1);
  double rpr = 0.0;
#pragma unroll
  for (int q = 0; q < SB / 2; ++q) {
    // L_B = [[l11, 0], [l21, l22]], l22^2 = det / b11: y1 = 1 / l11,
    // y2 = 1 / l22
    const double y1 = rsqrt_nr(bb[q][0]);
    const double l21 = bb[q][1] * y1;
    const double y2 = rsqrt_nr(bb[q][2] * y1 * y1);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double x1 = a[s][2 * q] * y1;
      a[s][2 * q + 1] = (a[s][2 * q + 1] - x1 * l21) * y2;
      a[s][2 * q] = x1;
    }
    rpr = (lane & 15) == 2 * q ? y1 : ((lane & 15) == 2 * q + 1 ? y2 : rpr);
  }
#pragma unroll
  for (int j = 0; j < SB; ++j) {
    if (owner && lane < SB && j <= lane) S[row[0] * LDD + c0 + j] = a[0][j];
#pragma unroll
    for (int s = 1; s < NS; ++s)
      if (row[s] < BM) S[row[s] * LDD + c0 + j] = a[s][j];
  }
  if (owner && lane < SB) rd[c0 + lane] = rpr;
}

// Waves that factor the panel at c0: the BM - c0 - SB rows below the leaf
// take one 64-row slot per wave (waves 0 and 1 when there are more than 64).
__device__ __forceinline__ int panel_waves(int c0) {
  return BM - c0 - SB > 64 ? 2 : 1;
}

// The panel at c0 on waves [0, panel_waves(c0)); others(pw) runs on the
// remaining waves.  Two waves each eliminate their own copy of the leaf, so
// both read it before either stores (barrier between load and factor).
template <class F>
__device__ __forceinline__ void panel_step(double* S, double* rd,
                                           const double* zs, int c0, int wave,
                                           int lane, int* fail, F others) {
  const int pw = panel_waves(c0);
  double a[2][SB];
  if (BM - c0 - SB > 0) {
    const int r1 = c0 + SB + 64 * wave;
    if (wave < pw) panel_load<2>(S, zs, c0, r1, lane, a);
    if (pw == 2) __syncthreads();
    if (wave < pw)
      panel_chol<2>(S, rd, c0, r1, wave == 0, lane, fail, a);
    else
      others(pw);
  } else if (wave == 0) {
    panel_load<1>(S, zs, c0, c0 + SB, lane, a);
    panel_chol<1>(S, rd, c0, c0 + SB, true, lane, fail, a);
  } else {
    others(1);
  }
}

// Step m of the leaf inverse (see leaf_inv): row m of X, formed in lane m
// from its accumulator, reaches the lanes of its row of 16 by a row
// broadcast; lanes of later rows add L[r][m] X[m][c].
template <int M>
__device__ __forceinline__ void leaf_inv_step(const double (&a)[SB],
                                              const double (&rp)[SB],
                                              double (&x)[SB]) {
  if constexpr (M + 1 < SB) {
#pragma unroll
    for (int c = 0; c <= M; ++c) {
      const double xmc = ((c == M ? 1.0 : 0.0) - row_bcast<M>(x[c])) * rp[M];
      x[c] = fma(a[M], xmc, x[c]);
    }
    leaf_inv_step<M + 1>(a, rp, x);
  }
}

// One wave: inverse X of the factored leaf at (c0, c0), row by row:
// X[m] = (e_m - sum_{m'<m} L[m][m'] X[m']) / L[m][m].  Lane r holds row
// r % 16 (each row of 16 lanes a copy) and accumulates
// sum_{m<r} L[r][m] X[m][:]; row m of X is formed from lane m's accumulator
// as it is broadcast.  The strict lower part of X is parked transposed in
// the leaf's strict upper triangle.
__device__ __forceinline__ void leaf_inv(double* S, const double* rd,
                                         const double* zs, int c0, int lane) {
  const int r = lane & (SB - 1);
  double a[SB], rp[SB], x[SB];
#pragma unroll
  for (int j = 0; j < SB; ++j) {
    a[j] = *(j < r ? S + (c0 + r) * LDD + c0 + j : zs);
    rp[j] = rd[c0 + j];
    x[j] = 0.0;
  }
  leaf_inv_step<0>(a, rp, x);
  const double rpr = rd[c0 + r];
#pragma unroll
  for (int c = 0; c < SB; ++c) x[c] = ((c == r ? 1.0 : 0.0) - x[c]) * rpr;
  if (lane < SB) {
#pragma unroll
    for (int j = 0; j < SB; ++j)
      if (j < r) S[(c0 + j) * LDD + c0 + r] = x[j];
  }
}

// Work of a deferred group update carried by the diagonal-block launch:
// sub-blocks [q0, q1) (64 x 64, see update_block) of the update from the
// panels [kA, kB) to the columns [jlo, jhi) and inverse rows [ilo, ...).
struct UpdFill {
  int kA = 0, kB = 0, jlo = 0, jhi = 0, ilo = 0, nu = 0, q0 = 0, q1 = 0;
};
template <int TM>
__device__ __forceinline__ void update_block(double* M, double* X, int64_t ld,
                                             int nt, int kA, int kB, int jlo,
                                             int jhi, int ilo, int nu, int q,
                                             int t, double* sA, double* sB);
constexpr int kFillTM = 64;
static_assert(2 * 4 * (size_t)stage_size<kFillTM>() * sizeof(double) <=
                  kDiagLds,
              "both halves' stages fit in the diagonal block's LDS");

// Per lane (blockIdx.y), workgroup 0 factors and inverts diagonal block k.
// Workgroups 1, 2, ... (one per CU: they take the same LDS) each compute
// two sub-blocks of the
// deferred update `fill`, one per half of the workgroup: the two 64 x 64
// halves of one 128 x 64 strip of a tile (the same reduction length, so both
// halves pass the same barriers).  The update touches tiles disjoint from
// block k's column and row; it only fills CUs the diagonal block leaves
// idle.
__global__ void __launch_bounds__(DT) diag_block_kernel(double* M, double* X,
                                                        int64_t ld, int k,
                                                        int* fail,
                                                        const int* skip,
                                                        Lanes ls,
                                                        UpdFill fill) {
  const int ln = blockIdx.y;
  M += ln * ls.mat;
  X += ln * ls.mat;
  fail += ln * ls.flag;
  if (skip) skip += ln * ls.flag;
  if (skip && *skip) return;
  extern __shared__ double S[];  // BM x LDD, then rdiag (BM), then a zero
  if (blockIdx.x > 0) {
    const int q = fill.q0 + 2 * ((int)blockIdx.x - 1);
    if (q >= fill.q1) return;  // uniform: q and q + 1 < q1 together
    constexpr int SS = 2 * stage_size<kFillTM>();
    const int half = (int)threadIdx.x >> 8;
    double* sA = S + half * 2 * SS;
    update_block<kFillTM>(M, X, ld, (int)(ld / BM), fill.kA, fill.kB,
                          fill.jlo, fill.jhi, fill.ilo, fill.nu, q + half,
                          (int)threadIdx.x & 255, sA, sA + SS);
    return;
  }
  double* rd = S + BM * LDD;
  double* zs = rd + BM;
  const int tid = threadIdx.x, lane = tid & 63;
  // wave-uniform, kept in a scalar register so that branches on it are
  // scalar branches
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int NW = DT / 64;
  double* Mk = M + (int64_t)k * BM * ld + (int64_t)k * BM;
  double* Xk = X + (int64_t)k * BM * ld + (int64_t)k * BM;
  auto Lv = [&](int i, int j) { return S[i * LDD + j]; };  // i >= j only
  // one unconditional read from the selected address (see panel_load)
  auto Xv = [&](int i, int j) {
    return *(i > j ? S + j * LDD + i : (i == j ? rd + i : zs));
  };
  auto Xt = [&](int m, int c) { return Xv(c, m); };  // X^T
  {
    constexpr int PER = BM * BM / DT;
    double v[PER];
    // the whole tile: nothing reads the part above the diagonal as data
    // (the leaf entries there are updated but never broadcast, and X is
    // parked there before it is read)
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * DT, i = idx / BM, c = idx % BM;
      v[q] = Mk[(int64_t)i * ld + c];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * DT, i = idx / BM, c = idx % BM;
      S[i * LDD + c] = v[q];
    }
    if (tid == 0) *zs = 0.0;
  }
  __syncthreads();
  // ---- factorisation --------------------------------------------------------
  // Step c0: the sub-panel below leaf c0, then the trailing update.  The
  // next panel's blocks are updated first; waves 0 (and 1) factor that panel
  // while the other waves finish the trailing update (disjoint blocks).
  panel_step(S, rd, zs, 0, wave, lane, fail, [](int) {});
  __syncthreads();
  auto Lt = [&](int m, int c) { return S[c * LDD + m]; };  // L^T
  for (int c0 = 0; c0 + SB < BM; c0 += SB) {
    const int r0 = c0 + SB, nb = (BM - r0) / 16;
    // A22 -= L21 L21^T, 16 x 16 block (bi, bj) of A22, bi >= bj
    auto trail = [&](int bi, int bj) {
      const f64x4 v =
          mfma_block(Lv, Lt, r0 + 16 * bi, r0 + 16 * bj, c0, c0 + SB, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        S[(r0 + 16 * bi + (lane >> 4) + 4 * q) * LDD + r0 + 16 * bj +
          (lane & 15)] -= v[q];
    };
    // the next panel's blocks first, one per wave
    if (wave < nb) trail(wave, 0);
    __syncthreads();
    // waves 0 (and 1) factor the next panel while the others update the rest
    panel_step(S, rd, zs, r0, wave, lane, fail, [&](int pw) {
      for (int b = wave - pw; b < (nb - 1) * nb / 2; b += NW - pw) {
        int bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
        trail(bi + 1, b - bi * (bi + 1) / 2 + 1);
      }
    });
    __syncthreads();
  }
  // ---- inverse: the leaves' inverses, one wave each, then
  // X21 = -X22 (L21 X11) at half sizes 16, 32 and 64 --------------------------
  static_assert(BM / SB == NW, "one leaf per wave");
  leaf_inv(S, rd, zs, wave * SB, lane);
  __syncthreads();
  auto Tv = [&](int m, int c) { return S[c * LDD + m]; };  // parked T / X21
  for (int h = SB; h < BM; h *= 2) {
    const int nh = BM / (2 * h);         // independent problems
    const int hb = h / 16;               // 16-blocks per side
    const int nblk = nh * hb * hb;       // <= 16: at most 2 per wave
    // T = L21 X11, parked where X21 goes
    for (int b = wave; b < nblk; b += NW) {
      const int p = b / (hb * hb), bi = (b / hb) % hb, bj = b % hb;
      const int b0 = p * 2 * h;
      const int row = b0 + h + 16 * bi, col = b0 + 16 * bj;
      const f64x4 v = mfma_block(Lv, Xv, row, col, col, b0 + h, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        S[(col + (lane & 15)) * LDD + row + (lane >> 4) + 4 * q] = v[q];
    }
    __syncthreads();
    // X21 = -X22 T, stored over T after all waves have read it
    f64x4 res[2];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int b = wave + sl * NW;
      const int p = b / (hb * hb), bi = (b / hb) % hb, bj = b % hb;
      const int b0 = p * 2 * h;
      const int row = b0 + h + 16 * bi, col = b0 + 16 * bj;
      if (b < nblk) res[sl] = mfma_block(Xv, Tv, row, col, b0 + h, row + 16, lane);
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int b = wave + sl * NW;
      const int p = b / (hb * hb), bi = (b / hb) % hb, bj = b % hb;
      const int b0 = p * 2 * h;
      const int row = b0 + h + 16 * bi, col = b0 + 16 * bj;
      if (b < nblk) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          S[(col + (lane & 15)) * LDD + row + (lane >> 4) + 4 * q] = -res[sl][q];
      }
    }
    __syncthreads();
  }
  // L_kk: lower triangle only (the upper part of M's diagonal tiles is never
  // read again); X_kk with explicit zeros above the diagonal, which the
  // panel, finalize and update products read as part of the full tile.
  for (int idx = tid; idx < BM * BM; idx += DT) {
    const int i = idx / BM, c = idx % BM;
    if (c <= i) Mk[(int64_t)i * ld + c] = S[i * LDD + c];
    Xk[(int64_t)i * ld + c] = Xv(i, c);
  }
}

// Step k after the diagonal block, first launch (both need only L_kk^-1),
// each 128 x 128 tile split in BM / H bands of width H on separate
// workgroups:
//   tiles [0, rem):        L[I, k] = M[I, k] L_kk^-T, I = k + 1 + b, in place;
//                          a band of H rows depends only on the same rows of
//                          M[I, k];
//   tiles [rem, rem + k):  X[k, j] = -L_kk^-1 S[k, j], j = b - rem, where S
//                          accumulated sum_{m<k} L[k, m] X[m, j] in place; a
//                          band of H columns depends only on the same columns
//                          of S[k, j].
template <int H>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
panel_finalize_kernel(double* M, double* X, int64_t ld, int k, int rem,
                      const int* skip, Lanes ls) {
  const int ln = blockIdx.y;
  M += ln * ls.mat;
  X += ln * ls.mat;
  if (skip) skip += ln * ls.flag;
  if (skip && *skip) return;
  constexpr int NBAND = BM / H;
  __shared__ double sA[2 * stage_size<BM>()], sB[2 * stage_size<BM>()];
  const int b = blockIdx.x / NBAND, half = (blockIdx.x % NBAND) * H;
  const double* Xkk = X + (int64_t)k * BM * ld + (int64_t)k * BM;
  if (b < rem) {
    const int I = k + 1 + b;
    double* Mik = M + (int64_t)I * BM * ld + (int64_t)k * BM + (int64_t)half * ld;
    f64x4 acc[H / 32][BM / 32];
    gemm_core<double, true, double, true, H, BM>(Mik, ld, Xkk, ld, nullptr, 0,
                                                 BM, acc, sA, sB);
    for_each_acc<H, BM>(acc, [&](int r, int c, double v) {
      Mik[(int64_t)r * ld + c] = v;
    });
  } else {
    const int j = b - rem;
    double* Skj = X + (int64_t)k * BM * ld + (int64_t)j * BM + half;
    f64x4 acc[BM / 32][H / 32];
    gemm_core<double, true, double, false, BM, H>(Xkk, ld, Skj, ld, nullptr, 0,
                                                  BM, acc, sA, sB);
    for_each_acc<BM, H>(acc, [&](int r, int c, double v) {
      Skj[(int64_t)r * ld + c] = -v;
    });
  }
}

// Tile sub-blocks for the update: a 128 x 128 tile is computed as
// (128 / TM)^2 sub-blocks of TM x TM by separate workgroups.  Safe because
// an update reads only panel tiles it does not write.
template <int TM>
__device__ __forceinline__ void sub_block(int b, int* tile, int* so, int* sc) {
  constexpr int Q = BM / TM;
  *tile = b / (Q * Q);
  *so = (b / Q) % Q * TM;
  *sc = b % Q * TM;
}

// Trailing update from the panel columns [kA, kB) (tile units), in one
// launch (needs those panels L[:, kA..kB) and rows X[kA..kB, :]):
//   tiles [0, nu):        M[I, J] -= sum_{k in [kA, kB)} L[I, k] L[J, k]^T
//                         for J in [jlo, jhi), J <= I < nt;
//   tiles [nu, nu + ni):  S[i, j] += sum_{k in [max(kA, j), kB)} L[i, k] X[k, j]
//                         for i in [ilo, ihi), j < kB (X[k, j] = 0 for k < j);
//                         stored rather than added when j >= kA (the first
//                         contribution), so X needs no clearing beforehand.
// The two sets touch disjoint tiles (columns J >= kB versus j < kB).
// Sub-block q (see sub_block) of that trailing update, computed by the 256
// threads t in [0, 256) of the calling workgroup with LDS stages sA, sB.
template <int TM>
__device__ __forceinline__ void update_block(double* M, double* X, int64_t ld,
                                             int nt, int kA, int kB, int jlo,
                                             int jhi, int ilo, int nu, int q,
                                             int t, double* sA, double* sB) {
  int b, so, sc;
  sub_block<TM>(q, &b, &so, &sc);
  f64x4 acc[TM / 32][TM / 32];
  constexpr int kEntries = (TM / 32) * (TM / 32) * 4;  // per thread
  const int lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * (TM / 2), wn = (w & 1) * (TM / 2);
  auto each = [&](auto f) {
#pragma unroll
    for (int i = 0; i < TM / 32; ++i)
#pragma unroll
      for (int j = 0; j < TM / 32; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          f(wm + i * 16 + (lane >> 4) + 4 * r, wn + j * 16 + (lane & 15),
            acc[i][j][r]);
  };
  if (b < nu) {
    int J = jlo;
    while (J < jhi && b >= nt - J) {   // column J holds tiles I = J .. nt-1
      b -= nt - J;
      ++J;
    }
    const int I = J + b;
    const double* Li = M + (int64_t)I * BM * ld + (int64_t)so * ld;
    const double* Lj = M + (int64_t)J * BM * ld + (int64_t)sc * ld;
    gemm_core<double, true, double, true, TM>(Li, ld, Lj, ld, nullptr,
                                              (int64_t)kA * BM,
                                              (int64_t)kB * BM, acc, sA, sB, t);
    // read-modify-write with every read issued first: a wait for a load
    // also waits for the stores before it, so alternating them would make
    // one memory round trip per entry
    double* Mij = M + (int64_t)I * BM * ld + (int64_t)J * BM;
    double old[kEntries];
    int e = 0;
    each([&](int r, int c, double) {
      old[e++] = Mij[(int64_t)(so + r) * ld + sc + c];
    });
    e = 0;
    each([&](int r, int c, double v) {
      Mij[(int64_t)(so + r) * ld + sc + c] = old[e++] - v;
    });
  } else {
    b -= nu;
    const int i = ilo + b / kB, j = b % kB;
    const int k0 = j > kA ? j : kA;
    const double* Li = M + (int64_t)i * BM * ld + (int64_t)so * ld;
    gemm_core<double, true, double, false, TM>(Li, ld, X + (int64_t)j * BM + sc,
                                               ld, nullptr, (int64_t)k0 * BM,
                                               (int64_t)kB * BM, acc, sA, sB, t);
    // the update whose reduction starts at k = j brings the first
    // contribution (X[k, j] = 0 for k < j): it stores, later ones add
    double* Sij = X + (int64_t)i * BM * ld + (int64_t)j * BM;
    if (j >= kA) {
      each([&](int r, int c, double v) {
        Sij[(int64_t)(so + r) * ld + sc + c] = v;
      });
    } else {
      double old[kEntries];
      int e = 0;
      each([&](int r, int c, double) {
        old[e++] = Sij[(int64_t)(so + r) * ld + sc + c];
      });
      e = 0;
      each([&](int r, int c, double v) {
        Sij[(int64_t)(so + r) * ld + sc + c] = old[e++] + v;
      });
    }
  }
}

// Occupancy: two workgroups per CU for 128-wide tiles (their LDS), three
// for the 64-wide group-update sub-blocks and four for the 32-wide in-group
// ones (the whole factorisation at n = 5504: 5.18 -> 4.96 -> 4.85 ms).
template <int TM>
constexpr int update_waves() { return TM == 32 ? 4 : TM == 64 ? 3 : 2; }
// Sub-blocks q0 + blockIdx.x of the update.
template <int TM>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(update_waves<TM>(), update_waves<TM>())))
update_kernel(double* M, double* X, int64_t ld, int nt, int kA, int kB,
              int jlo, int jhi, int ilo, int nu, int q0, const int* skip,
              Lanes ls) {
  const int ln = blockIdx.y;
  M += ln * ls.mat;
  X += ln * ls.mat;
  if (skip) skip += ln * ls.flag;
  if (skip && *skip) return;
  __shared__ double sA[2 * stage_size<TM>()], sB[2 * stage_size<TM>()];
  update_block<TM>(M, X, ld, nt, kA, kB, jlo, jhi, ilo, nu,
                   q0 + (int)blockIdx.x, (int)threadIdx.x, sA, sB);
}

// ------------------------------------------------------ matrix-vectors ----
// y = X v, X lower (np x np); one wave per row, rows < n.
// Dot products of the first len entries of one row with P vectors
// V + a * vs (one wave; row 16-byte aligned).  Each lane reads two
// consecutive entries of the row per load and keeps four such loads in
// flight, so that a wave streams 4 KB of the row at a time.
template <int P>
__device__ __forceinline__ void row_dots(const double* __restrict__ row,
                                         int64_t len,
                                         const double* __restrict__ V,
                                         int64_t vs, int lane, double (&s)[P]) {
  constexpr int U = 4;
  double acc[P][2];
#pragma unroll
  for (int a = 0; a < P; ++a) acc[a][0] = acc[a][1] = 0.0;
  int64_t k = 2 * lane;
  for (; k + 128 * (U - 1) + 1 < len; k += 128 * U) {
    double2 b[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      b[u] = *reinterpret_cast<const double2*>(row + k + 128 * u);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int a = 0; a < P; ++a) {
        const double* e = V + a * vs + k + 128 * u;
        acc[a][0] = fma(b[u].x, e[0], acc[a][0]);
        acc[a][1] = fma(b[u].y, e[1], acc[a][1]);
      }
  }
  for (; k < len; k += 128) {
#pragma unroll
    for (int a = 0; a < P; ++a) {
      acc[a][0] = fma(row[k], V[a * vs + k], acc[a][0]);
      if (k + 1 < len)
        acc[a][1] = fma(row[k + 1], V[a * vs + k + 1], acc[a][1]);
    }
  }
#pragma unroll
  for (int a = 0; a < P; ++a) s[a] = wave_sum(acc[a][0] + acc[a][1]);
}

__global__ void trmv_n_kernel(const double* __restrict__ X, int64_t ld,
                              int64_t n, const double* __restrict__ v,
                              double* __restrict__ y, const int* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double s[1];
  row_dots<1>(X + i * ld, i + 1, v, 0, lane, s);
  if (lane == 0) y[i] = s[0];
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

// W[a*n + i] = sum_j B[i][j] E[a*n + j], a < P (B full symmetric).
template <int P>
__global__ void symm_multi_kernel(const double* __restrict__ B, int64_t ld,
                                  int64_t n, const double* __restrict__ E,
                                  double* __restrict__ W, const int* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double s[P];
  row_dots<P>(B + i * ld, n, E, n, lane, s);
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < P; ++a) W[a * n + i] = s[a];
  }
}

}  // namespace

// ------------------------------------------------------------ launchers --

// XCD-aware SYRK order.  Workgroups go round-robin over the 8 XCDs, so XCD
// x runs the workgroups x, x + 8, ...  The 128-column blocks of A fall into
// 4 groups; XCD x < 6 takes the tiles of one off-diagonal pair of groups,
// XCDs 6 and 7 the tiles of two diagonal pairs each, and the lists are then
// evened out.  The tiles running together on one XCD then stream about half
// of A's column blocks, which its L2 holds band by band, instead of all of
// them.
std::vector<int> syrk_tile_order(int nt) {
  std::vector<int> out;
  if (nt < 16) return out;
  constexpr int NX = 8, NG = 4;
  int gs[NG + 1];
  for (int g = 0; g <= NG; ++g) gs[g] = g * nt / NG;
  std::vector<std::vector<std::pair<int, int>>> lists(NX);
  int x = 0;
  for (int gi = 1; gi < NG; ++gi)
    for (int gj = 0; gj < gi; ++gj, ++x)
      for (int I = gs[gi]; I < gs[gi + 1]; ++I)
        for (int J = gs[gj]; J < gs[gj + 1]; ++J) lists[x].push_back({I, J});
  for (int g = 0; g < NG; ++g)
    for (int I = gs[g]; I < gs[g + 1]; ++I)
      for (int J = gs[g]; J <= I; ++J) lists[6 + g / 2].push_back({I, J});
  for (;;) {
    int hi = 0, lo = 0;
    for (int k = 1; k < NX; ++k) {
      if (lists[k].size() > lists[hi].size()) hi = k;
      if (lists[k].size() < lists[lo].size()) lo = k;
    }
    if (lists[hi].size() <= lists[lo].size() + 1) break;
    lists[lo].push_back(lists[hi].back());
    lists[hi].pop_back();
  }
  size_t len = 0;
  for (const auto& l : lists) len = std::max(len, l.size());
  out.assign(2 * NX * len, -1);
  for (int k = 0; k < NX; ++k)
    for (size_t i = 0; i < lists[k].size(); ++i) {
      out[2 * (NX * i + k)] = lists[k][i].first;
      out[2 * (NX * i + k) + 1] = lists[k][i].second;
    }
  return out;
}

// Cost of one piece of the balanced SYRK beyond its slices (pipeline fill,
// drain, publish and arrival), in slices: at n = 5440, T = 12000 (752
// slices) bodies longer by 0, 8, 16 and 24 slices gave 5.71, 5.65, 5.68 and
// 5.72 ms per launch, and 8 is this cost times m / U there.
constexpr int64_t kPieceSlices = 10;

bool syrk_split_plan(int nt, int64_t ns, int slots, SyrkPlan* out) {
  constexpr int NX = 8;
  *out = SyrkPlan{};
  if (slots < NX || slots % NX != 0 || ns < 1) return false;
  const std::vector<int> ord = syrk_tile_order(nt);
  if (ord.empty()) return false;
  const int U = slots / NX;  // workgroups per XCD
  // list x holds its tiles at positions 0 .. len[x] - 1 (entry NX * i + x)
  const int64_t rows = (int64_t)ord.size() / (2 * NX);
  std::vector<int64_t> len(NX, 0);
  for (int x = 0; x < NX; ++x)
    for (int64_t i = 0; i < rows; ++i)
      if (ord[2 * (NX * i + x)] >= 0) len[x] = i + 1;
  const int64_t lmin = *std::min_element(len.begin(), len.end());
  const int R = (int)(lmin / U);
  // per workgroup its pieces (tile, first slice, end slice); per tile its
  // block indices and pieces in K order
  std::vector<std::vector<std::array<int, 3>>> wp(slots);
  std::vector<int> tiles;
  std::vector<int> npieces;
  for (int x = 0; x < NX; ++x) {
    const int64_t m = len[x] - (int64_t)R * U;  // tiles cut along K
    if (m <= 0) continue;
    // m <= U; every workgroup of the XCD gets an equal share.  The first m
    // take the bodies [0, Lb) of the m tiles, so that they sweep the same
    // slices of A together; the other U - m share the remainders [Lb, ns),
    // concatenated tile by tile.  A remainder workgroup runs about m /
    // (U - m) + 1 pieces, each with its own pipeline fill, drain and
    // publish, where a body runs one; equal times then need the bodies
    // longer by the piece cost times m / U.
    const int64_t Lb =
        std::min<int64_t>(ns, m * ns / U + kPieceSlices * m / U);
    if (m > U || Lb < 16) return false;
    const int t0 = (int)npieces.size();
    for (int64_t p = 0; p < m; ++p) {
      const int64_t e = NX * (R * U + p) + x;
      tiles.push_back(ord[2 * e]);
      tiles.push_back(ord[2 * e + 1]);
      npieces.push_back(0);
      wp[NX * p + x].push_back({(int)(t0 + p), 0, (int)Lb});
    }
    const int64_t rw = U - m, rem = ns - Lb, Q = m * rem;
    if (rem > 0 && rw == 0) return false;
    for (int64_t v = 0; v < rw && rem > 0; ++v) {
      const int64_t lo = v * Q / rw, hi = (v + 1) * Q / rw;
      const int w = (int)(NX * (m + v) + x);
      for (int64_t p = lo / rem; p < m && p * rem < hi; ++p) {
        const int64_t ks = std::max(lo, p * rem) - p * rem + Lb;
        const int64_t ke = std::min(hi, (p + 1) * rem) - p * rem + Lb;
        if (ke > ks) wp[w].push_back({(int)(t0 + p), (int)ks, (int)ke});
      }
    }
  }
  // piece indices in K order per tile (bodies first, then the remainders in
  // the order of their workgroups, which is ascending K); coverage check
  const int ntile2 = (int)npieces.size();
  std::vector<int64_t> next(ntile2, 0);
  std::vector<std::vector<std::array<int, 2>>> by_tile(ntile2);  // (w, j)
  for (int w = 0; w < slots; ++w)
    for (int j = 0; j < (int)wp[w].size(); ++j) by_tile[wp[w][j][0]].push_back({w, j});
  std::vector<std::vector<int>> pidx(slots);
  for (int w = 0; w < slots; ++w) pidx[w].assign(wp[w].size(), -1);
  for (int t = 0; t < ntile2; ++t) {
    auto& v = by_tile[t];
    std::sort(v.begin(), v.end(), [&](const std::array<int, 2>& a,
                                      const std::array<int, 2>& b) {
      return wp[a[0]][a[1]][1] < wp[b[0]][b[1]][1];
    });
    for (size_t k = 0; k < v.size(); ++k) {
      const auto& pc = wp[v[k][0]][v[k][1]];
      if (pc[1] != next[t]) return false;
      next[t] = pc[2];
      pidx[v[k][0]][v[k][1]] = (int)k;
    }
    if (next[t] != ns) return false;
    npieces[t] = (int)v.size();
  }
  int nslots = 0;
  std::vector<int> base(ntile2, -1);
  for (int t = 0; t < ntile2; ++t)
    if (npieces[t] > 1) {
      base[t] = nslots;
      nslots += npieces[t];
    }
  // device layout: per workgroup (first piece, count); the pieces; the tiles
  std::vector<int> plan(2 * (size_t)slots, 0);
  int np = 0;
  for (int w = 0; w < slots; ++w) {
    plan[2 * w] = np;
    plan[2 * w + 1] = (int)wp[w].size();
    np += (int)wp[w].size();
  }
  for (int w = 0; w < slots; ++w)
    for (size_t j = 0; j < wp[w].size(); ++j) {
      plan.push_back(wp[w][j][0]);
      plan.push_back(wp[w][j][1]);
      plan.push_back(wp[w][j][2]);
      plan.push_back(pidx[w][j]);
    }
  for (int t = 0; t < ntile2; ++t) {
    plan.push_back(tiles[2 * t]);
    plan.push_back(tiles[2 * t + 1]);
    plan.push_back(npieces[t]);
    plan.push_back(base[t]);
  }
  out->order.assign(ord.begin(), ord.begin() + 2 * (size_t)R * slots);
  out->plan = std::move(plan);
  out->slots = slots;
  out->rounds = R;
  out->ntile2 = ntile2;
  out->npieces = np;
  out->nslots = nslots;
  return true;
}

int syrk_split_slots() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, syrk_split_kernel<double>, NT, 0) != hipSuccess)
    return 0;
  return cus * per;
}

hipError_t launch_syrk(int precision, const void* A, int64_t lda, int64_t Tp,
                       const double* s, double* B, hipStream_t st,
                       const int* skip, Lanes ls, int nlanes,
                       const int* order, int64_t order_slots,
                       const SyrkSplit* split) {
  if (split && split->ws && split->cnt) {
    const SyrkSplit& p = *split;
    dim3 g((unsigned)p.slots, (unsigned)nlanes), b(NT);
    switch (precision) {
      case 0:
        hipLaunchKernelGGL(syrk_split_kernel<double>, g, b, 0, st,
                           (const double*)A, lda, Tp, s, B, skip, ls, p.order,
                           p.rounds, p.plan, p.npieces, p.ws, p.ws_lane,
                           p.cnt, p.cnt_lane);
        break;
      case 1:
        hipLaunchKernelGGL(syrk_split_kernel<float>, g, b, 0, st,
                           (const float*)A, lda, Tp, s, B, skip, ls, p.order,
                           p.rounds, p.plan, p.npieces, p.ws, p.ws_lane,
                           p.cnt, p.cnt_lane);
        break;
      case 2:
        hipLaunchKernelGGL(syrk_split_kernel<bf16_t>, g, b, 0, st,
                           (const bf16_t*)A, lda, Tp, s, B, skip, ls, p.order,
                           p.rounds, p.plan, p.npieces, p.ws, p.ws_lane,
                           p.cnt, p.cnt_lane);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const int64_t nt = lda / BM, ntiles = nt * (nt + 1) / 2;
  dim3 g((unsigned)(order ? order_slots : ntiles), (unsigned)nlanes), b(NT);
  switch (precision) {
    case 0:
      hipLaunchKernelGGL(syrk_kernel<double>, g, b, 0, st, (const double*)A,
                         lda, Tp, s, B, skip, ls, order);
      break;
    case 1:
      hipLaunchKernelGGL(syrk_kernel<float>, g, b, 0, st, (const float*)A, lda,
                         Tp, s, B, skip, ls, order);
      break;
    case 2:
      hipLaunchKernelGGL(syrk_kernel<bf16_t>, g, b, 0, st, (const bf16_t*)A,
                         lda, Tp, s, B, skip, ls, order);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t prepare_dense_kernels() {
  static bool attr_set = false;
  if (!attr_set) {
    const size_t lds = kDiagLds;
    hipError_t e = hipFuncSetAttribute(
        (const void*)diag_block_kernel,
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  return hipSuccess;
}

// Blocked Cholesky M = L L^T with the inverse X = L^-1, two levels: steps of
// one 128-column block inside groups of `group` blocks (4 unless tuned).
// Inside a group each step updates only the group's remaining columns and
// inverse rows; one update per group with a group * 128 deep reduction then
// brings every
// later column and inverse row up to date, so the trailing matrix is read
// and written once per group instead of once per step.
constexpr int kDefaultGroup = 4;
// Band width of the panel finalisation and sub-block of the in-group
// updates: the steps on the factorisation's critical path launch few tiles,
// so narrower pieces on more workgroups shorten each launch.  The group
// updates run in 64 x 64 sub-blocks: their tile counts (126 to 936 tiles of
// 128 x 128 at n = 5440) leave whole rounds of 512 slots part-empty, which
// four times as many pieces even out.  The defaults below; a caller may ask
// for 64 for either of the first two (the launcher's step_tm, fin_band).
constexpr int kFinBand = 32;
constexpr int kStepTM = 32;
constexpr int kGroupTM = 64;

// CUs of the current device (0 if unknown).
static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess)
    return 0;
  return cus;
}

hipError_t launch_potrf_trtri(double* M, double* X, int64_t np, int* fail,
                              hipStream_t st, const int* skip, int group,
                              Lanes ls, int nlanes, bool fill, int step_tm,
                              int fin_band) {
  const unsigned L = (unsigned)nlanes;
  const int kGroup = group > 0 ? group : kDefaultGroup;
  const int nt = (int)(np / BM);
  const size_t lds = kDiagLds;
  hipError_t pe = prepare_dense_kernels();
  if (pe != hipSuccess) return pe;
  constexpr int QS = (BM / kStepTM) * (BM / kStepTM);  // sub-blocks per tile
  constexpr int QG = (BM / kGroupTM) * (BM / kGroupTM);
  static_assert(kGroupTM == kFillTM, "deferred sub-blocks are group sub-blocks");
  // workgroups a diagonal-block launch can add per lane for the deferred
  // update: the CUs the lanes' own diagonal blocks leave, shared equally,
  // so that every lane's diagonal block starts at once (none if that leaves
  // fewer than 8 per lane)
  int nfill = 0;
  if (fill) {
    const int cus = device_cus();
    nfill = cus > nlanes ? (cus - nlanes) / nlanes : 0;
    if (nfill < 8) nfill = 0;
  }
  auto tiles = [&](int kB, int jlo, int jhi, int ilo, int ihi, int* nu) {
    *nu = 0;
    for (int J = jlo; J < jhi; ++J) *nu += nt - J;
    return *nu + (ihi - ilo) * kB;
  };
  auto update = [&](int kA, int kB, int jlo, int jhi, int ilo, int ihi,
                    bool small) {
    int nu;
    const int n = tiles(kB, jlo, jhi, ilo, ihi, &nu);
    if (n == 0) return;
    if (small && step_tm == 64)
      hipLaunchKernelGGL(update_kernel<64>, dim3(n * (BM / 64) * (BM / 64), L),
                         dim3(NT), 0, st, M, X, np, nt, kA, kB, jlo, jhi, ilo,
                         nu, 0, skip, ls);
    else if (small)
      hipLaunchKernelGGL(update_kernel<kStepTM>, dim3(n * QS, L), dim3(NT), 0,
                         st, M, X, np, nt, kA, kB, jlo, jhi, ilo, nu, 0, skip,
                         ls);
    else
      hipLaunchKernelGGL(update_kernel<kGroupTM>, dim3(n * QG, L), dim3(NT), 0,
                         st, M, X, np, nt, kA, kB, jlo, jhi, ilo, nu, 0, skip,
                         ls);
  };
  // The group update of group g is split: the next group's columns and
  // inverse rows at once (its steps need them), the rest (columns and
  // inverse rows from the group after next on) deferred into the next
  // group's diagonal-block launches, and what they do not absorb launched
  // before the next group update.  Every tile still receives the groups'
  // contributions in group order with the same arithmetic.
  UpdFill pend;
  for (int g0 = 0; g0 < nt; g0 += kGroup) {
    const int g1 = g0 + kGroup < nt ? g0 + kGroup : nt;
    for (int k = g0; k < g1; ++k) {
      UpdFill f = pend;
      int extra = 0;
      if (pend.q0 < pend.q1) {
        extra = std::min(nfill, (pend.q1 - pend.q0) / 2);
        f.q1 = pend.q0 + 2 * extra;
        pend.q0 = f.q1;
      }
      hipLaunchKernelGGL(diag_block_kernel, dim3(1 + extra, L), dim3(DT), lds,
                         st, M, X, np, k, fail, skip, ls, f);
      const int rem = nt - k - 1;
      if (rem + k > 0 && fin_band == 64)
        hipLaunchKernelGGL(panel_finalize_kernel<64>,
                           dim3((rem + k) * (BM / 64), L), dim3(NT), 0, st, M,
                           X, np, k, rem, skip, ls);
      else if (rem + k > 0)
        hipLaunchKernelGGL(panel_finalize_kernel<kFinBand>,
                           dim3((rem + k) * (BM / kFinBand), L), dim3(NT), 0,
                           st, M, X, np, k, rem, skip, ls);
      if (k + 1 < g1) update(k, k + 1, k + 1, g1, k + 1, g1, true);
    }
    if (pend.q0 < pend.q1)
      hipLaunchKernelGGL(update_kernel<kGroupTM>, dim3(pend.q1 - pend.q0, L),
                         dim3(NT), 0, st, M, X, np, nt, pend.kA, pend.kB,
                         pend.jlo, pend.jhi, pend.ilo, pend.nu, pend.q0, skip,
                         ls);
    pend = UpdFill{};
    if (g1 >= nt) continue;
    const int g2 = g1 + kGroup < nt ? g1 + kGroup : nt;
    if (nfill > 0 && g2 < nt) {
      update(g0, g1, g1, g2, g1, g2, false);
      int nu;
      const int n = tiles(g1, g2, nt, g2, nt, &nu);
      pend = UpdFill{g0, g1, g2, nt, g2, nu, 0, n * QG};
    } else {
      update(g0, g1, g1, nt, g1, nt, false);
    }
  }
  return hipGetLastError();
}

hipError_t launch_trace_gemm(int precision, const void* A, int64_t lda,
                             int64_t Tp, const double* X, int64_t np,
                             double* rn, hipStream_t st, const int* skip,
                             Lanes ls, int nlanes) {
  dim3 g((unsigned)((np / BM) * ((Tp / BM + 7) / 8 * 8)), (unsigned)nlanes),
      b(NT);
  switch (precision) {
    case 0:
      hipLaunchKernelGGL(trace_gemm_kernel<double>, g, b, 0, st,
                         (const double*)A, lda, Tp, X, np, rn, skip, ls);
      break;
    case 1:
      hipLaunchKernelGGL(trace_gemm_kernel<float>, g, b, 0, st,
                         (const float*)A, lda, Tp, X, np, rn, skip, ls);
      break;
    case 2:
      hipLaunchKernelGGL(trace_gemm_kernel<bf16_t>, g, b, 0, st,
                         (const bf16_t*)A, lda, Tp, X, np, rn, skip, ls);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Split counts: about 768 workgroups, every split a multiple of 16 long.
static int64_t block_chunk(int64_t len, int tiles) {
  int64_t parts = std::max<int64_t>(1, std::min<int64_t>(len / 16, 768 / tiles));
  return (len / 16 + parts - 1) / parts * 16;
}

int block_splits(int64_t Tp, int64_t lda, int* sv, int* sz) {
  const int64_t kc = block_chunk(lda, (int)(Tp / BM));
  const int64_t tc = block_chunk(Tp, (int)(lda / BM));
  *sv = (int)((lda + kc - 1) / kc);
  *sz = (int)((Tp + tc - 1) / tc);
  return 0;
}

hipError_t launch_block_av(int precision, const void* A, int64_t lda,
                           int64_t Tp, const double* V, double* Zp, double* Z,
                           hipStream_t st, const int* skip) {
  const int ntt = (int)(Tp / BM);
  const int64_t kc = block_chunk(lda, ntt);
  const int parts = (int)((lda + kc - 1) / kc);
  dim3 g((unsigned)(ntt * parts)), b(NT);
  switch (precision) {
    case 0:
      hipLaunchKernelGGL(block_av_kernel<double>, g, b, 0, st,
                         (const double*)A, lda, V, kc, Zp, Tp, skip);
      break;
    case 1:
      hipLaunchKernelGGL(block_av_kernel<float>, g, b, 0, st, (const float*)A,
                         lda, V, kc, Zp, Tp, skip);
      break;
    case 2:
      hipLaunchKernelGGL(block_av_kernel<bf16_t>, g, b, 0, st,
                         (const bf16_t*)A, lda, V, kc, Zp, Tp, skip);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(sum_slabs_kernel, dim3(1024), dim3(256), 0, st, Zp, parts,
                     Tp * BW, Z, skip);
  return hipGetLastError();
}

template <bool SC>
static void launch_atz_t(int precision, const void* A, int64_t lda,
                         int64_t Tp, const double* Z, const double* s,
                         int64_t tc, double* Yp, dim3 g, hipStream_t st,
                         const int* skip) {
  dim3 b(NT);
  if (precision == 0)
    hipLaunchKernelGGL((block_atz_kernel<double, SC>), g, b, 0, st,
                       (const double*)A, lda, Tp, Z, s, tc, Yp, skip);
  else if (precision == 1)
    hipLaunchKernelGGL((block_atz_kernel<float, SC>), g, b, 0, st,
                       (const float*)A, lda, Tp, Z, s, tc, Yp, skip);
  else
    hipLaunchKernelGGL((block_atz_kernel<bf16_t, SC>), g, b, 0, st,
                       (const bf16_t*)A, lda, Tp, Z, s, tc, Yp, skip);
}

hipError_t launch_block_atz(int precision, const void* A, int64_t lda,
                            int64_t Tp, const double* Z, const double* s,
                            double* Yp, double* Y, hipStream_t st,
                            const int* skip) {
  if (precision < 0 || precision > 2) return hipErrorInvalidValue;
  const int njt = (int)(lda / BM);
  const int64_t tc = block_chunk(Tp, njt);
  const int parts = (int)((Tp + tc - 1) / tc);
  dim3 g((unsigned)(njt * parts));
  if (s)
    launch_atz_t<true>(precision, A, lda, Tp, Z, s, tc, Yp, g, st, skip);
  else
    launch_atz_t<false>(precision, A, lda, Tp, Z, s, tc, Yp, g, st, skip);
  hipLaunchKernelGGL(sum_slabs_kernel, dim3(1024), dim3(256), 0, st, Yp, parts,
                     lda * BW, Y, skip);
  return hipGetLastError();
}

hipError_t launch_gemm64(const double* A, int64_t lda, bool at,
                         const double* B, int64_t ldb, bool bt, double* C,
                         int64_t ldc, int64_t M, int64_t N, int64_t K,
                         double alpha, double beta, hipStream_t st) {
  if (M % BM || N % BM || K % BKK || M <= 0 || N <= 0 || K <= 0)
    return hipErrorInvalidValue;
  const int ntn = (int)(N / BM);
  dim3 g((unsigned)((M / BM) * ntn)), b(NT);
  if (!at && !bt)
    hipLaunchKernelGGL((gemm64_kernel<true, false>), g, b, 0, st, A, lda, B,
                       ldb, C, ldc, K, ntn, alpha, beta);
  else if (!at && bt)
    hipLaunchKernelGGL((gemm64_kernel<true, true>), g, b, 0, st, A, lda, B,
                       ldb, C, ldc, K, ntn, alpha, beta);
  else if (at && !bt)
    hipLaunchKernelGGL((gemm64_kernel<false, false>), g, b, 0, st, A, lda, B,
                       ldb, C, ldc, K, ntn, alpha, beta);
  else
    hipLaunchKernelGGL((gemm64_kernel<false, true>), g, b, 0, st, A, lda, B,
                       ldb, C, ldc, K, ntn, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_lane_scale(const double* Z, const double* s, int64_t vec,
                             int nl, int64_t Tp, double* ZS, hipStream_t st,
                             const int* skip) {
  if (nl < 1 || nl > BW) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lane_scale_kernel, dim3(1024), dim3(256), 0, st, Z, s,
                     vec, nl, Tp, ZS, skip);
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
  const dim3 g((unsigned)((n + 3) / 4)), b(256);
  switch (p) {
    case 1:
      hipLaunchKernelGGL(symm_multi_kernel<1>, g, b, 0, st, B, ldb, n, E, W,
                         skip);
      break;
    case 2:
      hipLaunchKernelGGL(symm_multi_kernel<2>, g, b, 0, st, B, ldb, n, E, W,
                         skip);
      break;
    case 3:
      hipLaunchKernelGGL(symm_multi_kernel<3>, g, b, 0, st, B, ldb, n, E, W,
                         skip);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace yand
