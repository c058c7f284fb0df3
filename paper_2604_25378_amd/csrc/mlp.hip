// Warm-start MLP: FP32 forward, backward and Adam kernels, and the mapping
// between the network output and portfolio weights.
//
// Network: in -> H (tanh) -> H (tanh) -> H (tanh) -> out (linear), weights
// row-major W_k (fan_in x fan_out) followed by b_k, all FP32 in one buffer.
// Loss: (1/2N) sum |out - Y|^2.  Optimiser: Adam with bias correction.
// Every product is one tiled FP32 GEMM kernel on the FP32 matrix cores
// (64 x 64 tiles, 16-deep LDS slices, each wave a 32 x 32 block of
// v_mfma_f32_16x16x4f32 products) with transposition flags and a fused
// bias / tanh epilogue.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/yand.h"
#include "common.h"
#include "mlp.h"

namespace yand {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;    // output tile
constexpr int GK = 16;    // k slice
constexpr int GTH = 256;  // threads

// C[M x N] (ldc) = op(A)[M x K] op(B)[K x N]  (+ bias[n]) (tanh) (+ C if acc)
// op(A): TA ? A^T with A stored K x M (lda) : A stored M x K (lda)
// op(B): TB ? B^T with B stored N x K (ldb) : B stored K x N (ldb)
template <bool TA, bool TB>
__global__ void __launch_bounds__(GTH)
gemm_f32_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                const float* __restrict__ B, int ldb, float* __restrict__ C,
                int ldc, const float* __restrict__ bias, int act, int accum) {
  __shared__ float As[GK][GT + 4];
  __shared__ float Bs[GK][GT + 4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  // wave w: rows wm .. wm + 31, columns wn .. wn + 31 of the tile, as 2 x 2
  // blocks of 16 x 16; lane l feeds A[row l % 16][k l / 16] and
  // B[k l / 16][col l % 16] and holds C[4 (l / 16) + r][l % 16]
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + q * GTH;   // 0..1023 = 64 x 16
      int m, k;
      if (TA) {  // contiguous along m
        k = idx / GT;
        m = idx % GT;
      } else {   // contiguous along k
        m = idx / GK;
        k = idx % GK;
      }
      const int gm = m0 + m, gk = k0 + k;
      float v = 0.f;
      if (gm < M && gk < K) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      As[k][m] = v;
      int n, kb;
      if (TB) {  // B stored N x K: contiguous along k
        n = idx / GK;
        kb = idx % GK;
      } else {   // contiguous along n
        kb = idx / GT;
        n = idx % GT;
      }
      const int gn = n0 + n, gkb = k0 + kb;
      float w = 0.f;
      if (gn < N && gkb < K) w = TB ? B[(size_t)gn * ldb + gkb] : B[(size_t)gkb * ldb + gn];
      Bs[kb][n] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GK; k += 4) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[k + lk][wm + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[k + lk][wn + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j],
                                                          acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + 16 * i + 4 * lk + r;
        const int gn = n0 + wn + 16 * j + lr;
        if (gm >= M || gn >= N) continue;
        float v = acc[i][j][r];
        if (bias) v += bias[gn];
        if (act) v = tanhf(v);
        float* c = C + (size_t)gm * ldc + gn;
        *c = accum ? *c + v : v;
      }
}

// delta = (out - Y) / N; per-block partial of sum (out - Y)^2.
__global__ void mse_grad_kernel(const float* __restrict__ out,
                                const float* __restrict__ Y, int64_t count,
                                float invN, float* __restrict__ delta,
                                double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float r = out[i] - Y[i];
    delta[i] = r * invN;
    s += (double)r * (double)r;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// delta <- delta * (1 - a^2)
__global__ void tanh_back_kernel(float* __restrict__ delta,
                                 const float* __restrict__ a, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float t = a[i];
    delta[i] *= 1.f - t * t;
  }
}

// db[j] = sum_i delta[i][j] (column sums, fixed order)
__global__ void colsum_f32_kernel(const float* __restrict__ delta, int N,
                                  int cols, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int i = 0; i < N; ++i) s += delta[(size_t)i * cols + j];
  db[j] = s;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v,
                            int64_t count, float lr, float b1, float b2,
                            float c1, float c2, float eps) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Deterministic initial weights: counter-based splitmix64 -> Box-Muller,
// N(0, 1/fan_in) per weight, zero biases.
__device__ uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}
__global__ void init_layer_kernel(float* __restrict__ W, int64_t count,
                                  float scale, uint64_t seed, uint64_t offset) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t a = splitmix64(seed ^ (2 * (offset + i)));
    const uint64_t b = splitmix64(seed ^ (2 * (offset + i) + 1));
    const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
    const double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    W[i] = (float)(g * scale);
  }
}

unsigned grid1(int64_t count) {
  int64_t b = (count + 255) / 256;
  if (b > 2048) b = 2048;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

// ---------------------------------------------------------------- host ----

hipError_t mlp_gemm(hipStream_t st, bool ta, bool tb, int M, int N, int K,
                    const float* A, int lda, const float* B, int ldb, float* C,
                    int ldc, const float* bias, int act, int accum) {
  dim3 g((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT)),
      b(GTH);
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm_f32_kernel<false, false>), g, b, 0, st, M, N, K,
                       A, lda, B, ldb, C, ldc, bias, act, accum);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_f32_kernel<true, false>), g, b, 0, st, M, N, K, A,
                       lda, B, ldb, C, ldc, bias, act, accum);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_f32_kernel<false, true>), g, b, 0, st, M, N, K, A,
                       lda, B, ldb, C, ldc, bias, act, accum);
  else
    hipLaunchKernelGGL((gemm_f32_kernel<true, true>), g, b, 0, st, M, N, K, A,
                       lda, B, ldb, C, ldc, bias, act, accum);
  return hipGetLastError();
}

int Mlp::setup(int64_t in, int64_t out, int hidden_, int layers_,
               hipStream_t st) {
  in_dim = in;
  out_dim = out;
  hidden = hidden_;
  layers = layers_;
  stream = st;
  dims.clear();
  dims.push_back(in);
  for (int l = 0; l < layers - 1; ++l) dims.push_back(hidden);
  dims.push_back(out);
  offW.clear();
  offB.clear();
  int64_t off = 0;
  for (int l = 0; l < layers; ++l) {
    offW.push_back(off);
    off += dims[l] * dims[l + 1];
    offB.push_back(off);
    off += dims[l + 1];
  }
  nparam = off;
  size_t bytes = (size_t)nparam * sizeof(float);
  if (hipMalloc((void**)&params, bytes) != hipSuccess ||
      hipMalloc((void**)&grads, bytes) != hipSuccess ||
      hipMalloc((void**)&m, bytes) != hipSuccess ||
      hipMalloc((void**)&v, bytes) != hipSuccess)
    return YAND_ERR_OOM;
  if (hipMemsetAsync(grads, 0, bytes, st) != hipSuccess ||
      hipMemsetAsync(m, 0, bytes, st) != hipSuccess ||
      hipMemsetAsync(v, 0, bytes, st) != hipSuccess ||
      hipMemsetAsync(params, 0, bytes, st) != hipSuccess)
    return YAND_ERR_HIP;
  return YAND_OK;
}

int Mlp::ensure_batch(int64_t N) {
  if (N <= cap) return YAND_OK;
  // acts[0] is the caller's input, never owned
  for (size_t l = 1; l < acts.size(); ++l)
    if (acts[l]) (void)hipFree(acts[l]);
  acts.assign(layers + 1, nullptr);
  if (delta) (void)hipFree(delta);
  if (delta2) (void)hipFree(delta2);
  delta = delta2 = nullptr;
  cap = 0;
  int64_t widest = 0;
  for (int64_t d : dims) widest = std::max(widest, d);
  for (int l = 1; l <= layers; ++l)
    if (hipMalloc((void**)&acts[l], (size_t)N * dims[l] * sizeof(float)) !=
        hipSuccess)
      return YAND_ERR_OOM;
  if (hipMalloc((void**)&delta, (size_t)N * widest * sizeof(float)) !=
          hipSuccess ||
      hipMalloc((void**)&delta2, (size_t)N * widest * sizeof(float)) !=
          hipSuccess)
    return YAND_ERR_OOM;
  if (!part && hipMalloc((void**)&part, 2048 * sizeof(double)) != hipSuccess)
    return YAND_ERR_OOM;
  cap = N;
  return YAND_OK;
}

void Mlp::release() {
  for (size_t l = 1; l < acts.size(); ++l)
    if (acts[l]) (void)hipFree(acts[l]);
  acts.clear();
  float* ps[] = {params, grads, m, v, delta, delta2};
  for (float* p : ps)
    if (p) (void)hipFree(p);
  if (part) (void)hipFree(part);
  params = grads = m = v = delta = delta2 = nullptr;
  part = nullptr;
  cap = 0;
}

int Mlp::init_params(uint64_t seed) {
  for (int l = 0; l < layers; ++l) {
    const int64_t cnt = dims[l] * dims[l + 1];
    const float scale = 1.0f / std::sqrt((float)dims[l]);
    hipLaunchKernelGGL(init_layer_kernel, dim3(grid1(cnt)), dim3(256), 0,
                       stream, params + offW[l], cnt, scale, seed,
                       (uint64_t)offW[l]);
    if (hipMemsetAsync(params + offB[l], 0, dims[l + 1] * sizeof(float),
                       stream) != hipSuccess)
      return YAND_ERR_HIP;
  }
  return hipGetLastError() == hipSuccess ? YAND_OK : YAND_ERR_HIP;
}

int Mlp::forward(int64_t N, const float* X, float* out) {
  int rc = ensure_batch(N);
  if (rc) return rc;
  acts[0] = const_cast<float*>(X);
  for (int l = 0; l < layers; ++l) {
    const bool last = l == layers - 1;
    float* dst = last && out ? out : acts[l + 1];
    if (mlp_gemm(stream, false, false, (int)N, (int)dims[l + 1], (int)dims[l],
                 acts[l], (int)dims[l], params + offW[l], (int)dims[l + 1],
                 dst, (int)dims[l + 1], params + offB[l], last ? 0 : 1,
                 0) != hipSuccess)
      return YAND_ERR_HIP;
  }
  return YAND_OK;
}

// Gradient of the MSE loss into `grads`; loss (host) on request.
int Mlp::loss_grad(int64_t N, const float* X, const float* Y, double* loss) {
  int rc = forward(N, X, nullptr);
  if (rc) return rc;
  const int64_t cnt = N * out_dim;
  const unsigned nb = grid1(cnt);
  hipLaunchKernelGGL(mse_grad_kernel, dim3(nb), dim3(256), 0, stream,
                     acts[layers], Y, cnt, 1.0f / (float)N, delta, part);
  float* dcur = delta;
  float* dnext = delta2;
  for (int l = layers - 1; l >= 0; --l) {
    const int fi = (int)dims[l], fo = (int)dims[l + 1];
    // dW_l = a_l^T delta  (fi x fo)
    if (mlp_gemm(stream, true, false, fi, fo, (int)N, acts[l], fi, dcur, fo,
                 grads + offW[l], fo, nullptr, 0, 0) != hipSuccess)
      return YAND_ERR_HIP;
    hipLaunchKernelGGL(colsum_f32_kernel, dim3((fo + 255) / 256), dim3(256),
                       0, stream, dcur, (int)N, fo, grads + offB[l]);
    if (l > 0) {
      // delta_{l-1} = (delta W_l^T) * (1 - a_l^2)
      if (mlp_gemm(stream, false, true, (int)N, fi, fo, dcur, fo,
                   params + offW[l], fo, dnext, fi, nullptr, 0, 0) !=
          hipSuccess)
        return YAND_ERR_HIP;
      hipLaunchKernelGGL(tanh_back_kernel, dim3(grid1(N * fi)), dim3(256), 0,
                         stream, dnext, acts[l], N * fi);
      std::swap(dcur, dnext);
    }
  }
  if (hipGetLastError() != hipSuccess) return YAND_ERR_HIP;
  if (loss) {
    std::vector<double> hp(nb);
    if (hipMemcpyAsync(hp.data(), part, nb * sizeof(double),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return YAND_ERR_HIP;
    double s = 0.0;
    for (double x : hp) s += x;
    *loss = 0.5 * s / (double)N;
  }
  return YAND_OK;
}

int Mlp::adam(const float* g, double lr, int64_t t) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3(grid1(nparam)), dim3(256), 0, stream,
                     params, g, m, v, nparam, (float)lr, b1, b2, c1, c2, 1e-8f);
  return hipGetLastError() == hipSuccess ? YAND_OK : YAND_ERR_HIP;
}

// ------------------------------------------------ reduced coordinates ----

namespace {

constexpr int RT = 256;

// Block sum in a fixed order (one value per thread).
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = RT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// H x = x - kappa (v^T x) v with kappa = 2 / v^T v = 1 / (1 - 1/sqrt(n)),
// v_j = -1/sqrt(n) (j < n-1), v_{n-1} = 1 - 1/sqrt(n).
__global__ void __launch_bounds__(RT)
to_reduced_kernel(const double* __restrict__ W, int64_t n,
                  double* __restrict__ Y) {
  __shared__ double sh[RT];
  const double* w = W + (int64_t)blockIdx.x * n;
  double* y = Y + (int64_t)blockIdx.x * (n - 1);
  const double inv_n = 1.0 / (double)n, rs = 1.0 / sqrt((double)n);
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += RT) s += w[j] - inv_n;
  s = block_sum(s, sh);
  const double vx = (w[n - 1] - inv_n) - rs * s;
  const double kappa = 1.0 / (1.0 - rs);
  const double add = kappa * vx * rs;
  for (int64_t j = threadIdx.x; j < n - 1; j += RT) y[j] = (w[j] - inv_n) + add;
}

// W = 1/n + U y:  with e = (y, 0), v^T e = -(1/sqrt(n)) sum y, so
// W_j = 1/n + y_j + kappa (v^T e) / sqrt(n) (j < n-1), W_{n-1} = 1/n - v^T e.
template <class F>
__device__ void from_reduced_row(F yval, int64_t n, double* __restrict__ w,
                                 double* sh) {
  const double inv_n = 1.0 / (double)n, rs = 1.0 / sqrt((double)n);
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < n - 1; j += RT) s += yval(j);
  s = block_sum(s, sh);
  const double ve = -rs * s;
  const double kappa = 1.0 / (1.0 - rs);
  const double add = kappa * ve * rs;
  for (int64_t j = threadIdx.x; j < n - 1; j += RT) w[j] = inv_n + yval(j) + add;
  if (threadIdx.x == 0) w[n - 1] = inv_n - ve;
}

__global__ void __launch_bounds__(RT)
from_reduced_kernel(const double* __restrict__ Y, int64_t n,
                    double* __restrict__ W) {
  __shared__ double sh[RT];
  const double* y = Y + (int64_t)blockIdx.x * (n - 1);
  from_reduced_row([&](int64_t j) { return y[j]; }, n,
                   W + (int64_t)blockIdx.x * n, sh);
}

__global__ void __launch_bounds__(RT)
from_reduced_f32_kernel(const float* __restrict__ O,
                        const double* __restrict__ ybar, double s, int64_t n,
                        double* __restrict__ W) {
  __shared__ double sh[RT];
  const float* o = O + (int64_t)blockIdx.x * (n - 1);
  from_reduced_row([&](int64_t j) { return ybar[j] + s * (double)o[j]; }, n,
                   W + (int64_t)blockIdx.x * n, sh);
}

__global__ void col_stats_kernel(const double* __restrict__ Y, int64_t N,
                                 int64_t m, double* __restrict__ ybar,
                                 double* __restrict__ ss) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int64_t i = 0; i < N; ++i) s += Y[i * m + j];
  const double mean = s / (double)N;
  double q = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    const double d = Y[i * m + j] - mean;
    q += d * d;
  }
  ybar[j] = mean;
  ss[j] = q;
}

__global__ void standardize_kernel(const double* __restrict__ Y,
                                   const double* __restrict__ ybar,
                                   double inv_s, int64_t N, int64_t m,
                                   float* __restrict__ Z) {
  const int64_t cnt = N * m;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x)
    Z[i] = (float)((Y[i] - ybar[i % m]) * inv_s);
}

}  // namespace

hipError_t launch_to_reduced(const double* W, int64_t N, int64_t n, double* Y,
                             hipStream_t st) {
  hipLaunchKernelGGL(to_reduced_kernel, dim3((unsigned)N), dim3(RT), 0, st, W,
                     n, Y);
  return hipGetLastError();
}

hipError_t launch_from_reduced(const double* Y, int64_t N, int64_t n,
                               double* W, hipStream_t st) {
  hipLaunchKernelGGL(from_reduced_kernel, dim3((unsigned)N), dim3(RT), 0, st,
                     Y, n, W);
  return hipGetLastError();
}

hipError_t launch_from_reduced_f32(const float* O, const double* ybar,
                                   double s, int64_t N, int64_t n, double* W,
                                   hipStream_t st) {
  hipLaunchKernelGGL(from_reduced_f32_kernel, dim3((unsigned)N), dim3(RT), 0,
                     st, O, ybar, s, n, W);
  return hipGetLastError();
}

hipError_t launch_col_stats(const double* Y, int64_t N, int64_t m,
                            double* ybar, double* ss, hipStream_t st) {
  hipLaunchKernelGGL(col_stats_kernel, dim3((unsigned)((m + 255) / 256)),
                     dim3(256), 0, st, Y, N, m, ybar, ss);
  return hipGetLastError();
}

hipError_t launch_standardize(const double* Y, const double* ybar, double s,
                              int64_t N, int64_t m, float* Z, hipStream_t st) {
  hipLaunchKernelGGL(standardize_kernel, dim3(grid1(N * m)), dim3(256), 0, st,
                     Y, ybar, 1.0 / s, N, m, Z);
  return hipGetLastError();
}

}  // namespace yand

// ------------------------------------------------------------- C-ABI ----

using yand::Mlp;

extern "C" {

void yand_default_mlp_opts(yand_mlp_opts* o) {
  if (!o) return;
  o->hidden = 512;
  o->layers = 4;
  o->epochs = 2000;
  o->lr = 1e-3;
  o->seed = 0x5eedULL;
}

int yand_mlp_create(int64_t in_dim, int64_t out_dim, int hidden, int layers,
                    uint64_t seed, void* hip_stream, yand_mlp** out) {
  if (!out) return YAND_ERR_ARG;
  *out = nullptr;
  if (in_dim < 1 || out_dim < 1 || hidden < 1 || layers < 1 || layers > 16 ||
      in_dim > (1 << 20) || out_dim > (1 << 24) || hidden > (1 << 16))
    return YAND_ERR_ARG;
  yand_mlp* h = new yand_mlp();
  h->stream = (hipStream_t)hip_stream;
  int rc = h->net.setup(in_dim, out_dim, hidden, layers, h->stream);
  if (rc == YAND_OK) rc = h->net.init_params(seed);
  if (rc == YAND_OK && hipStreamSynchronize(h->stream) != hipSuccess)
    rc = YAND_ERR_HIP;
  if (rc != YAND_OK) {
    h->net.release();
    delete h;
    return rc;
  }
  *out = h;
  return YAND_OK;
}

int yand_mlp_destroy(yand_mlp* h) {
  if (!h) return YAND_OK;
  (void)hipStreamSynchronize(h->stream);
  h->net.release();
  if (h->ybar) (void)hipFree(h->ybar);
  delete h;
  return YAND_OK;
}

int64_t yand_mlp_num_params(const yand_mlp* h) {
  return h ? h->net.nparam : -1;
}

int yand_mlp_get_params(const yand_mlp* h, float* dst) {
  if (!h || !dst) return YAND_ERR_ARG;
  if (hipMemcpyAsync(dst, h->net.params, (size_t)h->net.nparam * 4,
                     hipMemcpyDeviceToDevice, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return YAND_ERR_HIP;
  return YAND_OK;
}

int yand_mlp_set_params(yand_mlp* h, const float* src) {
  if (!h || !src) return YAND_ERR_ARG;
  if (hipMemcpyAsync(h->net.params, src, (size_t)h->net.nparam * 4,
                     hipMemcpyDeviceToDevice, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return YAND_ERR_HIP;
  return YAND_OK;
}

int yand_mlp_forward(yand_mlp* h, int64_t N, const float* X, float* out) {
  if (!h || !X || !out || N < 1 || N > (1 << 24)) return YAND_ERR_ARG;
  int rc = h->net.forward(N, X, out);
  if (rc) return rc;
  return hipStreamSynchronize(h->stream) == hipSuccess ? YAND_OK
                                                       : YAND_ERR_HIP;
}

int yand_mlp_loss_grad(yand_mlp* h, int64_t N, const float* X, const float* Y,
                       float* grad, double* loss) {
  if (!h || !X || !Y || N < 1 || N > (1 << 24)) return YAND_ERR_ARG;
  int rc = h->net.loss_grad(N, X, Y, loss);
  if (rc) return rc;
  if (grad && hipMemcpyAsync(grad, h->net.grads, (size_t)h->net.nparam * 4,
                             hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
    return YAND_ERR_HIP;
  return hipStreamSynchronize(h->stream) == hipSuccess ? YAND_OK
                                                       : YAND_ERR_HIP;
}

int yand_mlp_adam_step(yand_mlp* h, const float* grad, double lr) {
  if (!h || !(lr > 0.0)) return YAND_ERR_ARG;
  h->t += 1;
  int rc = h->net.adam(grad ? grad : h->net.grads, lr, h->t);
  if (rc) return rc;
  return hipStreamSynchronize(h->stream) == hipSuccess ? YAND_OK
                                                       : YAND_ERR_HIP;
}

int yand_reduced_coords(int64_t N, int64_t n, const double* W, double* Y,
                        void* hip_stream) {
  if (N < 1 || n < 2 || !W || !Y || N > (1 << 30)) return YAND_ERR_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  if (yand::launch_to_reduced(W, N, n, Y, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return YAND_ERR_HIP;
  return YAND_OK;
}

int yand_from_reduced(int64_t N, int64_t n, const double* Y, double* W,
                      void* hip_stream) {
  if (N < 1 || n < 2 || !W || !Y || N > (1 << 30)) return YAND_ERR_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  if (yand::launch_from_reduced(Y, N, n, W, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return YAND_ERR_HIP;
  return YAND_OK;
}

}  // extern "C"
