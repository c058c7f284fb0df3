// Warm-start MLP: FP32 network state and the launchers of mlp.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace yand {

// Fully connected network dims[0] -> ... -> dims[layers] with tanh on every
// hidden layer and a linear output.  Parameters live in one FP32 buffer,
// layer by layer: W_l (dims[l] x dims[l+1], row-major) then b_l.
struct Mlp {
  int64_t in_dim = 0, out_dim = 0;
  int hidden = 0, layers = 0;
  std::vector<int64_t> dims, offW, offB;
  int64_t nparam = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  std::vector<float*> acts;  // acts[0] = input (borrowed), acts[l] owned
  float *delta = nullptr, *delta2 = nullptr;
  double* part = nullptr;    // loss partial sums
  int64_t cap = 0;           // batch rows the activation buffers hold
  hipStream_t stream = nullptr;

  int setup(int64_t in, int64_t out, int hidden, int layers, hipStream_t st);
  int ensure_batch(int64_t N);
  int init_params(uint64_t seed);
  // out (N x out_dim), nullable: the output stays in acts[layers]
  int forward(int64_t N, const float* X, float* out);
  // forward, then the gradient of (1/2N) sum |out - Y|^2 into grads
  int loss_grad(int64_t N, const float* X, const float* Y, double* loss);
  // one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with step count t >= 1
  int adam(const float* g, double lr, int64_t t);
  void release();
};

hipError_t mlp_gemm(hipStream_t st, bool ta, bool tb, int M, int N, int K,
                    const float* A, int lda, const float* B, int ldb, float* C,
                    int ldc, const float* bias, int act, int accum);

// Reduced coordinates in the fixed Householder basis of the budget tangent
// space {1^T x = 0}: H = I - 2 v v^T / v^T v, v = e_n - 1/sqrt(n) 1, whose
// first n-1 columns U are orthonormal and span that space.
//   to_reduced:   Y[b] = U^T (W[b] - 1/n)           (N x n -> N x (n-1))
//   from_reduced: W[b] = 1/n + U (ybar + s * O[b])  (N x (n-1) -> N x n)
hipError_t launch_to_reduced(const double* W, int64_t N, int64_t n,
                             double* Y, hipStream_t st);
hipError_t launch_from_reduced(const double* Y, int64_t N, int64_t n,
                               double* W, hipStream_t st);
hipError_t launch_from_reduced_f32(const float* O, const double* ybar,
                                   double s, int64_t N, int64_t n, double* W,
                                   hipStream_t st);
// Column means ybar (m) of Y (N x m) and per-column sums of squared
// deviations ss (m), then Z = (Y - ybar) / s as FP32.
hipError_t launch_col_stats(const double* Y, int64_t N, int64_t m,
                            double* ybar, double* ss, hipStream_t st);
hipError_t launch_standardize(const double* Y, const double* ybar, double s,
                              int64_t N, int64_t m, float* Z, hipStream_t st);

}  // namespace yand

// Handle behind the opaque yand_mlp of the C-ABI.
struct yand_mlp {
  yand::Mlp net;
  hipStream_t stream = nullptr;
  int64_t t = 0;  // Adam steps taken
  // warm-start model (set by training on solutions of one universe size)
  int64_t n = 0;
  std::vector<double> fmean, fscale;
  double* ybar = nullptr;  // device, n - 1
  double yscale = 1.0;
};
