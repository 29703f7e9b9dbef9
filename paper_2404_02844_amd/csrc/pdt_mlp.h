// Internal declarations of the warm-start network kernels (pdt_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace pdt {

struct GemmArgs {
  const __bf16* A;
  const __bf16* B;
  float* C;          // FP32 result (nullable)
  __bf16* Cbf;       // BF16 copy of the result (nullable)
  float* preact;     // result before the activation (nullable)
  const float* bias; // per output column (nullable)
  int M, N, K;
  long long lda, ldb, ldc;
  int a_trans, b_trans, gelu;
};

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s);
hipError_t launch_mse_grad(const float* Y, const float* T, long long n, float scale, float* dY, __bf16* dYb,
                           double* partials, int blocks, hipStream_t s);
hipError_t launch_gelu_back(const float* dH, const float* Z, long long n, float* dZ, __bf16* dZb, hipStream_t s);
hipError_t launch_colsum(const float* dZ, int rows, int cols, float* db, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, int t, __bf16* pbf, long long wcount, hipStream_t s);
hipError_t launch_f32_to_bf16(const float* a, __bf16* b, long long n, hipStream_t s);
hipError_t launch_features(const double* mu, const double* P, int D, int Npad, int bins, int n_grid, float* X,
                           __bf16* Xb, hipStream_t s);
hipError_t launch_assemble(const float* Y, int M, int bins, int N, int Npad, double* Pi0, hipStream_t s);

}  // namespace pdt
