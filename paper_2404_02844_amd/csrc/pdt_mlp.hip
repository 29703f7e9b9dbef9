// Warm-start network kernels (gfx950): BF16 MFMA GEMMs with FP32 accumulation, the
// tanh-GELU activation and its derivative, the MSE loss gradient, bias gradients,
// Adam on FP32 master weights, and the feature / assembly steps of the learned start.
//
// Network: 4 linear layers n_in -> H -> H -> H -> n_out, GELU after the first three;
// weights W_l are [out][in] row-major, a layer computes y = x W_l^T + b_l.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pdt_mlp.h"

namespace pdt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu_f(float x) {
  const float u = 0.7978845608028654f * (x + 0.044715f * x * x * x);
  return 0.5f * x * (1.0f + tanhf(u));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
  const float u = 0.7978845608028654f * (x + 0.044715f * x * x * x);
  const float t = tanhf(u);
  const float du = 0.7978845608028654f * (1.0f + 3.0f * 0.044715f * x * x);
  return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * du;
}

// ---------------------------------------------------------------------------------------
// C[M][N] = op(A)[M][K] op(B)[K][N] (+ bias[n]) (then GELU), BF16 operands, FP32 sums.
// A(m, k) = a_trans ? A[k * lda + m] : A[m * lda + k];  B(k, n) = b_trans ? B[n * ldb + k]
// : B[k * ldb + n].  64 x 64 output tile per workgroup of 4 waves (each 32 x 32 = 2 x 2
// MFMA 16x16x32 tiles), K in steps of 32 staged through LDS as [row][k].
// v_mfma_f32_16x16x32_bf16 lane layout: lane l holds A[l%16][8(l/16) + e],
// B[8(l/16) + e][l%16] (e = 0..7) and C[4(l/16) + r][l%16].
// ---------------------------------------------------------------------------------------
constexpr int GT = 64;
constexpr int GK = 32;
constexpr int GKP = GK + 8;  // padded LDS row (80 bytes, keeps 16-byte alignment)

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[GT][GKP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[GT][GKP];
  const int tid = threadIdx.x;
  const int wv = tid >> 6, lane = tid & 63, i = lane & 15, gq = lane >> 4;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int wr = 32 * (wv >> 1), wc = 32 * (wv & 1);
  f32x4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4v{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += GK) {
#pragma unroll
    for (int e = 0; e < (GT * GK) / 256; ++e) {
      const int idx = e * 256 + tid;
      int r, k;
      if (g.a_trans) { k = idx / GT; r = idx % GT; } else { r = idx / GK; k = idx % GK; }
      const int gm = m0 + r, gk = k0 + k;
      __bf16 v = (__bf16)0.0f;
      if (gm < g.M && gk < g.K) v = g.A[g.a_trans ? (long long)gk * g.lda + gm : (long long)gm * g.lda + gk];
      As[r][k] = v;
      int c, kk;
      if (g.b_trans) { c = idx / GK; kk = idx % GK; } else { kk = idx / GT; c = idx % GT; }
      const int gn = n0 + c, gk2 = k0 + kk;
      __bf16 w = (__bf16)0.0f;
      if (gn < g.N && gk2 < g.K) w = g.B[g.b_trans ? (long long)gn * g.ldb + gk2 : (long long)gk2 * g.ldb + gn];
      Bs[c][kk] = w;
    }
    __syncthreads();
    bf16x8 av[2], bv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      av[t] = *reinterpret_cast<const bf16x8*>(&As[wr + 16 * t + i][8 * gq]);
      bv[t] = *reinterpret_cast<const bf16x8*>(&Bs[wc + 16 * t + i][8 * gq]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr + 16 * a + 4 * gq + r;
        const int col = n0 + wc + 16 * b + i;
        if (row < g.M && col < g.N) {
          float v = acc[a][b][r];
          if (g.bias) v += g.bias[col];
          const long long o = (long long)row * g.ldc + col;
          if (g.preact) g.preact[o] = v;
          if (g.gelu) v = gelu_f(v);
          if (g.C) g.C[o] = v;
          if (g.Cbf) g.Cbf[o] = (__bf16)v;
        }
      }
}

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// elementwise pieces of the backward pass and the optimiser
// ---------------------------------------------------------------------------------------
// dY = 2 (Y - T) / count (count = rows * cols); per-block FP64 partials of sum (Y - T)^2
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* Y, const float* T, long long n, float scale,
                                                       float* dY, __bf16* dYb, double* partials) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
    const float d = Y[k] - T[k];
    s += (double)d * (double)d;
    const float g = scale * d;
    if (dY) dY[k] = g;
    if (dYb) dYb[k] = (__bf16)g;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && partials) partials[blockIdx.x] = sh[0];
}

// dZ = dH * gelu'(Z), written as BF16 (operand of the next GEMMs) and FP32
__global__ void gelu_back_kernel(const float* dH, const float* Z, long long n, float* dZ, __bf16* dZb) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float v = dH[k] * gelu_grad_f(Z[k]);
  dZ[k] = v;
  dZb[k] = (__bf16)v;
}

// db[c] = sum_r dZ[r][c], fixed order over r
__global__ void colsum_kernel(const float* dZ, int rows, int cols, float* db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += dZ[(long long)r * cols + c];
  db[c] = s;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                            float eps, float c1, float c2, __bf16* pbf, long long wcount) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  const float upd = lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  const float pk = p[k] - upd;
  p[k] = pk;
  if (pbf && k < wcount) pbf[k] = (__bf16)pk;
}

__global__ void f32_to_bf16_kernel(const float* a, __bf16* b, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = (__bf16)a[k];
}

// features of outcome n (rows 0..bins): P[:, n] linearly interpolated at 256 equally
// spaced mean photon numbers between mu[0] and mu[D-1], then n / bins and bins / 128
__global__ void features_kernel(const double* mu, const double* P, int D, int Npad, int bins, int n_grid,
                                float* X, __bf16* Xb) {
  const int n = blockIdx.x;
  const int j = threadIdx.x;
  const int n_in = n_grid + 2;
  if (n > bins) return;
  for (int q = j; q < n_in; q += blockDim.x) {
    float v;
    if (q < n_grid) {
      const double g = mu[0] + (mu[D - 1] - mu[0]) * (double)q / (double)(n_grid - 1);
      // last probe index with mu <= g
      int lo = 0, hi = D - 1;
      while (hi - lo > 1) {
        const int c = (lo + hi) >> 1;
        if (mu[c] <= g) lo = c; else hi = c;
      }
      double val;
      if (D == 1 || g <= mu[0]) {
        val = P[n];
      } else if (g >= mu[D - 1]) {
        val = P[(long long)(D - 1) * Npad + n];
      } else {
        const double w = (mu[hi] > mu[lo]) ? (g - mu[lo]) / (mu[hi] - mu[lo]) : 0.0;
        val = P[(long long)lo * Npad + n] * (1.0 - w) + P[(long long)hi * Npad + n] * w;
      }
      v = (float)val;
    } else if (q == n_grid) {
      v = (float)n / (float)bins;
    } else {
      v = (float)bins / 128.0f;
    }
    X[(long long)n * n_in + q] = v;
    if (Xb) Xb[(long long)n * n_in + q] = (__bf16)v;
  }
}

// Pi0[m][n] = Y[n][m] for the real outcomes n <= bins, 0 for the padding outcomes
__global__ void assemble_kernel(const float* Y, int M, int bins, int N, int Npad, double* Pi0) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)M * Npad) return;
  const int m = (int)(k / Npad), n = (int)(k % Npad);
  Pi0[k] = (n <= bins && n < N) ? (double)Y[(long long)n * M + m] : 0.0;
}

hipError_t launch_mse_grad(const float* Y, const float* T, long long n, float scale, float* dY, __bf16* dYb,
                           double* partials, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks), dim3(256), 0, s, Y, T, n, scale, dY, dYb, partials);
  return hipGetLastError();
}
hipError_t launch_gelu_back(const float* dH, const float* Z, long long n, float* dZ, __bf16* dZb, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gelu_back_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dH, Z, n, dZ, dZb);
  return hipGetLastError();
}
hipError_t launch_colsum(const float* dZ, int rows, int cols, float* db, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3((cols + 255) / 256), dim3(256), 0, s, dZ, rows, cols, db);
  return hipGetLastError();
}
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, int t, __bf16* pbf, long long wcount, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                     c1, c2, pbf, wcount);
  return hipGetLastError();
}
hipError_t launch_f32_to_bf16(const float* a, __bf16* b, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}
hipError_t launch_features(const double* mu, const double* P, int D, int Npad, int bins, int n_grid, float* X,
                           __bf16* Xb, hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3(bins + 1), dim3(256), 0, s, mu, P, D, Npad, bins, n_grid, X, Xb);
  return hipGetLastError();
}
hipError_t launch_assemble(const float* Y, int M, int bins, int N, int Npad, double* Pi0, hipStream_t s) {
  const long long n = (long long)M * Npad;
  hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Y, M, bins, N, Npad, Pi0);
  return hipGetLastError();
}

}  // namespace pdt
