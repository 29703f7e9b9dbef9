// Setup, decision and utility kernels of the projected-gradient detector-tomography
// solver (gfx950): band edges and tail mass, recursion tables, anchors, Hessian
// diagonal, power-iteration normalisation, the accept/reject decision, the standalone
// row projection and array fills.  The band-product kernels are in pdt_band.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <type_traits>

#include "pdt_decide.h"
#include "pdt_device.h"
#include "pdt_internal.h"
#include "pdt_pmf.h"

namespace pdt {

// ---------------------------------------------------------------------------------------
// Fixed-order reduction of the partials and the accept/reject decision.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void decide_kernel(const double* partials, int n, SolverState* st,
                                                     double* history, int mode, const double* rpart, int nr) {
  decide_body<256>(partials, n, st, history, mode, rpart, nr);
}

template <typename TS>
__global__ __launch_bounds__(256) void decide_batch_kernel(const BatchInst<TS>* insts, int mode) {
  const BatchInst<TS>& I = insts[blockIdx.x];
  decide_body<256>(I.b.partials, I.n_dt, I.st, I.b.history, mode, I.b.rpart, I.n_mt);
}

// Batches: every instance's state into one array (one copy to the host per chunk), and
// the host's stop flags into the states (instances whose phase is over).
__global__ __launch_bounds__(256) void gather_states_kernel(SolverState* const* st, int n, SolverState* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = *st[k];
}

__global__ __launch_bounds__(256) void mark_done_kernel(SolverState* const* st, const int* flags, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && flags[k]) st[k]->done = 1;
}

__global__ __launch_bounds__(256) void reduce_sum_kernel(const double* partials, int n, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += partials[k];
  const double f = block_sum256(s, sh);
  if (threadIdx.x == 0) *out = f;
}

// ---------------------------------------------------------------------------------------
// Setup: band edges and lumped tail mass per probe (one thread per probe).
// ---------------------------------------------------------------------------------------
__global__ void setup_bands_kernel(const double* mu, int D, int M, double tau, int lump, int* lo,
                                   int* hi, double* tail) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  const double m_ = mu[d];
  const double t = lump ? poisson_upper_tail(m_, M - 1) : 0.0;
  tail[d] = t;
  if (tau <= 0.0) {
    lo[d] = 0;
    hi[d] = M - 1;
    return;
  }
  const int last = M - 1;
  auto value = [&](int m) -> double { return (lump && m == last) ? t : poisson_pmf(m, m_); };
  double fl = floor(m_);
  int mode = fl > (double)last ? last : (int)fl;
  if (value(mode) < tau) {
    // the row never reaches the threshold (tail column excepted)
    if (lump && t >= tau) {
      lo[d] = last;
      hi[d] = last;
    } else {
      lo[d] = M;
      hi[d] = -1;
    }
    return;
  }
  // first m in [0, mode] with value >= tau (values non-decreasing there)
  int a = 0, bnd = mode;
  if (value(0) >= tau) {
    bnd = 0;
  } else {
    while (bnd - a > 1) {
      const int c = a + (bnd - a) / 2;
      if (value(c) >= tau) bnd = c; else a = c;
    }
  }
  lo[d] = bnd;
  // last m in [mode, end] with pmf >= tau (non-increasing there)
  int end = lump ? last - 1 : last;
  int h;
  if (mode >= end) {
    h = mode;
  } else if (value(end) >= tau) {
    h = end;
  } else {
    int g = mode, e = end;
    while (e - g > 1) {
      const int c = g + (e - g) / 2;
      if (value(c) >= tau) g = c; else e = c;
    }
    h = g;
  }
  if (lump && t >= tau) h = last;
  hi[d] = h;
}

__global__ void fill_rinv_kernel(double* rinv, double* r4, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  rinv[m] = m == 0 ? 0.0 : 1.0 / (double)m;
  const double a = (double)(m + 1) * (double)(m + 4);  // exact below 2^53
  const double b = (double)(m + 2) * (double)(m + 3);
  r4[m] = 1.0 / (a * b);
}

// F[d][16 t] for every probe d whose band is considered by row tile t (0 where the
// band misses the tile): the transposed product's anchors, fixed for the whole solve.
__global__ void setup_anchors_kernel(const double* mu, const int* lo, const int* hi, const int* mt_dlo,
                                     const int* mt_dhi, const long long* mt_aoff, int n_mt, int M, int lump,
                                     const double* tail, double* anchors) {
  const int t = blockIdx.x;
  if (t >= n_mt) return;
  const int dlo = mt_dlo[t], dhi = mt_dhi[t];
  const int m0 = 16 * t;
  double* out = anchors + mt_aoff[t];
  for (int d = dlo + (int)threadIdx.x; d <= dhi; d += (int)blockDim.x) {
    const int blo = lo[d], bhi = hi[d];
    double v = 0.0;
    if (m0 <= bhi && m0 + 15 >= blo) v = (lump && m0 == M - 1) ? tail[d] : poisson_pmf(m0, mu[d]);
    out[d - dlo] = v;
  }
}

// ---------------------------------------------------------------------------------------
// Row-wise simplex projection of a general [rows][cols] array: one wave per row.
// ---------------------------------------------------------------------------------------
template <typename T, int V>
__global__ __launch_bounds__(64) void project_rows_kernel(const T* X, T* Y, long long rows, int cols,
                                                          int ld_in, int ld_out) {
  const long long row = blockIdx.x;
  if (row >= rows) return;
  const int lane = threadIdx.x;
  T z[1][V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = v * 64 + lane;
    z[0][v] = c < cols ? X[row * ld_in + c] : neg_huge<T>();
  }
  T tau[1];
  simplex_threshold<T, 64, V, 1, 8>(z, tau);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = v * 64 + lane;
    if (c < ld_out) Y[row * ld_out + c] = c < cols ? fmax(z[0][v] - tau[0], (T)0) : (T)0;
  }
}

// power iteration on W^(1/2) H W^(1/2) with the iterate kept as u = W^(1/2) v:
// lambda = sqrt(sum_m w_m G_m^2), V_m = w_m G_m / lambda (w = null: all ones).  Two passes:
// per-block partial sums over a fixed row partition, then every block forms lambda from
// the partials in the same fixed order and scales its rows.
constexpr int kNormBlocks = 512;

__global__ __launch_bounds__(256) void power_partial_kernel(const double* G, int M, int ld, const double* w,
                                                            double* partials) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long long m = (long long)blockIdx.x * 256 + threadIdx.x; m < M; m += (long long)gridDim.x * 256) {
    const double g = G[(size_t)m * ld];
    s += (w ? w[m] : 1.0) * g * g;
  }
  const double t = block_sum256(s, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void power_scale_kernel(const double* G, double* V, int M, int ld, const double* w,
                                                          const double* partials, int nb, double* lam_out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) s += partials[k];
  const double lam = sqrt(block_sum256(s, sh));
  const double inv = lam > 0.0 ? 1.0 / lam : 0.0;
  for (long long m = (long long)blockIdx.x * 256 + threadIdx.x; m < M; m += (long long)gridDim.x * 256)
    V[(size_t)m * ld] = (w ? w[m] : 1.0) * G[(size_t)m * ld] * inv;
  if (blockIdx.x == 0 && threadIdx.x == 0) *lam_out = lam;
}

// Hessian diagonal of row m: 2 sum_d F[d][m]^2 over the probes whose band holds m (FP64
// Loader values, summed in increasing d), plus 2 gamma L[m][m] (1 at the ends, 2 inside).
__global__ __launch_bounds__(256) void setup_hdiag_kernel(ProbView pv, double* hdiag) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= pv.M) return;
  const int t = m >> 4;
  const int dlo = pv.mt_dlo[t], dhi = pv.mt_dhi[t];
  const bool lumped = pv.lump && m == pv.M - 1;
  double s = 0.0;
  for (int d = dlo; d <= dhi; ++d) {
    if (m < pv.lo[d] || m > pv.hi[d]) continue;
    const double v = lumped ? pv.tail[d] : poisson_pmf(m, pv.mu[d]);
    s += v * v;
  }
  const double ld = pv.M < 2 ? 0.0 : ((m == 0 || m == pv.M - 1) ? 1.0 : 2.0);
  hdiag[m] = 2.0 * s + 2.0 * pv.gamma * ld;
}

template <typename T>
__global__ void fill_rows_kernel(T* X, long long rows, int cols, int ld, T value) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * ld) return;
  const int c = (int)(idx % ld);
  X[idx] = c < cols ? value : (T)0;
}

template <typename T>
__global__ __launch_bounds__(256) void resid_cur_kernel(Bufs<T> b, const SolverState* st, long long n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  b.R_rej[idx] = b.O[st->ix_cur][idx] - b.P[idx];
}

template <typename Ts, typename Td>
__global__ void convert_pad_kernel(const Ts* src, Td* dst, long long rows, int cols, int ld_src,
                                   int ld_dst) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = rows * ld_dst;
  if (idx >= total) return;
  const long long r = idx / ld_dst;
  const int c = (int)(idx - r * ld_dst);
  dst[idx] = c < cols ? (Td)src[r * ld_src + c] : (Td)0;
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
int fx_num_tiles(const ProbView& pv) { return (pv.D + 15) / 16; }
int fx_num_waves(const ProbView& pv) {
  const int t = fx_num_tiles(pv);
  return pv.fx_split > 1 ? t * pv.fx_split + t : t;
}
int ftr_num_waves(const ProbView& pv) { return (pv.M + 15) / 16; }

template <typename TS>
hipError_t launch_decide_batch(const BatchInst<TS>* insts, int n_inst, int mode, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL((decide_batch_kernel<TS>), dim3(n_inst), dim3(256), 0, s, insts, mode);
  return hipGetLastError();
}

template hipError_t launch_decide_batch<double>(const BatchInst<double>*, int, int, hipStream_t);
template hipError_t launch_decide_batch<float>(const BatchInst<float>*, int, int, hipStream_t);

hipError_t launch_decide(const double* partials, int n, SolverState* st, double* history, int mode,
                         hipStream_t s, const double* rpart, int nr) {
  hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(256), 0, s, partials, n, st, history, mode, rpart, nr);
  return hipGetLastError();
}

hipError_t launch_gather_states(SolverState* const* st, int n, SolverState* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_states_kernel, dim3((n + 255) / 256), dim3(256), 0, s, st, n, out);
  return hipGetLastError();
}

hipError_t launch_mark_done(SolverState* const* st, const int* flags, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mark_done_kernel, dim3((n + 255) / 256), dim3(256), 0, s, st, flags, n);
  return hipGetLastError();
}

hipError_t launch_reduce_sum(const double* partials, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(256), 0, s, partials, n, out);
  return hipGetLastError();
}

hipError_t launch_setup_bands(const double* mu, int D, int M, double tau, int lump, int* lo, int* hi,
                              double* tail, hipStream_t s) {
  hipLaunchKernelGGL(setup_bands_kernel, dim3((D + 127) / 128), dim3(128), 0, s, mu, D, M, tau, lump, lo,
                     hi, tail);
  return hipGetLastError();
}

hipError_t launch_fill_rinv(double* rinv, double* r4, int n, hipStream_t s) {
  hipLaunchKernelGGL(fill_rinv_kernel, dim3((n + 255) / 256), dim3(256), 0, s, rinv, r4, n);
  return hipGetLastError();
}

hipError_t launch_setup_anchors(const ProbView& pv, const long long* mt_aoff, double* anchors, hipStream_t s) {
  const int n_mt = (pv.M + 15) / 16;
  hipLaunchKernelGGL(setup_anchors_kernel, dim3(n_mt), dim3(256), 0, s, pv.mu, pv.lo, pv.hi, pv.mt_dlo, pv.mt_dhi,
                     mt_aoff, n_mt, pv.M, pv.lump, pv.tail, anchors);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_project_rows(const T* X, T* Y, long long rows, int cols, int ld_in, int ld_out,
                               hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int v = (cols + 63) / 64;
  const dim3 g((unsigned)rows), blk(64);
  if (v <= 1) hipLaunchKernelGGL((project_rows_kernel<T, 1>), g, blk, 0, s, X, Y, rows, cols, ld_in, ld_out);
  else if (v <= 2) hipLaunchKernelGGL((project_rows_kernel<T, 2>), g, blk, 0, s, X, Y, rows, cols, ld_in, ld_out);
  else if (v <= 4) hipLaunchKernelGGL((project_rows_kernel<T, 4>), g, blk, 0, s, X, Y, rows, cols, ld_in, ld_out);
  else if (v <= 8) hipLaunchKernelGGL((project_rows_kernel<T, 8>), g, blk, 0, s, X, Y, rows, cols, ld_in, ld_out);
  else if (v <= 16) hipLaunchKernelGGL((project_rows_kernel<T, 16>), g, blk, 0, s, X, Y, rows, cols, ld_in, ld_out);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_power_normalize(double* G, double* V, int M, int ld, const double* w, double* scratch,
                                  double* lam_out, hipStream_t s) {
  const int nb = std::max(1, std::min(kNormBlocks, (M + 255) / 256));
  hipLaunchKernelGGL(power_partial_kernel, dim3(nb), dim3(256), 0, s, G, M, ld, w, scratch);
  hipLaunchKernelGGL(power_scale_kernel, dim3(nb), dim3(256), 0, s, G, V, M, ld, w, scratch, nb, lam_out);
  return hipGetLastError();
}

hipError_t launch_setup_hdiag(const ProbView& pv, double* hdiag, hipStream_t s) {
  if (pv.M <= 0) return hipSuccess;
  hipLaunchKernelGGL(setup_hdiag_kernel, dim3((pv.M + 255) / 256), dim3(256), 0, s, pv, hdiag);
  return hipGetLastError();
}

template <typename Ts, typename Td>
hipError_t launch_convert_pad(const Ts* src, Td* dst, long long rows, int cols, int ld_src, int ld_dst,
                              hipStream_t s) {
  const long long total = rows * ld_dst;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_pad_kernel<Ts, Td>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     src, dst, rows, cols, ld_src, ld_dst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_rows(T* X, long long rows, int cols, int ld, T value, hipStream_t s) {
  const long long total = rows * ld;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL((fill_rows_kernel<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, rows,
                     cols, ld, value);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_resid_cur(const Bufs<T>& b, const SolverState* st, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((resid_cur_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b, st, n);
  return hipGetLastError();
}
template hipError_t launch_resid_cur<double>(const Bufs<double>&, const SolverState*, long long, hipStream_t);
template hipError_t launch_resid_cur<float>(const Bufs<float>&, const SolverState*, long long, hipStream_t);

template hipError_t launch_fill_rows<double>(double*, long long, int, int, double, hipStream_t);
template hipError_t launch_fill_rows<float>(float*, long long, int, int, float, hipStream_t);

template hipError_t launch_project_rows<double>(const double*, double*, long long, int, int, int, hipStream_t);
template hipError_t launch_project_rows<float>(const float*, float*, long long, int, int, int, hipStream_t);
template hipError_t launch_convert_pad<double, double>(const double*, double*, long long, int, int, int,
                                                       hipStream_t);
template hipError_t launch_convert_pad<double, float>(const double*, float*, long long, int, int, int,
                                                      hipStream_t);
template hipError_t launch_convert_pad<float, double>(const float*, double*, long long, int, int, int,
                                                      hipStream_t);

}  // namespace pdt
