// Fixed-order reduction of the per-workgroup partials of f and the accept / reject
// decision with the momentum scalars (Nesterov's t, beta) of the iteration.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "pdt_internal.h"

namespace pdt {

__device__ __forceinline__ double block_sum256(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  return sh[0];
}

// p[tid] + p[tid + 256] + ... over the indices below n, added in that order from 0.0.
// The loads of up to 8 terms go out before their additions: a plain loop waits for each
// load in turn, and these partials come from HBM (written by another kernel).
__device__ __forceinline__ double strided_sum256(const double* p, int n, int tid) {
  constexpr int U = 8;
  double s = 0.0;
  for (int k0 = tid; k0 < n; k0 += U * 256) {
    double v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int k = k0 + j * 256;
      v[j] = k < n ? p[k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (k0 + j * 256 < n) s += v[j];
  }
  return s;
}

// The same sum over the values of the first 256 threads of a block of BS >= 256 threads
// (the others only join the barriers), so every block size adds in one order.
template <int BS>
__device__ __forceinline__ double first256_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  if (tid < 256) sh[tid] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  return sh[0];
}

// Run by every thread of one block of BS threads (BS = 256, or the forward product's
// workgroup when it takes the decision itself); the first 256 threads sum the partials.
// Gradient-restart test of the step just taken (O'Donoghue and Candes): the sum of the
// step's per-tile partials of sum_m (1 / w_m) sum_n (Y - X_new)(X_new - X_cur), added in
// one fixed order by every block that needs it (the forward product, for the residual it
// hands the next step, and the decision), so they all take the same decision.
template <int BS>
__device__ __forceinline__ bool restart_test(const double* rpart, int nr) {
  __shared__ double shr[256];
  const double s = threadIdx.x < 256 ? strided_sum256(rpart, nr, threadIdx.x) : 0.0;
  return first256_sum<BS>(s, shr) > 0.0;
}

template <int BS>
__device__ __forceinline__ void decide_body(const double* partials, int n, SolverState* st, double* history,
                                            int mode, const double* rpart = nullptr, int nr = 0) {
  __shared__ double sh[256];
  if ((mode == DEC_ITER || mode == DEC_RESYNC) && st->done) return;
  const bool reset = (mode == DEC_ITER && rpart) ? restart_test<BS>(rpart, nr) : false;
  const double s = threadIdx.x < 256 ? strided_sum256(partials, n, threadIdx.x) : 0.0;
  const double f = first256_sum<BS>(s, sh);
  if (mode == DEC_KKT) {
    // KKT residual sqrt(mean((X (g - min_n g))^2)) and Frank-Wolfe gap
    // sum_i (<g_i, X_i> - min_n g_i) of the current iterate
    __syncthreads();
    const double s2 = threadIdx.x < 256 ? strided_sum256(partials + n, n, threadIdx.x) : 0.0;
    const double fw = first256_sum<BS>(s2, sh);
    if (threadIdx.x != 0) return;
    st->kkt = sqrt(f / st->mn);
    st->fw = fw;
    if (st->kkt_tol > 0.0 && st->kkt <= st->kkt_tol) {
      st->done = 1;
      st->kkt_hit = 1;
    }
    return;
  }
  if (threadIdx.x != 0) return;
  if (mode == DEC_EVAL) {
    st->f_eval = f;
    return;
  }
  if (mode == DEC_RESYNC) {
    // the exact objective of the current iterate replaces the one accumulated from
    // FP32 updates, so later acceptance tests compare against the true value
    st->f_cur = f;
    st->f_new = f;
    if (st->f_star > 0.0 && f - st->f_star <= st->rel_tol * st->f_star) st->done = 1;
    return;
  }
  if (mode == DEC_INIT) {
    st->f_cur = f;
    st->f_new = f;
    st->t = 1.0;
    st->beta = 0.0;
    st->ix_cur = 0;
    st->ix_prev = 0;
    st->ix_new = 1;
    st->sel_acc = 0;
    // iter and rejects carry on (zero from the host's set-up, or the counts of a
    // reduced-precision phase that a refinement continues)
    st->done = (st->iter >= st->max_iters) ||
               (st->f_star > 0.0 && f - st->f_star <= st->rel_tol * st->f_star) ? 1 : 0;
    return;
  }
  const double t = st->t;
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
  double tt;
  st->f_new = f;
  if (f <= st->f_cur) {
    const int c = st->ix_cur, nw = st->ix_new;
    st->ix_prev = c;
    st->ix_cur = nw;
    st->ix_new = 3 - c - nw;
    st->f_cur = f;
    st->sel_acc = 1;
    tt = reset ? 1.0 : tn;
  } else {
    st->ix_prev = st->ix_cur;
    st->sel_acc = 0;
    st->rejects = st->rejects + 1;
    tt = 1.0;
  }
  st->t = tt;
  st->beta = (tt - 1.0) / (0.5 * (1.0 + sqrt(1.0 + 4.0 * tt * tt)));
  const long long k = st->iter;
  const long long hs = st->hist_stride > 1 ? st->hist_stride : 1;
  if (history && k % hs == 0) history[k / hs] = st->f_cur;
  st->iter = k + 1;
  if (k + 1 >= st->max_iters) st->done = 1;
  if (st->f_star > 0.0 && st->f_cur - st->f_star <= st->rel_tol * st->f_star) st->done = 1;
}

}  // namespace pdt
