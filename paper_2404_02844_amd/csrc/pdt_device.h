// Device helpers shared by the band kernels and the standalone kernels: reductions over
// groups of lanes and the row-wise simplex threshold.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>

namespace pdt {

template <typename T>
__device__ __forceinline__ T neg_huge();
template <>
__device__ __forceinline__ double neg_huge<double>() { return -DBL_MAX; }
template <>
__device__ __forceinline__ float neg_huge<float>() { return -FLT_MAX; }

// ---- reductions inside groups of G consecutive lanes (G = 16 or 64) -------------------
template <int G, typename V>
__device__ __forceinline__ V group_sum(V v) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}
template <int G, typename V>
__device__ __forceinline__ V group_max(V v) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, G));
  return v;
}
template <int G, typename V>
__device__ __forceinline__ V group_min(V v) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, G));
  return v;
}
template <int G>
__device__ __forceinline__ int group_isum(int v) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// ---- simplex projection of rows spread over G lanes x V values, R rows per lane -------
//
// tau* solves sum_i max(z_i - tau, 0) = 1 and lies in [max z - 1, max z].  A few
// wavefront-level bisection steps on tau narrow that bracket; then, from the bracket's lower end (a lower
// bound of tau*), the support-restricted threshold tau <- (sum_{z > tau} z - 1) /
// #{z > tau} increases monotonically to tau* and stops exactly when the support no
// longer changes (Michelot 1986).  Entries equal to neg_huge<T>() are padding.
template <typename T, int G, int V, int R, int BISECT>
__device__ __forceinline__ void simplex_threshold(const T (&z)[R][V], T (&tau)[R]) {
  T lo[R], hi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T mx = z[r][0];
#pragma unroll
    for (int v = 1; v < V; ++v) mx = fmax(mx, z[r][v]);
    mx = group_max<G>(mx);
    hi[r] = mx;
    lo[r] = mx - (T)1;
  }
  // Bisection on tau in FP32 arithmetic.  lo moves up only when the FP32 sum is above 1
  // by more than its rounding error can account for, so lo <= tau* always holds; the
  // exact phase below needs nothing else from the bracket.
#pragma unroll 1
  for (int it = 0; it < BISECT; ++it) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T mid = lo[r] + (T)0.5 * (hi[r] - lo[r]);
      float s = 0.0f;
#pragma unroll
      for (int v = 0; v < V; ++v) s += (float)fmax(z[r][v] - mid, (T)0);
      s = group_sum<G>(s);
      const bool up = s > 1.0f + 1e-4f;
      lo[r] = up ? mid : lo[r];
      hi[r] = up ? hi[r] : mid;
    }
  }
  int cnt_prev[R];
#pragma unroll
  for (int r = 0; r < R; ++r) cnt_prev[r] = -1;
#pragma unroll 1
  for (int it = 0; it < 4 * G * V + 8; ++it) {
    bool settled = true;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T s = 0;
      int c = 0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const bool in = z[r][v] > lo[r];
        s += in ? z[r][v] : (T)0;
        c += in ? 1 : 0;
      }
      s = group_sum<G>(s);
      c = group_isum<G>(c);
      const T t = (s - (T)1) / (T)c;
      const bool moved = c != cnt_prev[r];
      cnt_prev[r] = c;
      // the new threshold never falls below the bracket's lower end
      lo[r] = moved ? fmax(lo[r], t) : lo[r];
      tau[r] = t;
      settled = settled && !moved;
    }
    if (__all(settled)) break;
  }
}

}  // namespace pdt
