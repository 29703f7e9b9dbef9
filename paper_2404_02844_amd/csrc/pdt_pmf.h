// Poisson photon-number distribution of a coherent probe, on the device.
//
// F[d][m] = mu_d^m exp(-mu_d) / m!  (Eq. Fmatrix).  Anchors are evaluated in FP64
// with Loader's saddle-point form (C. Loader 2000, "Fast and accurate computation of
// binomial probabilities"):  log p = -delta(m) - bd0(m, mu) - log(2 pi m) / 2, where
// delta(m) = log m! - [(m + 1/2) log m - m + log(2 pi) / 2] is Stirling's remainder and
// bd0(x, l) = x log(x / l) + l - x is the deviance term, summed as a series when x is
// close to l so the two large terms never cancel.  Between anchors the kernels step
// p(m + 1) = p(m) * mu / (m + 1).
#pragma once

#include <hip/hip_runtime.h>

namespace pdt {

__device__ __forceinline__ double stirling_remainder(int n) {
  const double x = (double)n;
  if (n < 16) {
    // n! is exact in FP64 below 2^53; one rounding in the log
    double fact = 1.0;
    for (int k = 2; k <= n; ++k) fact *= (double)k;
    return log(fact) - ((x + 0.5) * log(x) - x + 0.91893853320467274178);
  }
  // asymptotic series: sum_k B_2k / (2k (2k - 1) x^(2k - 1)), seven terms
  const double u = 1.0 / x;
  const double u2 = u * u;
  double s = 1.0 / 156.0;
  s = 691.0 / 360360.0 - u2 * s;
  s = 1.0 / 1188.0 - u2 * s;
  s = 1.0 / 1680.0 - u2 * s;
  s = 1.0 / 1260.0 - u2 * s;
  s = 1.0 / 360.0 - u2 * s;
  s = 1.0 / 12.0 - u2 * s;
  return u * s;
}

__device__ __forceinline__ double deviance(double x, double l) {
  const double diff = x - l;
  const double tot = x + l;
  if (fabs(diff) < 0.1 * tot) {
    // x log(x/l) + l - x = diff * v + 2 x (v^3/3 + v^5/5 + ...),  v = diff / tot
    const double v = diff / tot;
    const double v2 = v * v;
    double sum = diff * v;
    double pw = 2.0 * x * v;
#pragma unroll 1
    for (int k = 3; k < 200; k += 2) {
      pw *= v2;
      const double next = sum + pw / (double)k;
      if (next == sum) break;
      sum = next;
    }
    return sum;
  }
  return x * log(x / l) + l - x;
}

__device__ __forceinline__ double poisson_logpmf(int m, double mu) {
  if (mu == 0.0) return m == 0 ? 0.0 : -INFINITY;
  if (m == 0) return -mu;
  const double x = (double)m;
  return -stirling_remainder(m) - deviance(x, mu) - 0.5 * log(6.283185307179586477 * x);
}

__device__ __forceinline__ double poisson_pmf(int m, double mu) {
  return exp(poisson_logpmf(m, mu));
}

// P(X >= k0) for X ~ Poisson(mu): compensated sum of the smaller side, terms by the
// ratio recursion with a fresh anchor every 256 terms.
__device__ inline double poisson_upper_tail(double mu, int k0) {
  if (k0 <= 0) return 1.0;
  if (mu == 0.0) return 0.0;
  const double sd = sqrt(mu);
  if ((double)k0 > mu + 40.0 * sd + 100.0) return 0.0;
  if ((double)k0 < mu - 45.0 * sd - 200.0) return 1.0;
  double sum = 0.0, comp = 0.0;
  if ((double)k0 >= mu) {
    int m = k0;
    double p = poisson_pmf(m, mu);
#pragma unroll 1
    for (int it = 0; it < 4000000; ++it) {
      const double t = sum + p;
      comp += (fabs(sum) >= fabs(p)) ? (sum - t) + p : (p - t) + sum;
      sum = t;
      if (p <= 1e-22 * sum) break;  // also ends a sum whose first term underflowed
      ++m;
      p = ((m & 255) == 0) ? poisson_pmf(m, mu) : p * (mu / (double)m);
    }
    return sum + comp;
  }
  int m = k0 - 1;
  double p = poisson_pmf(m, mu);
#pragma unroll 1
  for (int it = 0; it < 4000000 && m >= 0; ++it) {
    const double t = sum + p;
    comp += (fabs(sum) >= fabs(p)) ? (sum - t) + p : (p - t) + sum;
    sum = t;
    if (p <= 1e-22 * sum) break;  // also ends a sum whose first term underflowed
    const double ratio = (double)m / mu;
    --m;
    if (m < 0) break;
    p = ((m & 255) == 0) ? poisson_pmf(m, mu) : p * ratio;
  }
  return 1.0 - (sum + comp);
}

}  // namespace pdt
