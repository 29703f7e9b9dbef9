// Band-GEMM kernels of the projected-gradient detector-tomography solver (gfx950).
//
// The two products of every iteration are banded: F[d][m] is non-negligible only for
// m in [lo_d, hi_d] (Sec. 3.2, Data distribution), and F is never stored -- each
// kernel regenerates its F tile in registers from one FP64 anchor per 16 entries and
// the ratio recursion p(m+1) = p(m) mu / (m+1).
//
//   fx_kernel   O = F X over a 16-probe tile (MFMA 16x16x4, A = F tile, B = X rows),
//               epilogue: ||O - P||^2 partial, residuals for the next step, and the
//               nearest-neighbour regulariser (Eq. regul) over a slice of rows.
//   ftr_kernel  G = 2 F^T R + 2 gamma L Y over a 16-row tile of Pi (MFMA, A = F^T tile
//               staged through LDS, B = R rows); epilogue: gradient step, row-wise
//               Euclidean projection onto the simplex (Eq. Mp1_proj), write X_{k+1}.
//   decide      fixed-order FP64 reduction of the per-wave partials, accept/reject and
//               the momentum scalars.
//
// MFMA lane layout (v_mfma_{f64,f32}_16x16x4, measured on gfx950): lane l holds
// A[l%16][l/16] and B[l/16][l%16]; the result register r of lane l is C[row][l%16] with
// row = 4*(l/16) + r for FP32 but row = l/16 + 4*r for FP64.  The contraction index
// k = l/16 is mapped to whichever photon number / probe keeps the lane's F values
// consecutive.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <type_traits>

#include "pdt_internal.h"
#include "pdt_pmf.h"

namespace pdt {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc;
template <>
struct Acc<double> {
  typedef f64x4 type;
  __device__ static __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // tile row held in result register r of a lane in group kq = lane / 16
  __device__ static __forceinline__ int row(int kq, int r) { return kq + 4 * r; }
};
template <>
struct Acc<float> {
  typedef f32x4 type;
  __device__ static __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
};

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

// ---------------------------------------------------------------------------------------
// Forward band product O = F X, residuals and objective partials.
//
// One workgroup of KS waves per 16-probe tile; the waves split the tile's photon-number
// range in 64-wide chunks (wave w takes chunks w, w + KS, ...), each prefetching the X
// rows of the next PF contraction steps into a register ring.  Partial tiles are summed
// in LDS in a fixed order, then each wave finishes 4 of the 16 probe rows.  Every
// workgroup also sums the regulariser over a slice of rows.
// ---------------------------------------------------------------------------------------
constexpr int KS = 4;   // waves per workgroup splitting the contraction
constexpr int PF = 4;   // prefetch depth in contraction steps

// sum the KS partial 16 x (16 NT) tiles of a workgroup into S (LDS, row stride ld)
template <typename T, int NT, typename AccT>
__device__ __forceinline__ void reduce_tiles(const AccT (&acc)[NT], double* S, int ld, int wv, int i, int kq) {
  for (int w = 0; w < KS; ++w) {
    if (wv == w) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double* p = S + Acc<T>::row(kq, r) * ld + nt * 16 + i;
          *p = (w == 0) ? (double)acc[nt][r] : *p + (double)acc[nt][r];
        }
    }
    __syncthreads();
  }
}

// TS: storage type of X, O, R, P.  TC: MFMA operand type (TS, or float under TS = double
// for the mixed path, whose forward product works on X_new - X_cur: FX_DELTA).
template <typename TS, typename TC, int NT>
__device__ __forceinline__ void fx_body(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, int tile,
                                        int ntiles) {
  if ((mode == FX_ITER || mode == FX_DELTA) && st->done) return;
  typedef TS T;
  typedef typename Acc<TC>::type AccT;
  const bool iter = mode == FX_ITER || mode == FX_DELTA;
  constexpr int LDT = 16 * NT + 1;
  __shared__ double S[16 * LDT];
  __shared__ double red[KS];
  const int tid = threadIdx.x;
  const int wv = tid >> 6;
  const int lane = tid & 63;
  const int i = lane & 15;
  const int kq = lane >> 4;
  const int M = pv.M, D = pv.D, N = pv.N, Npad = pv.Npad;

  const int ix_cur = st->ix_cur;
  const int ix_x = iter ? st->ix_new : ix_cur;
  const T* __restrict__ X = b.X[ix_x];
  T* __restrict__ O = b.O[ix_x];
  const T* __restrict__ Ocur = b.O[ix_cur];
  // the mixed instantiation (float products on double storage) always forms the delta
  constexpr bool delta = !std::is_same<TS, TC>::value;

  const int d0 = tile << 4;
  const int d = d0 + i;
  const bool dval = d < D;
  const double mu = dval ? pv.mu[d] : 0.0;
  const int blo = dval ? pv.lo[d] : 1;
  const int bhi = dval ? pv.hi[d] : 0;
  const double tl = (dval && pv.lump) ? pv.tail[d] : 0.0;
  const int lumpm = pv.lump ? M - 1 : -1;
  const int mlo = pv.dt_mlo[tile];
  const int mhi = pv.dt_mhi[tile];

  AccT acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = AccT{0, 0, 0, 0};

  // Contraction step s of a 64-photon-number chunk at mb gives k-slot kq the photon
  // number mb + 4 s + kq, so each lane walks its probe's row of F with stride 4 across
  // the wave's whole (contiguous) share of the tile: F[d][m + 4] = F[d][m] mu^4 r4[m],
  // r4[m] = 1 / ((m+1)(m+2)(m+3)(m+4)).  A lane takes a fresh anchor where its band
  // starts and every 16 chunks.  X rows beyond M-1 are clamped: F is zero there.
  auto load_step = [&](int mrow, TC (&dst)[NT], double& r) {
    const int m = mrow < M - 1 ? mrow : M - 1;
    const unsigned base = (unsigned)m * (unsigned)Npad + (unsigned)i;
    if constexpr (delta) {
      // the candidate step, written in FP32 by the transposed product's epilogue
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) dst[nt] = (TC)b.dX[base + 16u * nt];
    } else {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) dst[nt] = (TC)X[base + 16u * nt];
    }
    r = pv.r4[mrow];
  };
  const int nch = mhi >= mlo ? (mhi - mlo) / kChunkM + 1 : 0;
  const int c0 = (nch * wv) / KS;
  const int c1 = (nch * (wv + 1)) / KS;
  const double mu4 = (mu * mu) * (mu * mu);
  TC xb[PF][NT];
  double rb[PF];
  if (c0 < c1) {
#pragma unroll
    for (int q = 0; q < PF; ++q) load_step(mlo + kChunkM * c0 + 4 * q + kq, xb[q], rb[q]);
  }
  double p = 0.0;
  for (int c = c0; c < c1; ++c) {
    const int mb = mlo + kChunkM * c;
    const bool more = c + 1 < c1;
    const int ma = mb + kq;
    if ((p == 0.0 || ((c - c0) & 15) == 0) && ma <= bhi && ma + 60 >= blo) p = poisson_pmf(ma, mu);
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int m = ma + 4 * st;
      double f = (m >= blo && m <= bhi) ? p : 0.0;
      f = (m == lumpm && m >= blo && m <= bhi) ? tl : f;
      p *= mu4 * rb[st % PF];
      const TC a = (TC)f;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[nt] = Acc<TC>::mfma(a, xb[st % PF][nt], acc[nt]);
      if (st + PF < 16) load_step(m + 4 * PF, xb[st % PF], rb[st % PF]);
      else if (more) load_step(m + 4 * PF, xb[st % PF], rb[st % PF]);
    }
  }
  reduce_tiles<TC, NT>(acc, S, LDT, wv, i, kq);

  // epilogue: wave wv finishes probe rows 4 wv + kq
  T beta_acc = 0;
  if (iter) {
    const double t = st->t;
    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    const double tnn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tn * tn));
    beta_acc = (T)((tn - 1.0) / tnn);
  }
  double part = 0.0;
  const int dd = d0 + 4 * wv + kq;
  if (dd < D) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + i;
      const size_t off = (size_t)dd * Npad + n;
      const T oc_ = iter ? Ocur[off] : (T)0;
      const T o = delta ? oc_ + (T)S[(4 * wv + kq) * LDT + n] : (T)S[(4 * wv + kq) * LDT + n];
      const T pv_ = b.P[off];
      O[off] = o;
      if (n < N) {
        const double e = (double)o - (double)pv_;
        part += e * e;
      }
      if (iter) {
        const T oc = oc_;
        b.R_acc[off] = o + beta_acc * (o - oc) - pv_;
        b.R_rej[off] = oc - pv_;
      } else {
        b.R_rej[off] = o - pv_;
      }
    }
  }

  // regulariser over this workgroup's slice of row pairs
  if (pv.gamma != 0.0 && M > 1) {
    double reg = 0.0;
    const long long pairs = (long long)(M - 1);
    const long long W = ntiles;
    const long long per = (pairs + W - 1) / W;
    const long long r0 = (long long)tile * per;
    const long long r1 = r0 + per < pairs ? r0 + per : pairs;
    const long long cnt = (r1 > r0 ? r1 - r0 : 0) * (long long)N;
    for (long long q = tid; q < cnt; q += 64 * KS) {
      const long long m = r0 + q / N;
      const int n = (int)(q % N);
      const double e = (double)X[m * Npad + n] - (double)X[(m + 1) * Npad + n];
      reg += e * e;
    }
    part += pv.gamma * reg;
  }
  part = group_sum<64>(part);
  if (lane == 0) red[wv] = part;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < KS; ++w) s += red[w];
    b.partials[tile] = s;
  }
}

// ---------------------------------------------------------------------------------------
// Transposed band product, regulariser gradient and the projected step.
//
// One workgroup of KS waves per 16-row tile of Pi; the waves split the tile's probe
// range in 64-probe chunks.  Per chunk a wave generates F[d][m0..m0+15] for its 64
// probes (lane = probe, recursion along m) into its own LDS slice and reads it back
// transposed as the MFMA A operand; the R rows of the next PF steps are prefetched.
// ---------------------------------------------------------------------------------------
template <typename TS, typename TC, int NT>
__device__ __forceinline__ void ftr_body(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode,
                                         double step, int mt) {
  if (mode == FTR_STEP && st->done) return;
  typedef TS T;
  typedef typename Acc<TC>::type AccT;
  constexpr int LDT = 16 * NT + 1;
  __shared__ double Ft[KS][kChunkD][17];
  __shared__ double S[16 * LDT];
  __shared__ double red[KS];

  const int tid = threadIdx.x;
  const int wv = tid >> 6;
  const int lane = tid & 63;
  const int i = lane & 15;
  const int kq = lane >> 4;
  const int m0 = mt << 4;
  const int M = pv.M, N = pv.N, Npad = pv.Npad;
  const int lumpm = pv.lump ? M - 1 : -1;
  const int dlo = pv.mt_dlo[mt];
  const int dhi = pv.mt_dhi[mt];
  const T* __restrict__ R = (mode == FTR_STEP && st->sel_acc) ? b.R_acc : b.R_rej;

  AccT acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = AccT{0, 0, 0, 0};

  // probes beyond dhi are clamped: their generated F entries are zero
  auto load_r = [&](int drow, TC (&dst)[NT]) {
    const int dd = drow < dhi ? drow : dhi;
    const unsigned base = (unsigned)(dd > 0 ? dd : 0) * (unsigned)Npad + (unsigned)i;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) dst[nt] = (TC)R[base + 16u * nt];
  };
  const int nchunks = dhi >= dlo ? (dhi - dlo) / kChunkD + 1 : 0;
  const int rounds = (nchunks + KS - 1) / KS;
  constexpr int stride = kChunkD * KS;
  // the tile's 16 photon numbers are shared by every probe: 1/(m+1) once per workgroup
  double inv[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) inv[j] = pv.rinv[m0 + j + 1];

  // generator state of one probe (lane) for a chunk: F[d][m0 + j], j = 0..15.  The
  // probe parameters are loaded one round before the anchor is formed from them.
  struct Gen {
    double mu, tl, p;
    int blo, bhi;
  };
  const double* __restrict__ anc = pv.anchors + pv.mt_aoff[mt];
  auto gen_params = [&](int dcc) {
    Gen g{0.0, 0.0, 0.0, 1, 0};
    const int d = dcc + lane;
    if (d <= dhi) {
      g.mu = pv.mu[d];
      g.blo = pv.lo[d];
      g.bhi = pv.hi[d];
      g.tl = pv.lump ? pv.tail[d] : 0.0;
      g.p = anc[d - dlo];  // F[d][m0] from the setup table (0 where the band misses the tile)
    }
    return g;
  };
  auto gen_anchor = [&](Gen&) {};
  auto gen_step = [&](Gen& g, int j) -> double {
    const int m = m0 + j;
    double f = (m >= g.blo && m <= g.bhi) ? g.p : 0.0;
    f = (m == lumpm && m >= g.blo && m <= g.bhi) ? g.tl : f;
    g.p *= g.mu * inv[j];
    return f;
  };

  int dc = dlo + kChunkD * wv;
  TC rb[PF][NT];
#pragma unroll
  for (int p = 0; p < PF; ++p) load_r(dc + 16 * kq + p, rb[p]);
  double vals[16];
  Gen gn;  // parameters of the chunk after the one being generated
  if (rounds > 0) {
    Gen g = gen_params(dc);
    gen_anchor(g);
#pragma unroll
    for (int j = 0; j < 16; ++j) vals[j] = gen_step(g, j);
    gn = gen_params(dc + stride);
  }
  for (int rd = 0; rd < rounds; ++rd, dc += stride) {
    const int dcn = dc + stride;
#pragma unroll
    for (int j = 0; j < 16; ++j) Ft[wv][lane][j] = vals[j];
    __syncthreads();
    // the next chunk's F values are generated between this chunk's MFMAs
    Gen g = gn;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const TC a = (TC)Ft[wv][16 * kq + s][i];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[nt] = Acc<TC>::mfma(a, rb[s % PF][nt], acc[nt]);
      if (s + PF < 16) load_r(dc + 16 * kq + s + PF, rb[s % PF]);
      else load_r(dcn + 16 * kq + s + PF - 16, rb[s % PF]);
      if (s == 1) gen_anchor(g);
      if (s == 2) gn = gen_params(dcn + stride);
      if (s >= 2) vals[s - 2] = gen_step(g, s - 2);
    }
    vals[14] = gen_step(g, 14);
    vals[15] = gen_step(g, 15);
    __syncthreads();
  }
  reduce_tiles<TC, NT>(acc, S, LDT, wv, i, kq);

  // epilogue: wave wv finishes rows m0 + 4 wv + kq (one row per 16-lane group)
  const int m = m0 + 4 * wv + kq;
  const bool mval = m < M;
  const T g2 = (T)(2.0 * pv.gamma);
  if (mode == FTR_STEP) {
    const T beta = (T)st->beta;
    const T* __restrict__ Xc = b.X[st->ix_cur];
    const T* __restrict__ Xp = b.X[st->ix_prev];
    T* __restrict__ Xn = b.X[st->ix_new];
    // row-scaled step: this group's row takes step * w_m
    const T stp = (T)((b.wrow && mval) ? step * b.wrow[m] : step);
    // the mixed instantiation also hands the forward product the step X_new - X_cur in FP32
    constexpr bool delta = !std::is_same<TS, TC>::value;
    T z[1][NT];
    T xcs[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + i;
      T zz = (n < N) ? (T)0 : neg_huge<T>();
      xcs[nt] = 0;
      if (mval && n < N) {
        const size_t off = (size_t)m * Npad + n;
        const T xc = Xc[off];
        xcs[nt] = xc;
        const T y = xc + beta * (xc - Xp[off]);
        T ly = 0;
        if (m > 0) {
          const T xm = Xc[off - Npad];
          ly += y - (xm + beta * (xm - Xp[off - Npad]));
        }
        if (m < M - 1) {
          const T xq = Xc[off + Npad];
          ly += y - (xq + beta * (xq - Xp[off + Npad]));
        }
        const T g = (T)2 * (T)S[(4 * wv + kq) * LDT + n] + g2 * ly;
        zz = y - stp * g;
      }
      z[0][nt] = zz;
    }
    T tau[1];
    simplex_threshold<T, 16, NT, 1, 8>(z, tau);
    if (mval) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int n = nt * 16 + i;
        const T xn = (n < N) ? fmax(z[0][nt] - tau[0], (T)0) : (T)0;
        Xn[(size_t)m * Npad + n] = xn;
        if constexpr (delta) b.dX[(size_t)m * Npad + n] = (float)(xn - xcs[nt]);
      }
    }
  } else {
    // gradient at X_cur (R_rej = F X_cur - P) and the KKT residual partial
    const T* __restrict__ Xc = b.X[st->ix_cur];
    double part = 0.0;
    T g[NT], x[NT];
    T gmin = FLT_MAX;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + i;
      g[nt] = 0;
      x[nt] = 0;
      if (mval && n < N) {
        const size_t off = (size_t)m * Npad + n;
        const T xc = Xc[off];
        T lx = 0;
        if (m > 0) lx += xc - Xc[off - Npad];
        if (m < M - 1) lx += xc - Xc[off + Npad];
        g[nt] = (T)2 * (T)S[(4 * wv + kq) * LDT + n] + g2 * lx;
        x[nt] = xc;
        gmin = fmin(gmin, g[nt]);
      }
      if (mval) b.G[(size_t)m * Npad + n] = g[nt];
    }
    gmin = group_min<16>(gmin);
    if (mval) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int n = nt * 16 + i;
        if (n < N) {
          const double e = (double)x[nt] * ((double)g[nt] - (double)gmin);
          part += e * e;
        }
      }
    }
    part = group_sum<64>(part);
    if (lane == 0) red[wv] = part;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < KS; ++w) s += red[w];
      b.partials[mt] = s;
    }
  }
}


template <typename TS, typename TC, int NT>
__global__ __launch_bounds__(64 * KS) void fx_kernel(ProbView pv, Bufs<TS> b, SolverState* st, int mode) {
  fx_body<TS, TC, NT>(pv, b, st, mode, blockIdx.x, gridDim.x);
}

template <typename TS, typename TC, int NT>
__global__ __launch_bounds__(64 * KS) void ftr_kernel(ProbView pv, Bufs<TS> b, SolverState* st, int mode,
                                                       double step) {
  ftr_body<TS, TC, NT>(pv, b, st, mode, step, blockIdx.x);
}

// Batched launches: one workgroup per (instance, tile) item of a work list; every
// instance carries its own problem view, buffers, state and step.
template <typename TS, typename TC, int NT>
__global__ __launch_bounds__(64 * KS) void fx_batch_kernel(const BatchInst<TS>* insts, const int2* items, int mode) {
  const int2 it = items[blockIdx.x];
  const BatchInst<TS>& I = insts[it.x];
  fx_body<TS, TC, NT>(I.pv, I.b, I.st, mode, it.y, I.n_dt);
}

template <typename TS, typename TC, int NT>
__global__ __launch_bounds__(64 * KS) void ftr_batch_kernel(const BatchInst<TS>* insts, const int2* items,
                                                             int mode) {
  const int2 it = items[blockIdx.x];
  const BatchInst<TS>& I = insts[it.x];
  ftr_body<TS, TC, NT>(I.pv, I.b, I.st, mode, I.step, it.y);
}

// ---------------------------------------------------------------------------------------
// Fixed-order reduction of the partials and the accept/reject decision.
// ---------------------------------------------------------------------------------------
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

__device__ __forceinline__ void decide_body(const double* partials, int n, SolverState* st, double* history,
                                            int mode) {
  __shared__ double sh[256];
  if (mode == DEC_ITER && st->done) return;
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += partials[k];
  const double f = block_sum256(s, sh);
  if (threadIdx.x != 0) return;
  if (mode == DEC_EVAL) {
    st->f_eval = f;
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
    st->iter = 0;
    st->rejects = 0;
    st->done = (st->max_iters <= 0) ||
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
    tt = tn;
  } else {
    st->ix_prev = st->ix_cur;
    st->sel_acc = 0;
    st->rejects = st->rejects + 1;
    tt = 1.0;
  }
  st->t = tt;
  st->beta = (tt - 1.0) / (0.5 * (1.0 + sqrt(1.0 + 4.0 * tt * tt)));
  const long long k = st->iter;
  if (history) history[k] = st->f_cur;
  st->iter = k + 1;
  if (k + 1 >= st->max_iters) st->done = 1;
  if (st->f_star > 0.0 && st->f_cur - st->f_star <= st->rel_tol * st->f_star) st->done = 1;
}

__global__ __launch_bounds__(256) void decide_kernel(const double* partials, int n, SolverState* st,
                                                     double* history, int mode) {
  decide_body(partials, n, st, history, mode);
}

template <typename TS>
__global__ __launch_bounds__(256) void decide_batch_kernel(const BatchInst<TS>* insts, int mode) {
  const BatchInst<TS>& I = insts[blockIdx.x];
  decide_body(I.b.partials, I.n_dt, I.st, I.b.history, mode);
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
// lambda = sqrt(sum_m w_m G_m^2), V_m = w_m G_m / lambda (w = null: all ones)
__global__ __launch_bounds__(256) void power_normalize_kernel(const double* G, double* V, int M, int ld,
                                                              const double* w, double* lam_out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int m = threadIdx.x; m < M; m += 256) {
    const double g = G[(size_t)m * ld];
    s += (w ? w[m] : 1.0) * g * g;
  }
  const double lam = sqrt(block_sum256(s, sh));
  const double inv = lam > 0.0 ? 1.0 / lam : 0.0;
  for (int m = threadIdx.x; m < M; m += 256) V[(size_t)m * ld] = (w ? w[m] : 1.0) * G[(size_t)m * ld] * inv;
  if (threadIdx.x == 0) *lam_out = lam;
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
int fx_num_waves(const ProbView& pv) { return (pv.D + 15) / 16; }
int ftr_num_waves(const ProbView& pv) { return (pv.M + 15) / 16; }

template <typename TS, typename TC, int NT>
static void fx_go(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, hipStream_t s) {
  hipLaunchKernelGGL((fx_kernel<TS, TC, NT>), dim3(fx_num_waves(pv)), dim3(64 * KS), 0, s, pv, b, st, mode);
}
template <typename TS, typename TC, int NT>
static void ftr_go(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, double step,
                   hipStream_t s) {
  hipLaunchKernelGGL((ftr_kernel<TS, TC, NT>), dim3(ftr_num_waves(pv)), dim3(64 * KS), 0, s, pv, b, st, mode,
                     step);
}

#define PDT_NT_SWITCH(NTV, CALL)                 \
  switch (NTV) {                                 \
    case 1: CALL(1); break;                      \
    case 2: CALL(2); break;                      \
    case 3: CALL(3); break;                      \
    case 4: CALL(4); break;                      \
    case 5: CALL(5); break;                      \
    case 6: CALL(6); break;                      \
    case 7: CALL(7); break;                      \
    case 8: CALL(8); break;                      \
    case 9: CALL(9); break;                      \
    case 10: CALL(10); break;                    \
    case 11: CALL(11); break;                    \
    case 12: CALL(12); break;                    \
    default: return hipErrorInvalidValue;        \
  }

template <typename TS, typename TC>
hipError_t launch_fx(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, hipStream_t s) {
#define PDT_FX(K) fx_go<TS, TC, K>(pv, b, st, mode, s)
  PDT_NT_SWITCH(pv.Npad / 16, PDT_FX)
#undef PDT_FX
  return hipGetLastError();
}

template <typename TS, typename TC>
hipError_t launch_ftr(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, double step,
                      hipStream_t s) {
#define PDT_FTR(K) ftr_go<TS, TC, K>(pv, b, st, mode, step, s)
  PDT_NT_SWITCH(pv.Npad / 16, PDT_FTR)
#undef PDT_FTR
  return hipGetLastError();
}

template <typename TS, typename TC, int NT>
static void fxb_go(const BatchInst<TS>* insts, const int2* items, int n_items, int mode, hipStream_t s) {
  hipLaunchKernelGGL((fx_batch_kernel<TS, TC, NT>), dim3(n_items), dim3(64 * KS), 0, s, insts, items, mode);
}
template <typename TS, typename TC, int NT>
static void ftrb_go(const BatchInst<TS>* insts, const int2* items, int n_items, int mode, hipStream_t s) {
  hipLaunchKernelGGL((ftr_batch_kernel<TS, TC, NT>), dim3(n_items), dim3(64 * KS), 0, s, insts, items, mode);
}

template <typename TS, typename TC>
hipError_t launch_fx_batch(int nt, const BatchInst<TS>* insts, const int2* items, int n_items, int mode,
                           hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
#define PDT_FXB(K) fxb_go<TS, TC, K>(insts, items, n_items, mode, s)
  PDT_NT_SWITCH(nt, PDT_FXB)
#undef PDT_FXB
  return hipGetLastError();
}

template <typename TS, typename TC>
hipError_t launch_ftr_batch(int nt, const BatchInst<TS>* insts, const int2* items, int n_items, int mode,
                            hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
#define PDT_FTRB(K) ftrb_go<TS, TC, K>(insts, items, n_items, mode, s)
  PDT_NT_SWITCH(nt, PDT_FTRB)
#undef PDT_FTRB
  return hipGetLastError();
}

template <typename TS>
hipError_t launch_decide_batch(const BatchInst<TS>* insts, int n_inst, int mode, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL((decide_batch_kernel<TS>), dim3(n_inst), dim3(256), 0, s, insts, mode);
  return hipGetLastError();
}

template hipError_t launch_fx_batch<double, double>(int, const BatchInst<double>*, const int2*, int, int, hipStream_t);
template hipError_t launch_fx_batch<float, float>(int, const BatchInst<float>*, const int2*, int, int, hipStream_t);
template hipError_t launch_fx_batch<double, float>(int, const BatchInst<double>*, const int2*, int, int, hipStream_t);
template hipError_t launch_ftr_batch<double, double>(int, const BatchInst<double>*, const int2*, int, int, hipStream_t);
template hipError_t launch_ftr_batch<float, float>(int, const BatchInst<float>*, const int2*, int, int, hipStream_t);
template hipError_t launch_ftr_batch<double, float>(int, const BatchInst<double>*, const int2*, int, int, hipStream_t);
template hipError_t launch_decide_batch<double>(const BatchInst<double>*, int, int, hipStream_t);
template hipError_t launch_decide_batch<float>(const BatchInst<float>*, int, int, hipStream_t);

hipError_t launch_decide(const double* partials, int n, SolverState* st, double* history, int mode,
                         hipStream_t s) {
  hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(256), 0, s, partials, n, st, history, mode);
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

hipError_t launch_power_normalize(double* G, double* V, int M, int ld, const double* w, double* lam_out,
                                  hipStream_t s) {
  hipLaunchKernelGGL(power_normalize_kernel, dim3(1), dim3(256), 0, s, G, V, M, ld, w, lam_out);
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
template hipError_t launch_fill_rows<double>(double*, long long, int, int, double, hipStream_t);
template hipError_t launch_fill_rows<float>(float*, long long, int, int, float, hipStream_t);

template hipError_t launch_fx<double, double>(const ProbView&, const Bufs<double>&, SolverState*, int,
                                              hipStream_t);
template hipError_t launch_fx<float, float>(const ProbView&, const Bufs<float>&, SolverState*, int, hipStream_t);
template hipError_t launch_fx<double, float>(const ProbView&, const Bufs<double>&, SolverState*, int, hipStream_t);
template hipError_t launch_ftr<double, double>(const ProbView&, const Bufs<double>&, SolverState*, int, double,
                                               hipStream_t);
template hipError_t launch_ftr<float, float>(const ProbView&, const Bufs<float>&, SolverState*, int, double,
                                             hipStream_t);
template hipError_t launch_ftr<double, float>(const ProbView&, const Bufs<double>&, SolverState*, int, double,
                                              hipStream_t);
template hipError_t launch_project_rows<double>(const double*, double*, long long, int, int, int, hipStream_t);
template hipError_t launch_project_rows<float>(const float*, float*, long long, int, int, int, hipStream_t);
template hipError_t launch_convert_pad<double, double>(const double*, double*, long long, int, int, int,
                                                       hipStream_t);
template hipError_t launch_convert_pad<double, float>(const double*, float*, long long, int, int, int,
                                                      hipStream_t);
template hipError_t launch_convert_pad<float, double>(const float*, double*, long long, int, int, int,
                                                      hipStream_t);

}  // namespace pdt
