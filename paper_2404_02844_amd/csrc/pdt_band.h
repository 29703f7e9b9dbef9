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
//
// This header holds the templates; pdt_band_{f64,f32,mixed,batch}.hip instantiate them.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <type_traits>

#include "pdt_decide.h"
#include "pdt_device.h"
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

// ---------------------------------------------------------------------------------------
// Forward band product O = F X, residuals and objective partials.
//
// One workgroup of KS waves per 16-probe tile; the waves split the tile's photon-number
// range in 64-wide chunks (wave w takes chunks w, w + KS, ...), each prefetching the X
// rows of the next PF contraction steps into a register ring.  Partial tiles are summed
// in LDS in a fixed order, then each wave finishes 4 of the 16 probe rows.  Every
// workgroup also sums the regulariser over a slice of rows.
// ---------------------------------------------------------------------------------------
// Prefetch depth in contraction steps of the forward (X rows) and transposed (R rows)
// products, per MFMA operand type.
template <typename TC>
struct Prefetch {
  static constexpr int fx = sizeof(TC) == 4 ? 8 : 4;
  static constexpr int ftr = sizeof(TC) == 4 ? 8 : 4;
};
// KS (a template parameter, 4 or 8) waves per workgroup split the contraction; the
// first four waves finish the tile's 16 rows in the epilogues.

// sum the KS partial 16 x (16 NT) tiles of a workgroup into S (LDS, row stride ld)
// Orders one wave's LDS accesses for the compiler (the hardware already completes them in
// issue order within a wave).
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// (the first ntv of the NT column tiles: a partial last pass of the transposed product)
template <typename T, int NT, int KS, typename AccT>
__device__ __forceinline__ void reduce_tiles(const AccT (&acc)[NT], double* S, int ld, int wv, int i, int kq,
                                             int ntv = NT) {
  for (int w = 0; w < KS; ++w) {
    if (wv == w) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        if (nt < ntv)
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
//
// Split contraction (pv.fx_split = S > 1, for problems with few probe tiles and long
// photon-number ranges): workgroup wg takes part wg % S of tile wg / S's chunks, writes
// its partial tile and its regulariser partial, and the last of the S workgroups to
// finish (a per-tile counter) sums the S partial tiles in workgroup order and runs the
// epilogue.  Partials: [wg] regulariser shares, then [nwg + tile] residual sums.
template <typename TS, typename TC, int NT, int KS>
__device__ __forceinline__ void fx_body(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, int wg,
                                        int nwg) {
  if ((mode == FX_ITER || mode == FX_DELTA || mode == FX_EVAL_PREV || mode == FX_RESYNC) && st->done) return;
  if (b.skip && *b.skip) return;
  const int nsplit = pv.fx_split;
  const int tile = wg / nsplit;
  const int sidx = wg - tile * nsplit;
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
  const int ix_x = iter ? st->ix_new : (mode == FX_EVAL_PREV ? st->ix_prev : ix_cur);
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

  // Wide rows (NT >= 8) with FP64 operands run the contraction in two passes over half
  // the column tiles each (accumulators and prefetch ring of one pass within two waves
  // per SIMD); each pass restarts the recursion from its anchors.
  constexpr int NTC = (NT >= 8 && sizeof(TC) == 8) ? (NT + 1) / 2 : NT;
  constexpr int NPASS = (NT + NTC - 1) / NTC;

  // Contraction step s of a 64-photon-number chunk at mb gives k-slot kq the photon
  // number mb + 4 s + kq, so each lane walks its probe's row of F with stride 4 across
  // the wave's whole (contiguous) share of the tile: F[d][m + 4] = F[d][m] mu^4 r4[m],
  // r4[m] = 1 / ((m+1)(m+2)(m+3)(m+4)).  A lane takes a fresh anchor where its band
  // starts and every 16 chunks.  X rows beyond M-1 are clamped: F is zero there.
  auto load_step = [&](int mrow, TC (&dst)[NTC], double& r, int nt0) {
    const int m = mrow < M - 1 ? mrow : M - 1;
    const unsigned base = (unsigned)m * (unsigned)Npad + (unsigned)i;
    if constexpr (delta) {
      // the candidate step, written in FP32 by the transposed product's epilogue
#pragma unroll
      for (int k = 0; k < NTC; ++k)
        if (NPASS == 1 || nt0 + k < NT) dst[k] = (TC)b.dX[base + 16u * (nt0 + k)];
    } else {
#pragma unroll
      for (int k = 0; k < NTC; ++k)
        if (NPASS == 1 || nt0 + k < NT) dst[k] = (TC)X[base + 16u * (nt0 + k)];
    }
    r = pv.r4[mrow];
  };
  const int nch = mhi >= mlo ? (mhi - mlo) / kChunkM + 1 : 0;
  const int cs0 = (nch * sidx) / nsplit, cs1 = (nch * (sidx + 1)) / nsplit;
  const int c0 = cs0 + ((cs1 - cs0) * wv) / KS;
  const int c1 = cs0 + ((cs1 - cs0) * (wv + 1)) / KS;
  const double mu4 = (mu * mu) * (mu * mu);
  // Anchor of the first chunk whose photon numbers come within reach of this lane's band
  // (ma + 60 >= lo_d, ma <= hi_d) and whose value does not underflow (dense rows of bright
  // probes), evaluated before any X row is in flight: inside the loop the evaluation's
  // registers would force the prefetched loads to drain.
  int cb = -1;
  double p_start = 0.0;
  {
    const int need = blo - 60 - kq - mlo;
    int cs = need <= 0 ? 0 : (need + kChunkM - 1) / kChunkM;
    cs = cs > c0 ? cs : c0;
#pragma unroll 1
    for (int c = cs; c < c1 && mlo + kChunkM * c + kq <= bhi; ++c) {
      const double v = poisson_pmf(mlo + kChunkM * c + kq, mu);
      if (v > 0.0) {
        cb = c;
        p_start = v;
        break;
      }
    }
  }
  constexpr int PF = Prefetch<TC>::fx;
  TC xb[PF][NTC];
  double rb[PF];
  if (c0 < c1) {
#pragma unroll
    for (int q = 0; q < PF; ++q) load_step(mlo + kChunkM * c0 + 4 * q + kq, xb[q], rb[q], 0);
  }

  // With the gradient restart, an accepted candidate whose step fails the test resets the
  // momentum: the residual handed to the next step is then F X_new - P (beta 0).  The
  // test is the decision kernel's own sum, in its order.
  const bool reset = (iter && b.rpart) ? restart_test<64 * KS>(b.rpart, (M + 15) / 16) : false;

  // Work of the epilogue that does not depend on the contraction is done here so that its
  // loads overlap the main loop: the regulariser over this workgroup's slice of row
  // pairs, and (when registers allow) O_cur and P of this group's output row.
  // The slice's row pairs (mm, mm + 1) go to the workgroup's 16-lane groups in turn; a
  // lane takes columns i, i + 16, ... of both rows, all loaded before they are used.
  // After a step (b.regpart) the pairs inside each 16-row tile were summed by the step's
  // epilogue, one partial per row tile: this workgroup then takes its slice of the pairs
  // across tile edges, (16 t + 15, 16 t + 16), and its slice of those partials.
  double reg = 0.0;
  const bool edges = iter && b.regpart;
  if (pv.gamma != 0.0 && M > 1) {
    const long long nmt = (M + 15) / 16;
    const long long pairs = edges ? nmt - 1 : (long long)(M - 1);
    const long long W = nwg;
    const long long per = (pairs + W - 1) / W;
    const long long r0 = (long long)wg * per;
    const long long r1 = r0 + per < pairs ? r0 + per : pairs;
    if (edges) {
      const long long pt = (nmt + W - 1) / W;
      const long long q0 = (long long)wg * pt;
      const long long q1 = q0 + pt < nmt ? q0 + pt : nmt;
      for (long long t = q0 + tid; t < q1; t += 64 * KS) reg += b.regpart[t];
    }
#pragma unroll 2
    for (long long q = r0 + (tid >> 4); q < r1; q += 4 * KS) {
      const long long mm = edges ? 16 * q + 15 : q;
      const T* __restrict__ xa = X + (size_t)mm * Npad + i;
      T va[NT], vb[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        va[nt] = xa[16 * nt];
        vb[nt] = xa[Npad + 16 * nt];
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const double e = (double)va[nt] - (double)vb[nt];
        reg += (nt * 16 + i < N) ? e * e : 0.0;
      }
    }
  }
  const int dd = d0 + 4 * wv + kq;  // epilogue row of this 16-lane group
  const bool dval_e = wv < 4 && dd < D;
  constexpr bool kHoist = NT >= 4 && NT <= 5;
  T hoc[NT], hp[NT];
  if constexpr (kHoist) {
    if (dval_e) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const size_t off = (size_t)dd * Npad + nt * 16 + i;
        hoc[nt] = iter ? Ocur[off] : (T)0;
        hp[nt] = b.P[off];
      }
    }
  }
#pragma unroll 1
  for (int pass = 0; pass < NPASS; ++pass) {
    const int nt0 = pass * NTC;
    if (pass > 0 && c0 < c1) {
#pragma unroll
      for (int q = 0; q < PF; ++q) load_step(mlo + kChunkM * c0 + 4 * q + kq, xb[q], rb[q], nt0);
    }
    AccT acc[NTC];
#pragma unroll
    for (int k = 0; k < NTC; ++k) acc[k] = AccT{0, 0, 0, 0};
    double p = 0.0;
    // blocks of 16 chunks; the recursion restarts from an exact anchor at each block after
    // the band-start chunk, which bounds the growth of its rounding error
#pragma unroll 1
    for (int cblk = c0; cblk < c1; cblk += 16) {
      if (cb >= 0 && cblk > cb) {
        const int ma = mlo + kChunkM * cblk + kq;
        if (ma <= bhi && ma + 60 >= blo) p = poisson_pmf(ma, mu);
      }
      const int cend = cblk + 16 < c1 ? cblk + 16 : c1;
      for (int c = cblk; c < cend; ++c) {
        const int mb = mlo + kChunkM * c;
        const bool more = c + 1 < c1;
        const int ma = mb + kq;
        if (c == cb) p = p_start;
#pragma unroll
        for (int st = 0; st < 16; ++st) {
          const int m = ma + 4 * st;
          double f = (m >= blo && m <= bhi) ? p : 0.0;
          f = (m == lumpm && m >= blo && m <= bhi) ? tl : f;
          p *= mu4 * rb[st % PF];
          const TC a = (TC)f;
#pragma unroll
          for (int k = 0; k < NTC; ++k)
            if (NPASS == 1 || nt0 + k < NT) acc[k] = Acc<TC>::mfma(a, xb[st % PF][k], acc[k]);
          if (st + PF < 16) load_step(m + 4 * PF, xb[st % PF], rb[st % PF], nt0);
          else if (more) load_step(m + 4 * PF, xb[st % PF], rb[st % PF], nt0);
        }
      }
    }
    reduce_tiles<TC, NTC, KS>(acc, S + 16 * nt0, LDT, wv, i, kq, NT - nt0);
  }

  if (nsplit > 1) {
    constexpr int kTile = 16 * 16 * NT;
    double* mine = b.fx_part + (size_t)wg * kTile;
    for (int q = tid; q < kTile; q += 64 * KS) mine[q] = S[(q / (16 * NT)) * LDT + q % (16 * NT)];
    double rp = (pv.gamma != 0.0 && M > 1) ? pv.gamma * reg : 0.0;
    rp = group_sum<64>(rp);
    if (lane == 0) red[wv] = rp;
    // Every wave's stores have completed at the barrier; one device-scope release by one
    // thread then publishes the workgroup's partial tile (a device-scope fence writes the
    // XCD's L2 back, so it is issued once per workgroup, not once per thread).
    __syncthreads();
    __shared__ int is_last;
    if (tid == 0) {
      double sr = 0.0;
#pragma unroll
      for (int w = 0; w < KS; ++w) sr += red[w];
      b.partials[wg] = sr;
      __threadfence();
      const unsigned prev = atomicAdd(&b.fx_count[tile], 1u);
      is_last = prev == (unsigned)(nsplit - 1);
      if (is_last) {
        b.fx_count[tile] = 0u;  // ready for the next launch
        __threadfence();        // acquire: the other workgroups' partial tiles
      }
    }
    __syncthreads();
    if (!is_last) return;
    const double* parts = b.fx_part + (size_t)tile * nsplit * kTile;
    for (int q = tid; q < kTile; q += 64 * KS) {
      double v = 0.0;
      for (int sp = 0; sp < nsplit; ++sp) v += __builtin_nontemporal_load(parts + (size_t)sp * kTile + q);
      S[(q / (16 * NT)) * LDT + q % (16 * NT)] = v;
    }
    __syncthreads();
  }

  // epilogue: wave wv finishes probe rows 4 wv + kq
  T beta_acc = 0;
  if (iter && !reset) {
    const double t = st->t;
    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    const double tnn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tn * tn));
    beta_acc = (T)((tn - 1.0) / tnn);
  }
  double part = 0.0;
  if (dval_e) {
    if constexpr (!kHoist) {
      // every column tile's loads are issued before the first store (which the compiler
      // may not move them across)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const size_t off = (size_t)dd * Npad + nt * 16 + i;
        hoc[nt] = iter ? Ocur[off] : (T)0;
        hp[nt] = b.P[off];
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + i;
      const size_t off = (size_t)dd * Npad + n;
      const T oc_ = hoc[nt], pv_ = hp[nt];
      const T o = delta ? oc_ + (T)S[(4 * wv + kq) * LDT + n] : (T)S[(4 * wv + kq) * LDT + n];
      O[off] = o;
      if (n < N) {
        const double e = (double)o - (double)pv_;
        part += e * e;
      }
      if (iter) {
        const T oc = oc_;
        const T ra = o + beta_acc * (o - oc) - pv_, rr = oc - pv_;
        b.R_acc[off] = ra;
        b.R_rej[off] = rr;
        if (b.R32_acc) {
          b.R32_acc[off] = (float)ra;
          b.R32_rej[off] = (float)rr;
        }
      } else if (mode == FX_RESYNC) {
        // the next step's residual if it keeps its momentum (F Y = O + beta (O - O_prev))
        // or restarts, both from exact products
        const T op = b.O[st->ix_prev][off];
        const T ra = o + (T)st->beta * (o - op) - pv_, rr = o - pv_;
        b.R_acc[off] = ra;
        b.R_rej[off] = rr;
        if (b.R32_acc) {
          b.R32_acc[off] = (float)ra;
          b.R32_rej[off] = (float)rr;
        }
      } else if (mode != FX_EVAL_PREV) {
        const T rr = o - pv_;
        b.R_rej[off] = rr;
        if (b.R32_rej) b.R32_rej[off] = (float)rr;
      }
    }
  }

  // the regulariser partial formed before the main loop (split: already written per
  // workgroup)
  if (nsplit == 1 && pv.gamma != 0.0 && M > 1) part += pv.gamma * reg;
  part = group_sum<64>(part);
  if (lane == 0) red[wv] = part;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < KS; ++w) s += red[w];
    b.partials[nsplit == 1 ? tile : nwg + tile] = s;
  }
}

// ---------------------------------------------------------------------------------------
// Transposed band product, regulariser gradient and the projected step.
//
// One workgroup of KS waves per 16-row tile of Pi; the waves split the tile's probe
// range in 64-probe chunks.  Per chunk a wave generates F[d][m0..m0+15] for its 64
// probes (lane = probe, recursion along m) into its own LDS slice and reads it back
// transposed as the MFMA A operand; the R rows of the next PF steps are prefetched.
//
// Split contraction (pv.ftr_split = S > 1, for row tiles whose probe ranges are long
// against the number of tiles): two launches.  In the first (FTR_PART) workgroup wg
// takes the contiguous part wg % S of tile wg / S's chunks and writes its partial tile;
// in the second (FTR_FINISH) workgroup mt sums tile mt's S partial tiles in part order
// and runs the epilogue.  (The kernel boundary publishes the partial tiles; a per-tile
// handshake inside one launch would need a device-scope fence per workgroup, which
// writes the XCD's L2 back each time.)
// ---------------------------------------------------------------------------------------
// NW: every row tile of the problem has a narrow probe range (pv.ftr_narrow_all), so
// the chunked contraction and its LDS staging are compiled out.
template <typename TS, typename TC, int NT, int KS, bool NW = false>
__device__ __forceinline__ void ftr_body(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode,
                                         double step, int wg, int phase = FTR_FUSED) {
  if (mode == FTR_STEP && st->done) return;
  if (b.skip && *b.skip) return;
  const int nsplit = phase == FTR_FUSED ? 1 : pv.ftr_split;
  const int mt = phase == FTR_PART ? wg / nsplit : wg;
  const int sidx = phase == FTR_PART ? wg - mt * nsplit : 0;
  typedef TS T;
  typedef typename Acc<TC>::type AccT;
  constexpr int LDT = 16 * NT + 1;
  // Wide rows (NT >= 8) with FP64 operands are contracted in two passes over half the
  // column tiles each, which keeps the accumulators and the prefetch ring of one pass
  // within the register budget of two waves per SIMD; every pass reduces into its
  // columns of the full tile.  (FP32 operands fit two waves in one pass.)
  constexpr int NTC = (NT >= 8 && sizeof(TC) == 8) ? (NT + 1) / 2 : NT;
  constexpr int NPASS = (NT + NTC - 1) / NTC;
  // the F^T staging tiles of the main loop and the reduction tile share one LDS block
  // (a single pass), or sit side by side (two passes)
  // F^T staging in the MFMA operand type (doubles of LDS per wave: 64 x 17 operands)
  constexpr int kFt = NW ? 0 : (KS * kChunkD * 17 * (int)sizeof(TC) + 7) / 8, kS = 16 * LDT;
  __shared__ double lds[NPASS > 1 ? kFt + kS : (kFt > kS ? kFt : kS)];
  TC(*Ft)[kChunkD][17] = reinterpret_cast<TC(*)[kChunkD][17]>(lds);
  double* S = NPASS > 1 ? lds + kFt : lds;
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
  // FP32 operands on FP64 storage (the mixed path) read the FP32 copies of R the forward
  // product wrote (the same values as converting R at the load, at half the bytes)
  constexpr bool kR32 = !std::is_same<TS, TC>::value;
  const float* __restrict__ R32 = (mode == FTR_STEP && st->sel_acc) ? b.R32_acc : b.R32_rej;

  // probes beyond dhi are clamped: their generated F entries are zero
  auto load_r = [&](int drow, TC (&dst)[NTC], int nt0) {
    const int dd = drow < dhi ? drow : dhi;
    const unsigned base = (unsigned)(dd > 0 ? dd : 0) * (unsigned)Npad + (unsigned)i;
#pragma unroll
    for (int k = 0; k < NTC; ++k)
      if (NPASS == 1 || nt0 + k < NT) {
        if constexpr (kR32) dst[k] = (TC)R32[base + 16u * (nt0 + k)];
        else dst[k] = (TC)R[base + 16u * (nt0 + k)];
      }
  };
  const int nchunks = dhi >= dlo ? (dhi - dlo) / kChunkD + 1 : 0;
  // this workgroup's part of the chunks: [cs0, cs1)
  const int cs0 = (nchunks * sidx) / nsplit, ncs = (nchunks * (sidx + 1)) / nsplit - cs0;
  // wave wv takes chunks cs0 + wv, cs0 + wv + KS, ...: its rounds end with its last
  // nonempty chunk (chunks past dhi would only add exact zeros)
  const int rounds = (phase != FTR_FINISH && wv < ncs) ? (ncs - wv + KS - 1) / KS : 0;
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


  const int m = m0 + 4 * wv + kq;  // epilogue row of this 16-lane group
  const bool mval = wv < 4 && m < M;
  const T beta = (T)st->beta;
  const T* __restrict__ Xc = b.X[st->ix_cur];
  const T* __restrict__ Xp = b.X[st->ix_prev];
  // Y = X + beta (X - X_prev) for the Laplacian along m: each 16-lane group loads its own
  // row of both iterates (the tile's first and last group also the row just outside the
  // tile), all column tiles before any is used.  Rows r - 1 and r + 1 of the same wave
  // are lanes -16 / +16 (shuffles); a wave's first and last rows and the two outside rows
  // pass through LDS (Yb: 2 rows per wave, then rows m0 - 1 and m0 + 16).
  __shared__ double Yb[10 * LDT];
  auto form_y = [&](T (&xc)[NT], T (&y)[NT], T (&ly)[NT]) {
    const int mc = m < M - 1 ? m : M - 1;
    const size_t r0 = (size_t)mc * Npad + i;
    const bool lo_h = wv == 0 && kq == 0 && m0 > 0;
    const bool hi_h = wv == 3 && kq == 3 && m0 + 16 < M;
    const size_t rh = (size_t)(lo_h ? m0 - 1 : (hi_h ? m0 + 16 : mc)) * Npad + i;
    T a[NT], ap[NT], h[NT], hp[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      a[nt] = Xc[r0 + 16 * nt];
      ap[nt] = Xp[r0 + 16 * nt];
    }
    if (lo_h || hi_h) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        h[nt] = Xc[rh + 16 * nt];
        hp[nt] = Xp[rh + 16 * nt];
      }
    }
    T up[NT], dn[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const T yy = a[nt] + beta * (a[nt] - ap[nt]);
      y[nt] = yy;
      up[nt] = __shfl(yy, (lane + 48) & 63);
      dn[nt] = __shfl(yy, (lane + 16) & 63);
      if (wv < 4 && (kq == 0 || kq == 3)) Yb[(2 * wv + (kq == 3)) * LDT + 16 * nt + i] = (double)yy;
      if (lo_h || hi_h) Yb[(lo_h ? 8 : 9) * LDT + 16 * nt + i] = (double)(h[nt] + beta * (h[nt] - hp[nt]));
    }
    __syncthreads();
    const int rup = wv > 0 ? 2 * wv - 1 : 8;  // Yb row of row 4 wv - 1
    const int rdn = wv < 3 ? 2 * wv + 2 : 9;  // Yb row of row 4 wv + 4
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const bool v = mval && nt * 16 + i < N;
      const T yy = y[nt];
      const T ym = kq > 0 ? up[nt] : (wv < 4 ? (T)Yb[rup * LDT + 16 * nt + i] : (T)0);
      const T yq = kq < 3 ? dn[nt] : (wv < 4 ? (T)Yb[rdn * LDT + 16 * nt + i] : (T)0);
      const T lm = m > 0 ? yy - ym : (T)0;
      const T lq = m < M - 1 ? yy - yq : (T)0;
      xc[nt] = v ? a[nt] : (T)0;
      y[nt] = v ? yy : (T)0;
      ly[nt] = v ? lm + lq : (T)0;
    }
  };
  T hx[NT], hy[NT], hly[NT];

  // Narrow probe ranges (at most kNarrowD probes: the thin row tiles of sparse, wide
  // bands, e.g. mu_d = d^2) skip the 64-probe chunks.  Contraction step q takes probes
  // dlo + 4q .. dlo + 4q + 3 (one per 16-lane group) and goes to wave q % KS; each lane
  // forms its own F[d][m0 + i] from the tile's anchor by the same recursion (the same
  // products in the same order as the chunked generator), and the NT products of the
  // step read R rows directly.  The waves' partial tiles are summed as below.
  const bool narrow = phase == FTR_FUSED && (NW || (dhi >= dlo && dhi - dlo < kNarrowD));
  // (in the same column passes as the chunked contraction)
#pragma unroll 1
  for (int pass = 0; pass < (narrow ? NPASS : 0); ++pass) {
    const int nt0 = pass * NTC;
    AccT acc[NTC];
#pragma unroll
    for (int k = 0; k < NTC; ++k) acc[k] = AccT{0, 0, 0, 0};
    const int nks = dhi >= dlo ? (dhi - dlo) / 4 + 1 : 0;
    const int mm = m0 + i;
#pragma unroll 1
    for (int q = wv; q < nks; q += KS) {
      const int d = dlo + 4 * q + kq;
      const int dr = d < dhi ? d : dhi;
      TC rv[NTC];
      const unsigned base = (unsigned)dr * (unsigned)Npad + (unsigned)i + 16u * (unsigned)nt0;
#pragma unroll
      for (int k = 0; k < NTC; ++k)
        if (NPASS == 1 || nt0 + k < NT) {
          if constexpr (kR32) rv[k] = (TC)R32[base + 16u * k];
          else rv[k] = (TC)R[base + 16u * k];
        }
      double f = 0.0;
      if (d <= dhi) {
        const double mu = pv.mu[d];
        const int blo = pv.lo[d], bhi = pv.hi[d];
        double p = anc[d - dlo];
#pragma unroll
        for (int j = 0; j < 15; ++j) p = j < i ? p * (mu * inv[j]) : p;
        const bool in = mm >= blo && mm <= bhi;
        f = in ? p : 0.0;
        if (mm == lumpm && in) f = pv.tail[d];
      }
      const TC a = (TC)f;
#pragma unroll
      for (int k = 0; k < NTC; ++k)
        if (NPASS == 1 || nt0 + k < NT) acc[k] = Acc<TC>::mfma(a, rv[k], acc[k]);
    }
    reduce_tiles<TC, NTC, KS>(acc, S + 16 * nt0, LDT, wv, i, kq, NT - nt0);
  }
#pragma unroll 1
  for (int pass = 0; pass < ((NW || phase == FTR_FINISH || narrow) ? 0 : NPASS); ++pass) {
    const int nt0 = pass * NTC;
    AccT acc[NTC];
#pragma unroll
    for (int k = 0; k < NTC; ++k) acc[k] = AccT{0, 0, 0, 0};
    int dc = dlo + kChunkD * (cs0 + wv);
    constexpr int PF = Prefetch<TC>::ftr;
    TC rb[PF][NTC];
#pragma unroll
    for (int p = 0; p < PF; ++p) load_r(dc + 16 * kq + p, rb[p], nt0);
    double vals[16];
    Gen gn;  // parameters of the chunk after the one being generated
    if (rounds > 0) {
      Gen g = gen_params(dc);
      gen_anchor(g);
#pragma unroll
      for (int j = 0; j < 16; ++j) vals[j] = gen_step(g, j);
      gn = gen_params(dc + stride);
    }
    // Each wave stages only its own Ft[wv] slice, so the waves need no barrier between
    // rounds: a wave's LDS operations complete in issue order, and wave_lds_order() keeps
    // the compiler from moving them across each other.
    for (int rd = 0; rd < rounds; ++rd, dc += stride) {
      const int dcn = dc + stride;
#pragma unroll
      for (int j = 0; j < 16; ++j) Ft[wv][lane][j] = (TC)vals[j];
      wave_lds_order();
      // the chunk's 16 A operands are read back at once, so no step waits on LDS
      TC av[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) av[s] = Ft[wv][16 * kq + s][i];
      // the next chunk's F values are generated between this chunk's MFMAs
      Gen g = gn;
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const TC a = av[s];
#pragma unroll
        for (int k = 0; k < NTC; ++k)
          if (NPASS == 1 || nt0 + k < NT) acc[k] = Acc<TC>::mfma(a, rb[s % PF][k], acc[k]);
        if (s + PF < 16) load_r(dc + 16 * kq + s + PF, rb[s % PF], nt0);
        else load_r(dcn + 16 * kq + s + PF - 16, rb[s % PF], nt0);
        if (s == 1) gen_anchor(g);
        if (s == 2) gn = gen_params(dcn + stride);
        if (s >= 2) vals[s - 2] = gen_step(g, s - 2);
      }
      vals[14] = gen_step(g, 14);
      vals[15] = gen_step(g, 15);
      wave_lds_order();
    }
    __syncthreads();  // a single pass: S shares its LDS with every wave's Ft slice
    reduce_tiles<TC, NTC, KS>(acc, S + 16 * nt0, LDT, wv, i, kq, NT - nt0);
  }

  constexpr int kTile = 16 * 16 * NT;
  if (phase == FTR_PART) {
    double* mine = b.ftr_part + (size_t)wg * kTile;
    for (int q = tid; q < kTile; q += 64 * KS) mine[q] = S[(q / (16 * NT)) * LDT + q % (16 * NT)];
    return;
  }
  if (phase == FTR_FINISH) {
    const double* parts = b.ftr_part + (size_t)mt * nsplit * kTile;
    for (int q = tid; q < kTile; q += 64 * KS) {
      double v = 0.0;
      for (int sp = 0; sp < nsplit; ++sp) v += parts[(size_t)sp * kTile + q];
      S[(q / (16 * NT)) * LDT + q % (16 * NT)] = v;
    }
    __syncthreads();
  }

  // epilogue: wave wv finishes rows m0 + 4 wv + kq (one row per 16-lane group)
  const T g2 = (T)(2.0 * pv.gamma);
  if (mode == FTR_STEP) {
    T* __restrict__ Xn = b.X[st->ix_new];
    // row-scaled step: this group's row takes step * w_m
    const T stp = (T)((b.wrow && mval) ? step * b.wrow[m] : step);
    // the mixed instantiation also hands the forward product the step X_new - X_cur in FP32
    constexpr bool delta = !std::is_same<TS, TC>::value;
    T z[1][NT];
    T xcs[NT], ys[NT];
    form_y(hx, hy, hly);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + i;
      const T xc = hx[nt], y = hy[nt], ly = hly[nt];
      xcs[nt] = xc;
      ys[nt] = y;
      T zz = (n < N) ? (T)0 : neg_huge<T>();
      if (mval && n < N) {
        const T g = (T)2 * (T)S[(4 * wv + kq) * LDT + n] + g2 * ly;
        zz = y - stp * g;
      }
      z[0][nt] = zz;
    }
    T tau[1];
    simplex_threshold<T, 16, NT, 1, 8>(z, tau);
    double rr = 0.0;  // this row's gradient-restart term, sum_n (Y - X_new)(X_new - X_cur) / w_m
    // the regulariser's row pairs inside the tile are summed here from the new rows (each
    // group's row replaces its gradient row in S: only that group reads or writes it)
    const bool regp = b.regpart && pv.gamma != 0.0 && M > 1;
    const int r = 4 * wv + kq;
    if (mval) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int n = nt * 16 + i;
        const T xn = (n < N) ? fmax(z[0][nt] - tau[0], (T)0) : (T)0;
        Xn[(size_t)m * Npad + n] = xn;
        if constexpr (delta) b.dX[(size_t)m * Npad + n] = (float)(xn - xcs[nt]);
        if (n < N) rr += ((double)ys[nt] - (double)xn) * ((double)xn - (double)xcs[nt]);
        if (regp) S[r * LDT + n] = (double)xn;
      }
      if (b.wrow) rr /= b.wrow[m];
    }
    if (b.rpart) {
      rr = group_sum<64>(rr);
      if (lane == 0) red[wv] = rr;
      __syncthreads();
      if (tid == 0) {
        double sr = 0.0;
#pragma unroll
        for (int w = 0; w < KS; ++w) sr += red[w];
        b.rpart[mt] = sr;
      }
    }
    if (regp) {
      // pairs (m, m + 1) with both rows in this tile; the pair across the tile's lower edge
      // is the forward product's
      __shared__ double regred[KS];
      __syncthreads();
      double rs = 0.0;
      if (mval && r < 15 && m + 1 < M) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int n = nt * 16 + i;
          if (n < N) {
            const double e = S[r * LDT + n] - S[(r + 1) * LDT + n];
            rs += e * e;
          }
        }
      }
      rs = group_sum<64>(rs);
      if (lane == 0) regred[wv] = rs;
      __syncthreads();
      if (tid == 0) {
        double sg = 0.0;
#pragma unroll
        for (int w = 0; w < KS; ++w) sg += regred[w];
        b.regpart[mt] = sg;
      }
    }
  } else {
    // gradient at X_cur (R_rej = F X_cur - P) and the KKT residual partial
    double part = 0.0;
    T g[NT], x[NT];
    T gmin = FLT_MAX;
    // rows m-1, m, m+1 of every column tile are loaded before any is used
    const int mc = m < M - 1 ? m : M - 1;
    const size_t r0 = (size_t)mc * Npad + i;
    const size_t rm = mc > 0 ? r0 - Npad : r0;
    const size_t rq = mc < M - 1 ? r0 + Npad : r0;
    T a[NT], am[NT], aq[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      a[nt] = Xc[r0 + 16 * nt];
      am[nt] = Xc[rm + 16 * nt];
      aq[nt] = Xc[rq + 16 * nt];
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + i;
      g[nt] = 0;
      x[nt] = 0;
      if (mval && n < N) {
        const T xc = a[nt];
        const T lx = (m > 0 ? xc - am[nt] : (T)0) + (m < M - 1 ? xc - aq[nt] : (T)0);
        g[nt] = (T)2 * (T)S[(4 * wv + kq) * LDT + n] + g2 * lx;
        x[nt] = xc;
        gmin = fmin(gmin, g[nt]);
      }
      if (mval) b.G[(size_t)m * Npad + n] = g[nt];
    }
    gmin = group_min<16>(gmin);
    // and the Frank-Wolfe gap partial: sum over the row of x (g - min g)
    double gap = 0.0;
    if (mval) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int n = nt * 16 + i;
        if (n < N) {
          const double e = (double)x[nt] * ((double)g[nt] - (double)gmin);
          part += e * e;
          gap += e;
        }
      }
    }
    part = group_sum<64>(part);
    gap = group_sum<64>(gap);
    __shared__ double red2[KS];
    if (lane == 0) {
      red[wv] = part;
      red2[wv] = gap;
    }
    __syncthreads();
    if (tid == 0) {
      double s = 0.0, s2 = 0.0;
#pragma unroll
      for (int w = 0; w < KS; ++w) {
        s += red[w];
        s2 += red2[w];
      }
      b.partials[mt] = s;
      b.partials[(M + 15) / 16 + mt] = s2;
    }
  }
}


// At least two waves per SIMD: the forward product's loads and recursion are
// latency-bound.  Workgroups are dispatched in blockIdx order, and the band work of a tile grows with its
// photon numbers (probe means): the grid runs from the last tile to the first, so the
// heaviest tiles start first and the light ones fill the tail of the launch.  Each tile
// still writes its own partials, so the order of every sum is unchanged.
template <typename TS, typename TC, int NT, int KS>
__global__ __launch_bounds__(64 * KS, 2) void fx_kernel(ProbView pv, Bufs<TS> b,
                                                                                            SolverState* st, int mode) {
  fx_body<TS, TC, NT, KS>(pv, b, st, mode, gridDim.x - 1 - blockIdx.x, gridDim.x);
}

template <typename TS, typename TC, int NT, int KS>
__global__ __launch_bounds__(64 * KS) void ftr_kernel(ProbView pv, Bufs<TS> b, SolverState* st, int mode,
                                                       double step, int phase) {
  ftr_body<TS, TC, NT, KS>(pv, b, st, mode, step, gridDim.x - 1 - blockIdx.x, phase);
}

// every row tile narrow: no chunk staging, a smaller register and LDS footprint
template <typename TS, typename TC, int NT>
__global__ __launch_bounds__(256, NT <= 9 ? 4 : 3) void ftr_narrow_kernel(ProbView pv, Bufs<TS> b, SolverState* st, int mode,
                                                          double step) {
  ftr_body<TS, TC, NT, 4, true>(pv, b, st, mode, step, gridDim.x - 1 - blockIdx.x, FTR_FUSED);
}

// Batched launches: one workgroup per (instance, tile) item of a work list; every
// instance carries its own problem view, buffers, state and step.
template <typename TS, typename TC, int NT, int KS>
__global__ __launch_bounds__(64 * KS) void fx_batch_kernel(const BatchInst<TS>* insts, const int2* items, int mode) {
  const int2 it = items[blockIdx.x];
  const BatchInst<TS>& I = insts[it.x];
  fx_body<TS, TC, NT, KS>(I.pv, I.b, I.st, mode, it.y, I.n_dt);
}

template <typename TS, typename TC, int NT, int KS>
__global__ __launch_bounds__(64 * KS) void ftr_batch_kernel(const BatchInst<TS>* insts, const int2* items,
                                                             int mode) {
  const int2 it = items[blockIdx.x];
  const BatchInst<TS>& I = insts[it.x];
  ftr_body<TS, TC, NT, KS>(I.pv, I.b, I.st, mode, I.step, it.y);
}


// ---------------------------------------------------------------------------------------
// Launchers: the column-tile class NT = Npad / 16 and the waves per workgroup KS (4 or 8,
// from the problem view, or per work list for batches) select the instantiation.
// ---------------------------------------------------------------------------------------
template <typename TS, typename TC, int NT, int KS>
static void fx_go(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, hipStream_t s) {
  hipLaunchKernelGGL((fx_kernel<TS, TC, NT, KS>), dim3(fx_num_tiles(pv) * pv.fx_split), dim3(64 * KS), 0, s, pv, b,
                     st, mode);
}
template <typename TS, typename TC, int NT, int KS>
static void ftr_go(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, double step,
                   hipStream_t s) {
  if (pv.ftr_split > 1) {
    hipLaunchKernelGGL((ftr_kernel<TS, TC, NT, KS>), dim3(ftr_num_waves(pv) * pv.ftr_split), dim3(64 * KS), 0, s,
                       pv, b, st, mode, step, (int)FTR_PART);
    hipLaunchKernelGGL((ftr_kernel<TS, TC, NT, KS>), dim3(ftr_num_waves(pv)), dim3(64 * KS), 0, s, pv, b, st, mode,
                       step, (int)FTR_FINISH);
  } else {
    hipLaunchKernelGGL((ftr_kernel<TS, TC, NT, KS>), dim3(ftr_num_waves(pv)), dim3(64 * KS), 0, s, pv, b, st, mode,
                       step, (int)FTR_FUSED);
  }
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
  if (pv.ks_fx == 8) {
#define PDT_FX(K) fx_go<TS, TC, K, 8>(pv, b, st, mode, s)
    PDT_NT_SWITCH(pv.Npad / 16, PDT_FX)
#undef PDT_FX
  } else if (pv.ks_fx == 4) {
#define PDT_FX(K) fx_go<TS, TC, K, 4>(pv, b, st, mode, s)
    PDT_NT_SWITCH(pv.Npad / 16, PDT_FX)
#undef PDT_FX
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TS, typename TC>
hipError_t launch_ftr(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, double step,
                      hipStream_t s) {
  if (pv.ftr_narrow_all && pv.ftr_split == 1) {
#define PDT_FTRN(K)                                                                                             \
  hipLaunchKernelGGL((ftr_narrow_kernel<TS, TC, K>), dim3(ftr_num_waves(pv)), dim3(256), 0, s, pv, b, st, mode, \
                     step)
    PDT_NT_SWITCH(pv.Npad / 16, PDT_FTRN)
#undef PDT_FTRN
  } else if (pv.ks_ftr == 8) {
#define PDT_FTR(K) ftr_go<TS, TC, K, 8>(pv, b, st, mode, step, s)
    PDT_NT_SWITCH(pv.Npad / 16, PDT_FTR)
#undef PDT_FTR
  } else if (pv.ks_ftr == 4) {
#define PDT_FTR(K) ftr_go<TS, TC, K, 4>(pv, b, st, mode, step, s)
    PDT_NT_SWITCH(pv.Npad / 16, PDT_FTR)
#undef PDT_FTR
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TS, typename TC, int NT, int KS>
static void fxb_go(const BatchInst<TS>* insts, const int2* items, int n_items, int mode, hipStream_t s) {
  hipLaunchKernelGGL((fx_batch_kernel<TS, TC, NT, KS>), dim3(n_items), dim3(64 * KS), 0, s, insts, items, mode);
}
template <typename TS, typename TC, int NT, int KS>
static void ftrb_go(const BatchInst<TS>* insts, const int2* items, int n_items, int mode, hipStream_t s) {
  hipLaunchKernelGGL((ftr_batch_kernel<TS, TC, NT, KS>), dim3(n_items), dim3(64 * KS), 0, s, insts, items, mode);
}

template <typename TS, typename TC>
hipError_t launch_fx_batch(int nt, int ks, const BatchInst<TS>* insts, const int2* items, int n_items, int mode,
                           hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (ks == 8) {
#define PDT_FXB(K) fxb_go<TS, TC, K, 8>(insts, items, n_items, mode, s)
    PDT_NT_SWITCH(nt, PDT_FXB)
#undef PDT_FXB
  } else if (ks == 4) {
#define PDT_FXB(K) fxb_go<TS, TC, K, 4>(insts, items, n_items, mode, s)
    PDT_NT_SWITCH(nt, PDT_FXB)
#undef PDT_FXB
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TS, typename TC>
hipError_t launch_ftr_batch(int nt, int ks, const BatchInst<TS>* insts, const int2* items, int n_items, int mode,
                            hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (ks == 8) {
#define PDT_FTRB(K) ftrb_go<TS, TC, K, 8>(insts, items, n_items, mode, s)
    PDT_NT_SWITCH(nt, PDT_FTRB)
#undef PDT_FTRB
  } else if (ks == 4) {
#define PDT_FTRB(K) ftrb_go<TS, TC, K, 4>(insts, items, n_items, mode, s)
    PDT_NT_SWITCH(nt, PDT_FTRB)
#undef PDT_FTRB
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pdt
