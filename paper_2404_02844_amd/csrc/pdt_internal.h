// Internal declarations shared by the HIP kernels and the host driver of libpdt.
//
// Layout in device memory (one tomography instance):
//   mu      [D]           probe mean photon numbers, FP64
//   lo, hi  [D]           first/last photon number of each probe's F band (int32)
//   tail    [D]           F[d][M-1] when the tail is lumped into the last column
//   rinv    [M + 128]     1/m (rinv[0] = 0): the recursion p(m+1) = p(m) mu / (m+1)
//   r4      [M + 128]     1/((m+1)(m+2)(m+3)(m+4)): the stride-4 recursion of the forward product
//   anchors               F[d][16 t] for each 16-row tile t and each probe d it meets
//   dt_mlo/dt_mhi         per 16-probe tile: photon-number range its bands cover
//   mt_dlo/mt_dhi         per 16-row tile of Pi: probe range whose bands touch it
//   P       [D][Npad]     outcome frequencies, zero padded to Npad = 16 * ceil(N / 16)
//   X[3]    [M][Npad]     iterates of Pi (current, previous, candidate; roles rotate)
//   O[3]    [D][Npad]     F X for the three iterates
//   R_acc, R_rej [D][Npad] residual F Y - P for the next step, if the candidate is
//                         accepted / rejected (both formed before the decision)
//   dX      [M][Npad]     FP32 candidate step X_new - X_cur (mixed path only)
//   R32_acc, R32_rej [D][Npad] FP32 copies of the residual candidates (mixed path only)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdt {

constexpr int kTile = 16;         // MFMA tile edge
constexpr int kChunkM = 64;       // photon numbers per forward-product chunk
constexpr int kChunkD = 64;       // probes per transposed-product chunk
constexpr int kNarrowD = 32;      // probe ranges up to this many probes skip the chunks
constexpr int kMaxNT = 12;        // outcome columns up to 192
constexpr int kWave = 64;

// FX_EVAL_PREV / FX_RESYNC: exact FP64 products of X_prev and X_cur that end each chunk
// of the mixed path (O, both residual candidates and f of X_cur made exact again)
enum FxMode { FX_ITER = 0, FX_INIT = 1, FX_EVAL = 2, FX_DELTA = 3, FX_EVAL_PREV = 4, FX_RESYNC = 5 };
enum FtrMode { FTR_STEP = 0, FTR_GRAD = 1 };
// Phases of the transposed product: one fused launch, or (split contraction) a launch of
// partial tiles followed by a launch that sums them and runs the epilogue.
enum FtrPhase { FTR_FUSED = 0, FTR_PART = 1, FTR_FINISH = 2 };
// DEC_KKT: the KKT residual and Frank-Wolfe gap of X_cur from a gradient launch's
// partials ([n] KKT sums, then [n] gap sums), and the KKT stopping test
enum DecideMode { DEC_ITER = 0, DEC_INIT = 1, DEC_EVAL = 2, DEC_RESYNC = 3, DEC_KKT = 4 };

// Device-resident solver state of one instance.  Written only by the decide kernel
// (one thread, vector stores), read by every other kernel.
struct SolverState {
  double f_cur;    // objective at the current iterate
  double f_new;    // objective of the latest candidate
  double f_eval;   // objective of the last plain evaluation
  double t;        // momentum parameter t_k
  double beta;     // extrapolation weight for the next transposed-product launch
  double f_star;   // target optimum (<= 0: none)
  double rel_tol;  // stop once f_cur - f_star <= rel_tol * f_star
  double kkt;      // last KKT residual (DEC_KKT)
  double fw;       // last Frank-Wolfe gap (DEC_KKT)
  double kkt_tol;  // stop once kkt <= kkt_tol (<= 0: no KKT test)
  double mn;       // M N, the count of the KKT residual's mean
  long long iter;
  long long rejects;
  long long max_iters;
  long long hist_stride;  // history[k / stride] = f after iteration k, k % stride == 0 (0 acts as 1)
  int ix_cur, ix_prev, ix_new;
  int sel_acc;     // 1: next step uses R_acc, 0: R_rej
  int done;
  int kkt_hit;     // 1: done was set by the KKT test
};

struct ProbView {
  const double* mu;
  const int* lo;
  const int* hi;
  const double* tail;
  const double* rinv;
  const double* r4;       // 1 / ((m+1)(m+2)(m+3)(m+4))
  const double* anchors;  // F[d][16 t] per row tile t and probe d of its range
  const long long* mt_aoff;
  const int* dt_mlo;
  const int* dt_mhi;
  const int* mt_dlo;
  const int* mt_dhi;
  int M, D, N, Npad, lump;
  double gamma;
  int ks_fx = 4;   // waves per workgroup of the forward product (4 or 8)
  int ks_ftr = 4;  // waves per workgroup of the transposed product (4 or 8)
  int fx_split = 1;  // workgroups sharing one 16-probe tile of the forward product
  int ftr_split = 1;  // workgroups sharing one 16-row tile of the transposed product
  int ftr_narrow_all = 0;  // every row tile's probe range is narrow (under kNarrowD probes)
};

template <typename T>
struct Bufs {
  T* X[3];
  T* O[3];
  const T* P;
  T* R_acc;
  T* R_rej;
  T* G;              // gradient output (FTR_GRAD)
  double* partials;  // one FP64 partial per wave
  int n_partials;
  double* history;   // f after every iteration (may be null)
  const double* wrow = nullptr;  // [M] per-row step weights (null: every row takes the step)
  float* dX = nullptr;           // [M][Npad] FP32 X_new - X_cur (mixed path: written by the
                                 // transposed product, read by the forward product)
  double* fx_part = nullptr;     // [tiles * fx_split][16][16 NT] partial tiles (split forward product)
  unsigned* fx_count = nullptr;  // [tiles] finished workgroups per tile, zero between launches
  double* ftr_part = nullptr;    // [row tiles * ftr_split][16][16 NT] partial tiles (split
                                 // transposed product)
  const int* skip = nullptr;     // when set and *skip != 0 the launch returns at once (the
                                 // Hessian products of a conjugate-gradient solve that stopped)
  double* rpart = nullptr;       // [ceil(M / 16)] gradient-restart partials, one per row tile,
                                 // written by the step (null: function restart only)
  double* regpart = nullptr;     // [ceil(M / 16)] the new iterate's regulariser sums over the row
                                 // pairs inside each 16-row tile, written by the step and read
                                 // by the forward product of the same iteration (null: the
                                 // forward product sums every pair itself)
  float* R32_acc = nullptr;      // [D][Npad] FP32 copies of R_acc / R_rej (mixed path): every
  float* R32_rej = nullptr;      // forward-product epilogue that writes R writes them too, and
                                 // the FP32-operand transposed product reads them instead of R
};

// One instance of a batched launch: its problem view, buffers, state and step; n_dt
// = number of 16-probe tiles (forward-product work items and objective partials).
template <typename T>
struct BatchInst {
  ProbView pv;
  Bufs<T> b;
  SolverState* st;
  double step;
  int n_dt;
  int n_mt;
};

// Launchers (pdt_kernels.hip).
// TS: storage type, TC: MFMA operand type (TC = TS, or float products on FP64 storage)
template <typename TS, typename TC = TS>
hipError_t launch_fx(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, hipStream_t s);
template <typename TS, typename TC = TS>
hipError_t launch_ftr(const ProbView& pv, const Bufs<TS>& b, SolverState* st, int mode, double step,
                      hipStream_t s);
// rpart / nr: the step's gradient-restart partials (DEC_ITER; null: function restart only)
hipError_t launch_decide(const double* partials, int n, SolverState* st, double* history, int mode,
                         hipStream_t s, const double* rpart = nullptr, int nr = 0);
hipError_t launch_setup_bands(const double* mu, int D, int M, double tau, int lump, int* lo, int* hi,
                              double* tail, hipStream_t s);
hipError_t launch_fill_rinv(double* rinv, double* r4, int n, hipStream_t s);
hipError_t launch_setup_anchors(const ProbView& pv, const long long* mt_aoff, double* anchors, hipStream_t s);
template <typename T>
hipError_t launch_project_rows(const T* X, T* Y, long long rows, int cols, int ld_in, int ld_out,
                               hipStream_t s);
// Hessian diagonal per row: h[m] = 2 sum_d F[d][m]^2 + 2 gamma L[m][m]
hipError_t launch_setup_hdiag(const ProbView& pv, double* hdiag, hipStream_t s);
// lambda = sqrt(sum_m w_m G_m^2), V_m = w_m G_m / lambda (w = null: all ones);
// scratch: device [512] doubles
hipError_t launch_power_normalize(double* G, double* V, int M, int ld, const double* w, double* scratch,
                                  double* lam_out, hipStream_t s);
hipError_t launch_reduce_sum(const double* partials, int n, double* out, hipStream_t s);
// batches: out[k] = *st[k]; st[k]->done = 1 where flags[k] != 0
hipError_t launch_gather_states(SolverState* const* st, int n, SolverState* out, hipStream_t s);
hipError_t launch_mark_done(SolverState* const* st, const int* flags, int n, hipStream_t s);
template <typename Ts, typename Td>
hipError_t launch_convert_pad(const Ts* src, Td* dst, long long rows, int cols, int ld_src, int ld_dst,
                              hipStream_t s);

// Message returned by pdt_last_error() for the calling thread (pdt_capi.hip); "" clears it.
void set_last_error(const char* msg);

// Long-range smoothing (pdt_smooth.hip); scratch: device [smooth_scratch_doubles(M, N)]
long long smooth_scratch_doubles(long long M, int N);
hipError_t launch_smooth_rows(const double* Pi, double* out, long long M, int N, int divisor, long long skip,
                              double* scratch, hipStream_t s);

// R_rej = O[ix_cur] - P over [D][Npad]: the residual of the current iterate, which a
// gradient launch (FTR_GRAD) reads
template <typename T>
hipError_t launch_resid_cur(const Bufs<T>& b, const SolverState* st, long long n, hipStream_t s);

template <typename T>
hipError_t launch_fill_rows(T* X, long long rows, int cols, int ld, T value, hipStream_t s);

// batched launches over work lists of (instance, tile) items of one column-tile class nt
template <typename TS, typename TC = TS>
hipError_t launch_fx_batch(int nt, int ks, const BatchInst<TS>* insts, const int2* items, int n_items, int mode,
                           hipStream_t s);
template <typename TS, typename TC = TS>
hipError_t launch_ftr_batch(int nt, int ks, const BatchInst<TS>* insts, const int2* items, int n_items, int mode,
                            hipStream_t s);
template <typename TS>
hipError_t launch_decide_batch(const BatchInst<TS>* insts, int n_inst, int mode, hipStream_t s);

// 16-probe tiles of the forward product; its partials (the decide kernels' count):
// one per tile, or with a split contraction one per workgroup plus one per tile
int fx_num_tiles(const ProbView& pv);
int fx_num_waves(const ProbView& pv);
int ftr_num_waves(const ProbView& pv);

}  // namespace pdt
