// C ABI and host driver of libpdt: problem setup, the projected-gradient loop, and
// the objective / projection entry points declared in include/pdt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "pdt.h"
#include "pdt_internal.h"
#include "pdt_newton.h"
#include "pdt_tuning.h"
#include "pdt_mlp.h"

using namespace pdt;

namespace {

thread_local std::string g_last_error;

struct DevError {
  hipError_t code;
  std::string what;
};
struct OomError {
  std::string what;
};
struct ArgError {
  std::string what;
};

#define HIPCHK(...)                                                              \
  do {                                                                           \
    hipError_t e_ = (__VA_ARGS__);                                               \
    if (e_ != hipSuccess)                                                        \
      throw DevError{e_, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// Device allocations owned by one problem.
struct Arena {
  std::vector<void*> ptrs;
  template <typename T>
  T* alloc(size_t n) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw OomError{"hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

// kernel variants of the iteration: storage / MFMA type
enum Variant { VAR_FP64 = 0, VAR_FP32 = 1, VAR_MIXED = 2 };

template <typename T>
struct Work {
  float* dX = nullptr;  // FP32 X_new - X_cur of the mixed path (FP64 storage only)
  float* R32_acc = nullptr;  // FP32 copies of R_acc / R_rej for the mixed path's transposed product
  float* R32_rej = nullptr;
  T* X[3] = {nullptr, nullptr, nullptr};
  T* O[3] = {nullptr, nullptr, nullptr};
  T* R_acc = nullptr;
  T* R_rej = nullptr;
  T* G = nullptr;
  const T* P = nullptr;
  bool ready = false;
};

// Buffers of the Newton solver ([M][Npad] unless noted), allocated on first use.
struct NewtonWork {
  bool ready = false;
  double* Dir = nullptr;  // Newton direction (stage 2: reduced variables)
  double* res = nullptr;  // CG residual
  double* z = nullptr;    // preconditioned residual
  double* p = nullptr;    // CG search direction
  double* q = nullptr;    // D p
  double* Vf = nullptr;   // free part of p (stage 2: expanded by T), the Hessian's operand
  double* Gh = nullptr;   // H Vf
  double* G = nullptr;    // gradient at the current iterate
  double* Oh = nullptr;   // [D][Npad] F Vf
  double* Rh = nullptr;   // [D][Npad] F Vf (the transposed product's operand)
  double* Pz = nullptr;   // [D][Npad] zeros: the data term of a Hessian product
  double* Rg = nullptr;   // [D][Npad] F X - P of the last evaluated point
  double* part = nullptr;  // [4 kNtBlocks] row-kernel partials
  double* bpart = nullptr;  // band-kernel partials
  uint8_t* mask = nullptr;
  int* mi = nullptr;       // [M] row maxima of stage 2
  NewtonState* ns = nullptr;
  SolverState* st = nullptr;  // ix_cur = 0, never done: plain evaluations
  int* flag_h = nullptr;      // pinned, coherent host [2]: CG completion flags
  int* flag_d = nullptr;      // their device address
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t cg_graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [stage - 1][flag slot]
};

struct Instance {
  int64_t M = 0, N = 0, D = 0, Npad = 0;
  double gamma = 0, tau = 0;
  int lump = 0;
  double L_hat = 0;
  double L_w = 0;  // 1.05 lambda_max(W^(1/2) H W^(1/2)) for the row-scaled step (0: not yet computed)
  int64_t nnz = 0;
  int bins = 0;  // last outcome column with any probability mass (outcomes 0..bins are real)
  std::vector<int> lo_h, hi_h;
  std::vector<double> tail_h;
  double* mu = nullptr;
  int* lo = nullptr;
  int* hi = nullptr;
  double* tail = nullptr;
  double* rinv = nullptr;
  double* r4 = nullptr;
  double* anchors = nullptr;
  long long* mt_aoff = nullptr;
  int* dt_mlo = nullptr;
  int* dt_mhi = nullptr;
  int* mt_dlo = nullptr;
  int* mt_dhi = nullptr;
  double* P64 = nullptr;
  float* P32 = nullptr;
  double* hdiag = nullptr;  // [M] Hessian diagonal per row
  double* wrow = nullptr;   // [M] w_m = 1 / max(h_m, 1e-12 max h)
  std::vector<double> hdiag_h, wrow_h;
  Work<double> w64;
  Work<float> w32;
  double* partials = nullptr;
  int n_partials = 0;
  double* rpart = nullptr;  // [ceil(M / 16)] gradient-restart partials of the step
  double* regpart = nullptr;  // [ceil(M / 16)] in-tile regulariser sums of the step's iterate
  SolverState* st = nullptr;
  SolverState* st_eval = nullptr;
  double* scalar = nullptr;
  // captured chunks of iterations, one slot per kernel variant, reused while
  // (step, history) match
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
  double graph_step[3] = {0.0, 0.0, 0.0};
  double* graph_hist[3] = {nullptr, nullptr, nullptr};
  const double* graph_w[3] = {nullptr, nullptr, nullptr};
  bool graph_kkt[3] = {false, false, false};
  const double* graph_rp[3] = {nullptr, nullptr, nullptr};
  // waves per workgroup forced per variant and kernel (0: from the tuning table)
  int ks_force[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  // split contraction of the forward product: workgroups per 16-probe tile
  int fx_split = 1;
  int fx_split_auto = 1;
  size_t fx_part_cap = 0;        // doubles allocated for fx_part
  double* fx_part = nullptr;
  unsigned* fx_count = nullptr;
  // split contraction of the transposed product: workgroups per 16-row tile
  int ftr_split = 1;
  int ftr_split_auto = 1;
  int ftr_narrow_all = 0;  // every row tile's probe range is under kNarrowD probes
  size_t ftr_part_cap = 0;       // doubles allocated for ftr_part
  double* ftr_part = nullptr;
  NewtonWork nw;
};

}  // namespace

namespace pdt {
void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }
}  // namespace pdt

struct pdt_model_s;

// One launch of a batched phase: the items of one column-tile class and workgroup shape.
struct LaunchList {
  int nt = 0, ks = 4;
  int2* items = nullptr;
  int n = 0;
};

struct BatchPlan {
  int prec = -1;
  int scaling = -1;
  int restart = -1;
  std::vector<double> steps;
  void* insts = nullptr;          // device BatchInst<T>[n]
  std::vector<LaunchList> fx, ftr;
  hipGraphExec_t graph = nullptr;
};

struct pdt_problem_s {
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;  // library-owned stream used only to record graphs
  BatchPlan plan[2];              // batched launches: [0] FP64, [1] FP32
  Arena plan_arena[2];
  SolverState** st_ptrs = nullptr;   // device [n_instances]: every instance's state
  SolverState* st_gather = nullptr;  // device [n_instances]: their copies, read once per chunk
  int* st_flags = nullptr;           // device [n_instances]: stop flags set by the host
  int device = 0;
  Arena arena;
  std::vector<Instance> inst;
};

namespace {

pdt_status set_err(pdt_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

// Maps the exception in flight to a status; nothing may leave an extern "C" entry point.
pdt_status status_of_current_exception() {
  try {
    throw;
  } catch (const ArgError& e) {
    return set_err(PDT_ERR_INVALID_ARG, e.what);
  } catch (const OomError& e) {
    return set_err(PDT_ERR_OUT_OF_MEMORY, e.what);
  } catch (const DevError& e) {
    return set_err(PDT_ERR_DEVICE, e.what);
  } catch (const std::bad_alloc&) {
    return set_err(PDT_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return set_err(PDT_ERR_DEVICE, "unexpected exception");
  }
}

ProbView view_of(const Instance& I) {
  ProbView pv;
  pv.mu = I.mu;
  pv.lo = I.lo;
  pv.hi = I.hi;
  pv.tail = I.tail;
  pv.rinv = I.rinv;
  pv.r4 = I.r4;
  pv.anchors = I.anchors;
  pv.mt_aoff = I.mt_aoff;
  pv.dt_mlo = I.dt_mlo;
  pv.dt_mhi = I.dt_mhi;
  pv.mt_dlo = I.mt_dlo;
  pv.mt_dhi = I.mt_dhi;
  pv.M = (int)I.M;
  pv.D = (int)I.D;
  pv.N = (int)I.N;
  pv.Npad = (int)I.Npad;
  pv.lump = I.lump;
  pv.gamma = I.gamma;
  pv.fx_split = I.fx_split;
  pv.ftr_split = I.ftr_split;
  pv.ftr_narrow_all = I.ftr_narrow_all;
  return pv;
}

// Waves per workgroup of the band kernels for the view's column-tile class and tile
// counts: forced per instance, or from the tuning table.
void apply_ks(ProbView& pv, const Instance& I, int var) {
  const int nt = pv.Npad / 16;
  pv.ks_fx = I.ks_force[var][0] ? I.ks_force[var][0] : choose_ks(var, 0, nt, (pv.D + 15) / 16);
  pv.ks_ftr = I.ks_force[var][1] ? I.ks_force[var][1] : choose_ks(var, 1, nt, (pv.M + 15) / 16);
}

ProbView view_var(const Instance& I, int var) {
  ProbView pv = view_of(I);
  apply_ks(pv, I, var);
  return pv;
}

// r32: also hand the kernels the FP32 residual copies (the mixed path's launches);
// restart: the gradient restart's partials (pdt_restart)
template <typename T>
Bufs<T> bufs_of(const Instance& I, const Work<T>& w, double* history, const double* wrow = nullptr,
                bool r32 = false, int restart = PDT_RESTART_FUNCTION) {
  Bufs<T> b;
  for (int k = 0; k < 3; ++k) {
    b.X[k] = w.X[k];
    b.O[k] = w.O[k];
  }
  b.fx_part = I.fx_part;
  b.fx_count = I.fx_count;
  b.ftr_part = I.ftr_part;
  b.P = w.P;
  b.R_acc = w.R_acc;
  b.R_rej = w.R_rej;
  b.G = w.G;
  b.partials = I.partials;
  b.n_partials = I.n_partials;
  b.history = history;
  b.wrow = wrow;
  b.dX = w.dX;
  if (r32) {
    b.R32_acc = w.R32_acc;
    b.R32_rej = w.R32_rej;
  }
  if (restart == PDT_RESTART_GRADIENT) b.rpart = I.rpart;
  b.regpart = I.regpart;
  return b;
}

template <typename T>
void ensure_work(Arena& A, Instance& I, Work<T>& w, const T* P) {
  if (w.ready) return;
  const size_t xm = (size_t)I.M * I.Npad, od = (size_t)I.D * I.Npad;
  for (int k = 0; k < 3; ++k) {
    w.X[k] = A.alloc<T>(xm);
    w.O[k] = A.alloc<T>(od);
  }
  w.R_acc = A.alloc<T>(od);
  w.R_rej = A.alloc<T>(od);
  w.G = A.alloc<T>(xm);
  w.P = P;
  w.ready = true;
}

void validate_desc(const pdt_problem_desc& d) {
  if (d.M < 1 || d.N < 1 || d.D < 1) throw ArgError{"M, N and D must be >= 1"};
  if (d.N > 16 * kMaxNT) throw ArgError{"N must be <= " + std::to_string(16 * kMaxNT)};
  if (d.M > (int64_t)INT_MAX - 1024 || d.D > (int64_t)INT_MAX - 1024) throw ArgError{"M or D too large"};
  const int64_t npad = (d.N + 15) / 16 * 16;
  // the kernels address [M][Npad] and [D][Npad] arrays with 32-bit offsets
  if (d.M * npad > (int64_t)INT_MAX || d.D * npad > (int64_t)INT_MAX)
    throw ArgError{"M*Npad and D*Npad must be < 2^31 (Npad = 16 * ceil(N / 16))"};
  if (!d.mu || !d.P) throw ArgError{"mu and P must not be NULL"};
  if (!std::isfinite(d.gamma) || d.gamma < 0) throw ArgError{"gamma must be finite and >= 0"};
  if (!std::isfinite(d.pmf_threshold) || d.pmf_threshold < 0 || d.pmf_threshold >= 1)
    throw ArgError{"pmf_threshold must be in [0, 1)"};
  if (d.tail_mode != PDT_TAIL_TRUNCATE && d.tail_mode != PDT_TAIL_LUMP) throw ArgError{"bad tail_mode"};
  for (int64_t k = 0; k < d.D; ++k) {
    const double m = d.mu[k];
    if (!std::isfinite(m) || m < 0) throw ArgError{"mu must be finite and >= 0"};
    if (k > 0 && m < d.mu[k - 1]) throw ArgError{"mu must be non-decreasing"};
    if (m > 1e12) throw ArgError{"mu too large"};
  }
  if (!d.P_on_device) {
    const int64_t n = d.D * d.N;
    for (int64_t k = 0; k < n; ++k)
      if (!std::isfinite(d.P[k]) || d.P[k] < 0) throw ArgError{"P must be finite and >= 0"};
  }
}

constexpr int kMaxFxSplit = 16;

// Workgroups per 16-probe tile of the forward product; grows the partial-tile scratch
// when needed (allocations stay with the problem).
void set_fx_split(Arena& A, Instance& I, int split) {
  const size_t n_dt = (size_t)((I.D + 15) / 16);
  const size_t need = split > 1 ? n_dt * (size_t)split * 16 * (size_t)I.Npad : 0;
  if (need > I.fx_part_cap) {
    I.fx_part = A.alloc<double>(need);
    I.fx_part_cap = need;
  }
  I.fx_split = split;
}

constexpr int kMaxFtrSplit = 16;

// Workgroups per 16-row tile of the transposed product (the same scratch rule).
void set_ftr_split(Arena& A, Instance& I, int split) {
  const size_t n_mt = (size_t)((I.M + 15) / 16);
  const size_t need = split > 1 ? n_mt * (size_t)split * 16 * (size_t)I.Npad : 0;
  if (need > I.ftr_part_cap) {
    I.ftr_part = A.alloc<double>(need);
    I.ftr_part_cap = need;
  }
  I.ftr_split = split;
}

// Power iteration for lambda_max(W^(1/2) (2 F^T F + 2 gamma L) W^(1/2)) with the band
// kernels (N = 1); W = diag(wrow), or the identity when wrow is null.
double lipschitz_power(pdt_problem_s* pb, Instance& I, int iters, const double* wrow = nullptr) {
  Arena tmp;
  hipStream_t s = pb->stream;
  ProbView pv = view_of(I);
  pv.N = 1;
  pv.Npad = 16;
  apply_ks(pv, I, VAR_FP64);
  const size_t xm = (size_t)I.M * 16, od = (size_t)I.D * 16;
  try {
    Work<double> w;
    w.X[0] = tmp.alloc<double>(xm);
    w.X[1] = w.X[2] = w.X[0];
    w.O[0] = tmp.alloc<double>(od);
    w.O[1] = w.O[2] = w.O[0];
    double* Pz = tmp.alloc<double>(od);
    w.R_rej = tmp.alloc<double>(od);
    w.R_acc = w.R_rej;
    w.G = tmp.alloc<double>(xm);
    w.P = Pz;
    SolverState* st = tmp.alloc<SolverState>(1);
    double* lam = tmp.alloc<double>(1);
    double* norm_scratch = tmp.alloc<double>(512);
    HIPCHK(hipMemsetAsync(Pz, 0, od * sizeof(double), s));
    std::vector<double> v0(xm, 0.0);
    const double inv = 1.0 / std::sqrt((double)I.M);
    for (int64_t m = 0; m < I.M; ++m) v0[(size_t)m * 16] = wrow ? std::sqrt(I.wrow_h[(size_t)m]) * inv : inv;
    HIPCHK(hipMemcpyAsync(w.X[0], v0.data(), xm * sizeof(double), hipMemcpyHostToDevice, s));
    SolverState s0;
    std::memset(&s0, 0, sizeof(s0));
    HIPCHK(hipMemcpyAsync(st, &s0, sizeof(s0), hipMemcpyHostToDevice, s));
    Bufs<double> b = bufs_of(I, w, nullptr);
    for (int it = 0; it < iters; ++it) {
      HIPCHK(launch_fx<double>(pv, b, st, FX_EVAL, s));
      HIPCHK(launch_ftr<double>(pv, b, st, FTR_GRAD, 0.0, s));
      HIPCHK(launch_power_normalize(w.G, w.X[0], (int)I.M, 16, wrow, norm_scratch, lam, s));
    }
    double lam_h = 0;
    HIPCHK(hipMemcpyAsync(&lam_h, lam, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    tmp.release();
    return 1.05 * lam_h;
  } catch (...) {
    (void)hipStreamSynchronize(s);
    tmp.release();
    throw;
  }
}

void setup_instance(pdt_problem_s* pb, Instance& I, const pdt_problem_desc& d) {
  Arena& A = pb->arena;
  hipStream_t s = pb->stream;
  I.M = d.M;
  I.N = d.N;
  I.D = d.D;
  I.Npad = (d.N + 15) / 16 * 16;
  I.gamma = d.gamma;
  I.tau = d.pmf_threshold;
  I.lump = d.tail_mode == PDT_TAIL_LUMP;
  const size_t D = (size_t)I.D, M = (size_t)I.M, Np = (size_t)I.Npad, N = (size_t)I.N;

  I.mu = A.alloc<double>(D);
  I.lo = A.alloc<int>(D);
  I.hi = A.alloc<int>(D);
  I.tail = A.alloc<double>(D);
  I.rinv = A.alloc<double>(M + 128);
  I.r4 = A.alloc<double>(M + 128);
  I.P64 = A.alloc<double>(D * Np);
  HIPCHK(hipMemcpyAsync(I.mu, d.mu, D * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(I.P64, 0, D * Np * sizeof(double), s));
  HIPCHK(hipMemcpy2DAsync(I.P64, Np * sizeof(double), d.P, N * sizeof(double), N * sizeof(double), D,
                          d.P_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  {
    std::vector<double> Ph(D * N);
    HIPCHK(hipMemcpy2DAsync(Ph.data(), N * sizeof(double), I.P64, Np * sizeof(double), N * sizeof(double), D,
                            hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    I.bins = 0;
    for (size_t n = 0; n < N; ++n) {
      double cs = 0;
      for (size_t k = 0; k < D; ++k) cs += Ph[k * N + n];
      if (cs > 0) I.bins = (int)n;
    }
  }
  HIPCHK(launch_fill_rinv(I.rinv, I.r4, (int)(M + 128), s));
  HIPCHK(launch_setup_bands(I.mu, (int)D, (int)M, I.tau, I.lump, I.lo, I.hi, I.tail, s));

  I.lo_h.resize(D);
  I.hi_h.resize(D);
  I.tail_h.resize(D);
  HIPCHK(hipMemcpyAsync(I.lo_h.data(), I.lo, D * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(I.hi_h.data(), I.hi, D * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(I.tail_h.data(), I.tail, D * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));

  // tile work lists: photon-number range of every 16-probe tile, probe range of every
  // 16-row tile of Pi
  const size_t n_dt = (D + 15) / 16, n_mt = (M + 15) / 16;
  std::vector<int> dt_mlo(n_dt, INT_MAX), dt_mhi(n_dt, -1), mt_dlo(n_mt, INT_MAX), mt_dhi(n_mt, -1);
  I.nnz = 0;
  for (size_t k = 0; k < D; ++k) {
    const int l = I.lo_h[k], h = I.hi_h[k];
    if (l > h) continue;
    I.nnz += (int64_t)(h - l + 1);
    const size_t t = k / 16;
    dt_mlo[t] = std::min(dt_mlo[t], l);
    dt_mhi[t] = std::max(dt_mhi[t], h);
    for (int q = l / 16; q <= h / 16; ++q) {
      mt_dlo[q] = std::min(mt_dlo[q], (int)k);
      mt_dhi[q] = std::max(mt_dhi[q], (int)k);
    }
  }
  for (size_t t = 0; t < n_dt; ++t)
    if (dt_mhi[t] < 0) dt_mlo[t] = 0;
  for (size_t t = 0; t < n_mt; ++t)
    if (mt_dhi[t] < 0) mt_dlo[t] = 0;
  I.dt_mlo = A.alloc<int>(n_dt);
  I.dt_mhi = A.alloc<int>(n_dt);
  I.mt_dlo = A.alloc<int>(n_mt);
  I.mt_dhi = A.alloc<int>(n_mt);
  HIPCHK(hipMemcpyAsync(I.dt_mlo, dt_mlo.data(), n_dt * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(I.dt_mhi, dt_mhi.data(), n_dt * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(I.mt_dlo, mt_dlo.data(), n_mt * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(I.mt_dhi, mt_dhi.data(), n_mt * sizeof(int), hipMemcpyHostToDevice, s));

  // anchors of the transposed product: one FP64 value per (row tile, probe in its range)
  std::vector<long long> aoff(n_mt + 1, 0);
  for (size_t t = 0; t < n_mt; ++t) aoff[t + 1] = aoff[t] + (mt_dhi[t] >= mt_dlo[t] ? mt_dhi[t] - mt_dlo[t] + 1 : 0);
  I.mt_aoff = A.alloc<long long>(n_mt + 1);
  I.anchors = A.alloc<double>((size_t)aoff[n_mt]);
  HIPCHK(hipMemcpyAsync(I.mt_aoff, aoff.data(), (n_mt + 1) * sizeof(long long), hipMemcpyHostToDevice, s));
  HIPCHK(launch_setup_anchors(view_of(I), I.mt_aoff, I.anchors, s));

  // Forward products of problems with few probe tiles and long photon-number ranges
  // split each tile's contraction over up to 16 workgroups (about three workgroups per
  // CU in all, at least 32 64-entry chunks per workgroup).
  int maxch = 0;
  for (size_t t = 0; t < n_dt; ++t)
    if (dt_mhi[t] >= dt_mlo[t]) maxch = std::max(maxch, (dt_mhi[t] - dt_mlo[t]) / kChunkM + 1);
  I.fx_split_auto = 1;
  if (n_dt < 256) I.fx_split_auto = std::max(1, std::min({16, (int)((768 + n_dt - 1) / n_dt), maxch / 32}));
  I.fx_count = A.alloc<unsigned>(n_dt);
  HIPCHK(hipMemsetAsync(I.fx_count, 0, n_dt * sizeof(unsigned), s));
  set_fx_split(A, I, I.fx_split_auto);
  I.ftr_split_auto = 1;
  I.ftr_narrow_all = 1;
  for (size_t t = 0; t < n_mt; ++t)
    if (mt_dhi[t] >= mt_dlo[t] && mt_dhi[t] - mt_dlo[t] >= kNarrowD) I.ftr_narrow_all = 0;
  set_ftr_split(A, I, I.ftr_split_auto);
  // room for the partials of any split up to kMaxFxSplit
  // and for the gradient launch's KKT and Frank-Wolfe partials (2 per row tile)
  I.n_partials = (int)std::max(n_dt * (kMaxFxSplit + 1), 2 * n_mt);
  I.partials = A.alloc<double>(I.n_partials);
  I.rpart = A.alloc<double>(n_mt);
  I.regpart = A.alloc<double>(n_mt);
  HIPCHK(hipMemsetAsync(I.regpart, 0, n_mt * sizeof(double), s));
  I.st = A.alloc<SolverState>(1);
  I.st_eval = A.alloc<SolverState>(1);
  I.scalar = A.alloc<double>(4);
  // Hessian diagonal and the row weights of the scaled step (floored at 1e-12 max h so
  // that rows no probe sees keep a finite step)
  I.hdiag = A.alloc<double>(M);
  I.wrow = A.alloc<double>(M);
  HIPCHK(launch_setup_hdiag(view_of(I), I.hdiag, s));
  I.hdiag_h.resize(M);
  I.wrow_h.resize(M);
  HIPCHK(hipMemcpyAsync(I.hdiag_h.data(), I.hdiag, M * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double hmax = 0.0;
  for (double h : I.hdiag_h) hmax = std::max(hmax, h);
  for (size_t m = 0; m < M; ++m) I.wrow_h[m] = hmax > 0.0 ? 1.0 / std::max(I.hdiag_h[m], 1e-12 * hmax) : 1.0;
  HIPCHK(hipMemcpyAsync(I.wrow, I.wrow_h.data(), M * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  I.L_hat = lipschitz_power(pb, I, 100);
}

// Lipschitz constant of the row-scaled step, computed on first use.
double scaled_lipschitz(pdt_problem_s* pb, Instance& I) {
  if (I.L_w <= 0.0) I.L_w = lipschitz_power(pb, I, 100, I.wrow);
  return I.L_w;
}

template <typename T>
Work<T>& work_of(Instance& I);
template <>
Work<double>& work_of<double>(Instance& I) { return I.w64; }
template <>
Work<float>& work_of<float>(Instance& I) { return I.w32; }

void init_state(hipStream_t s, SolverState* dst, int64_t max_iters, double f_star, double rel_tol,
                double kkt_tol = 0.0, double mn = 1.0, int64_t hist_stride = 1) {
  SolverState s0;
  std::memset(&s0, 0, sizeof(s0));
  s0.ix_cur = 0;
  s0.ix_prev = 0;
  s0.ix_new = 1;
  s0.t = 1.0;
  s0.max_iters = max_iters;
  s0.f_star = f_star;
  s0.rel_tol = rel_tol;
  s0.kkt_tol = kkt_tol;
  s0.mn = mn;
  s0.hist_stride = hist_stride > 1 ? hist_stride : 1;
  HIPCHK(hipMemcpyAsync(dst, &s0, sizeof(s0), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
}

SolverState read_state(hipStream_t s, const SolverState* src) {
  SolverState h;
  HIPCHK(hipMemcpyAsync(&h, src, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return h;
}

void write_state(hipStream_t s, SolverState* dst, const SolverState& h) {
  HIPCHK(hipMemcpyAsync(dst, &h, sizeof(h), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
}

// The state of a refinement that starts over from X[0] of FP64 storage: the counts and
// targets of the phase before it, no stop, the buffer roles and momentum of a fresh
// start (the start's forward product reads X[ix_cur], so ix_cur must name X[0]).
SolverState restart_state(SolverState h) {
  h.done = 0;
  h.kkt_hit = 0;
  h.ix_cur = 0;
  h.ix_prev = 0;
  h.ix_new = 1;
  h.t = 1.0;
  h.beta = 0.0;
  h.sel_acc = 0;
  return h;
}

// f and (optionally) the gradient of the FP64 iterate already in I.w64.X[0], with the
// KKT residual and the Frank-Wolfe gap of that iterate (host outputs, nullable).
double eval_fp64(pdt_problem_s* pb, Instance& I, bool grad, double* kkt_out, double* fw_out = nullptr) {
  hipStream_t s = pb->stream;
  const ProbView pv = view_var(I, VAR_FP64);
  Bufs<double> b = bufs_of(I, I.w64, nullptr);
  init_state(s, I.st_eval, 0, 0.0, 0.0);
  HIPCHK(launch_fx<double>(pv, b, I.st_eval, FX_EVAL, s));
  HIPCHK(launch_decide(I.partials, fx_num_waves(pv), I.st_eval, nullptr, DEC_EVAL, s));
  if (grad || kkt_out || fw_out) {
    const int nmt = ftr_num_waves(pv);
    HIPCHK(launch_ftr<double>(pv, b, I.st_eval, FTR_GRAD, 0.0, s));
    HIPCHK(launch_reduce_sum(I.partials, nmt, I.scalar, s));
    HIPCHK(launch_reduce_sum(I.partials + nmt, nmt, I.scalar + 1, s));
  }
  SolverState h = read_state(s, I.st_eval);
  if (kkt_out || fw_out) {
    double sum[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(sum, I.scalar, sizeof(sum), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (kkt_out) *kkt_out = std::sqrt(sum[0] / ((double)I.M * (double)I.N));
    if (fw_out) *fw_out = sum[1];
  }
  return h.f_eval;
}

constexpr int64_t kGraphIters = 64;


template <typename TS, typename TC>
void enqueue_iters(const ProbView& pv, const Bufs<TS>& b, SolverState* st, double step, int64_t n, bool delta,
                   hipStream_t s) {
  const int nfx = fx_num_waves(pv);
  for (int64_t k = 0; k < n; ++k) {
    HIPCHK((launch_ftr<TS, TC>(pv, b, st, FTR_STEP, step, s)));
    HIPCHK((launch_fx<TS, TC>(pv, b, st, delta ? FX_DELTA : FX_ITER, s)));
    HIPCHK(launch_decide(b.partials, nfx, st, b.history, DEC_ITER, s, b.rpart, ftr_num_waves(pv)));
  }
}

// KKT test of the current iterate (every kGraphIters iterations when opts.kkt_tol > 0):
// its residual F X_cur - P, the gradient product at X_cur with the KKT and Frank-Wolfe
// partials, then DEC_KKT, which stops the solve once the residual is small enough.
// pvs is the view of the storage precision (the mixed path's gradient runs in FP64,
// after the chunk's exact resync).
template <typename TS>
void enqueue_kkt(const ProbView& pvs, const Bufs<TS>& b, SolverState* st, hipStream_t s) {
  HIPCHK(launch_resid_cur<TS>(b, st, (long long)pvs.D * pvs.Npad, s));
  HIPCHK((launch_ftr<TS, TS>(pvs, b, st, FTR_GRAD, 0.0, s)));
  HIPCHK(launch_decide(b.partials, ftr_num_waves(pvs), st, nullptr, DEC_KKT, s));
}

// End of a chunk of the mixed path: exact products of X_prev and X_cur replace the
// FP32-updated ones, with both residual candidates and f_cur formed from them.
template <typename TS>
void enqueue_resync(const ProbView& pv64, const Bufs<TS>& b, SolverState* st, hipStream_t s) {
  HIPCHK((launch_fx<TS, TS>(pv64, b, st, FX_EVAL_PREV, s)));
  HIPCHK((launch_fx<TS, TS>(pv64, b, st, FX_RESYNC, s)));
  HIPCHK(launch_decide(b.partials, fx_num_waves(pv64), st, nullptr, DEC_RESYNC, s));
}

void drop_graphs(Instance& I) {
  for (int v = 0; v < 3; ++v) {
    if (I.graph[v]) (void)hipGraphExecDestroy(I.graph[v]);
    I.graph[v] = nullptr;
  }
  for (auto& row : I.nw.cg_graph)
    for (hipGraphExec_t& g : row) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// One graph = kGraphIters iterations of a variant.  The mixed variant forms F X_new by
// the FP32 delta F (X_new - X_cur) on FP64 storage, so it ends with exact FP64 forward
// products of the previous and current iterates and the exact objective, which remove
// the drift of those updates.
template <typename TS, typename TC>
hipGraphExec_t get_graph(pdt_problem_s* pb, Instance& I, int var, const Bufs<TS>& b, double step, bool kkt) {
  if (I.graph[var] && I.graph_step[var] == step && I.graph_hist[var] == b.history && I.graph_w[var] == b.wrow &&
      I.graph_kkt[var] == kkt && I.graph_rp[var] == b.rpart)
    return I.graph[var];
  if (I.graph[var]) (void)hipGraphExecDestroy(I.graph[var]);
  I.graph[var] = nullptr;
  // recorded on the library's own stream (the caller's may be the legacy default
  // stream, which cannot be captured); replayed on the caller's stream
  if (!pb->capture) HIPCHK(hipStreamCreateWithFlags(&pb->capture, hipStreamNonBlocking));
  hipStream_t cs = pb->capture;
  const ProbView pv = view_var(I, var);
  const ProbView pv64 = view_var(I, VAR_FP64);
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  try {
    enqueue_iters<TS, TC>(pv, b, I.st, step, kGraphIters, var == VAR_MIXED, cs);
    if (var == VAR_MIXED) enqueue_resync<TS>(pv64, b, I.st, cs);
    if (kkt) enqueue_kkt<TS>(var == VAR_MIXED ? pv64 : pv, b, I.st, cs);
  } catch (...) {
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPCHK(hipStreamEndCapture(cs, &g));
  hipGraphExec_t ge = nullptr;
  hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e);
  I.graph[var] = ge;
  I.graph_step[var] = step;
  I.graph_hist[var] = b.history;
  I.graph_w[var] = b.wrow;
  I.graph_kkt[var] = kkt;
  I.graph_rp[var] = b.rpart;
  return ge;
}

// Runs iterations of one variant from the current device state until it reports done,
// its iterations run out, or (stall > 0) a chunk lowers f by less than stall relative.
// With kkt, every chunk ends with the KKT test.  Returns the state read after the last
// chunk.
template <typename TS, typename TC>
SolverState run_chunks(pdt_problem_s* pb, Instance& I, int var, const Bufs<TS>& b, double step, double stall,
                       bool kkt) {
  hipStream_t s = pb->stream;
  const ProbView pv = view_var(I, var);
  const ProbView pv64 = view_var(I, VAR_FP64);
  SolverState h = read_state(s, I.st);
  while (!h.done && h.iter < h.max_iters) {
    const double f0 = h.f_cur;
    const int64_t left = h.max_iters - h.iter;
    if (left >= kGraphIters) {
      HIPCHK(hipGraphLaunch(get_graph<TS, TC>(pb, I, var, b, step, kkt), s));
    } else {
      enqueue_iters<TS, TC>(pv, b, I.st, step, left, var == VAR_MIXED, s);
      if (var == VAR_MIXED) enqueue_resync<TS>(pv64, b, I.st, s);
      if (kkt) enqueue_kkt<TS>(var == VAR_MIXED ? pv64 : pv, b, I.st, s);
    }
    h = read_state(s, I.st);
    if (stall > 0 && f0 - h.f_cur <= stall * h.f_cur) break;
  }
  return h;
}

// Starts a solve (or a refinement) from X[0] of the storage precision: exact products,
// f, fresh momentum and the KKT test of the start; iterations carry on from the state.
template <typename T>
void start_from_x0(pdt_problem_s* pb, Instance& I, const Bufs<T>& b, int var, bool kkt) {
  hipStream_t s = pb->stream;
  const ProbView pv = view_var(I, var);
  HIPCHK(launch_fx<T>(pv, b, I.st, FX_INIT, s));
  HIPCHK(launch_decide(I.partials, fx_num_waves(pv), I.st, nullptr, DEC_INIT, s));
  if (kkt) enqueue_kkt<T>(pv, b, I.st, s);
}

// Stall thresholds per 64-iteration chunk: FP32 products on FP64 iterates resolve the
// objective to ~1e-10 relative after each exact resync; FP32 iterates cannot take steps
// below their own rounding, which shows as progress under ~1e-6 relative.
constexpr double kStallMixed = 1e-10;
constexpr double kStallFp32 = 1e-6;

// Mixed path: FP32 products on FP64 iterates until progress stalls, then the FP64
// refinement continues from the same state to the requested tolerance.  A stop raised
// during the FP32-product phase by the objective test compared values built from FP32
// updates; it is provisional until an exact resync confirms it.
void run_mixed(pdt_problem_s* pb, Instance& I, const pdt_solve_opts& o, double step, const double* wrow,
               SolverState& out, int64_t& refine_iters) {
  hipStream_t s = pb->stream;
  const bool kkt = o.kkt_tol > 0;
  if (!I.w64.dX) {
    const size_t xm = (size_t)I.M * I.Npad, od = (size_t)I.D * I.Npad;
    I.w64.dX = pb->arena.alloc<float>(xm);
    I.w64.R32_acc = pb->arena.alloc<float>(od);
    I.w64.R32_rej = pb->arena.alloc<float>(od);
    HIPCHK(hipMemsetAsync(I.w64.dX, 0, xm * sizeof(float), s));
  }
  Bufs<double> b = bufs_of(I, I.w64, o.history, wrow, true, o.restart);
  start_from_x0<double>(pb, I, b, VAR_FP64, kkt);
  SolverState h = run_chunks<double, float>(pb, I, VAR_MIXED, b, step, kStallMixed, kkt);
  const int64_t mixed_iters = h.iter;
  if (h.done && !h.kkt_hit && h.iter < h.max_iters) {
    // the objective test held on FP32-updated products: redo it on exact ones
    h.done = 0;
    write_state(s, I.st, h);
    enqueue_resync<double>(view_var(I, VAR_FP64), b, I.st, s);
    h = read_state(s, I.st);
  }
  // the refinement's FP64 launches need no FP32 residual copies
  if (!h.done && !o.skip_refine)
    h = run_chunks<double, double>(pb, I, VAR_FP64, bufs_of(I, I.w64, o.history, wrow, false, o.restart), step,
                                   0.0, kkt);
  refine_iters = h.iter - mixed_iters;
  out = h;
}

// FP32 path: FP32 iterates and products until progress stalls (or a test holds on FP32
// values); then, unless skip_refine, the iterate is promoted to FP64 and the FP64 method
// continues from it with fresh momentum.  The promoted iterate is left in X64[0] either way.
void run_fp32(pdt_problem_s* pb, Instance& I, const pdt_solve_opts& o, double step, const double* wrow,
              SolverState& out, int64_t& refine_iters) {
  hipStream_t s = pb->stream;
  Arena& A = pb->arena;
  const size_t Np = (size_t)I.Npad, M = (size_t)I.M;
  const bool kkt = o.kkt_tol > 0;
  if (!I.P32) {
    I.P32 = A.alloc<float>((size_t)I.D * Np);
    HIPCHK(launch_convert_pad<double, float>(I.P64, I.P32, (long long)I.D, (int)Np, (int)Np, (int)Np, s));
  }
  ensure_work<float>(A, I, I.w32, I.P32);
  HIPCHK(launch_convert_pad<double, float>(I.w64.X[0], I.w32.X[0], (long long)M, (int)Np, (int)Np, (int)Np, s));
  Bufs<float> b32 = bufs_of(I, I.w32, o.history, wrow, false, o.restart);
  start_from_x0<float>(pb, I, b32, VAR_FP32, kkt);
  SolverState h = run_chunks<float, float>(pb, I, VAR_FP32, b32, step, o.skip_refine ? 0.0 : kStallFp32, kkt);
  HIPCHK(launch_convert_pad<float, double>(I.w32.X[h.ix_cur], I.w64.X[0], (long long)M, (int)Np, (int)Np, (int)Np,
                                           s));
  const int64_t fp32_iters = h.iter;
  if (!o.skip_refine && h.iter < h.max_iters) {
    // FP32 rows sum to 1 only to FP32 rounding; the FP64 method starts on the constraint
    // set (an infeasible start can undercut every feasible step's objective and stall)
    HIPCHK(launch_project_rows<double>(I.w64.X[0], I.w64.X[0], (long long)M, (int)I.N, (int)Np, (int)Np, s));
    // every FP32-phase stop is provisional: the FP64 start re-tests it on exact values
    write_state(s, I.st, restart_state(h));
    Bufs<double> b64 = bufs_of(I, I.w64, o.history, wrow, false, o.restart);
    start_from_x0<double>(pb, I, b64, VAR_FP64, kkt);
    h = run_chunks<double, double>(pb, I, VAR_FP64, b64, step, 0.0, kkt);
    if (h.ix_cur != 0)
      HIPCHK(hipMemcpyAsync(I.w64.X[0], I.w64.X[h.ix_cur], M * Np * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  refine_iters = h.iter - fp32_iters;
  out = h;
}

// ---------------------------------------------------------------------------------------
// Two-stage two-metric projected truncated Newton method (App. B, Algorithms 1-3).
// Host-driven: the host reads one scalar record per binding-set tolerance, slope and
// line-search trial; the CG iterations run back to back on the device, each queued
// before the completion flag of the previous one has been read.
// ---------------------------------------------------------------------------------------
constexpr double kNtBeta = 0.75;     // Armijo backtracking factor
constexpr double kNtArmijo = 0.1;    // Armijo constant c
constexpr int kNtMaxTrials = 60;     // beta^60 ~ 3e-8

NewtonWork& ensure_newton(pdt_problem_s* pb, Instance& I) {
  NewtonWork& nw = I.nw;
  if (nw.ready) return nw;
  Arena& A = pb->arena;
  hipStream_t s = pb->stream;
  const size_t xm = (size_t)I.M * I.Npad, od = (size_t)I.D * I.Npad;
  nw.Dir = A.alloc<double>(xm);
  nw.res = A.alloc<double>(xm);
  nw.z = A.alloc<double>(xm);
  nw.p = A.alloc<double>(xm);
  nw.q = A.alloc<double>(xm);
  nw.Vf = A.alloc<double>(xm);
  nw.Gh = A.alloc<double>(xm);
  nw.G = A.alloc<double>(xm);
  nw.Oh = A.alloc<double>(od);
  nw.Rh = A.alloc<double>(od);
  nw.Pz = A.alloc<double>(od);
  nw.Rg = A.alloc<double>(od);
  nw.part = A.alloc<double>(4 * kNtBlocks);
  nw.bpart = A.alloc<double>((size_t)I.n_partials);
  nw.mask = A.alloc<uint8_t>(xm);
  nw.mi = A.alloc<int>((size_t)I.M);
  nw.ns = A.alloc<NewtonState>(1);
  nw.st = A.alloc<SolverState>(1);
  HIPCHK(hipMemsetAsync(nw.Pz, 0, od * sizeof(double), s));
  HIPCHK(hipMemsetAsync(nw.mi, 0, (size_t)I.M * sizeof(int), s));
  HIPCHK(hipMemsetAsync(nw.ns, 0, sizeof(NewtonState), s));
  init_state(s, nw.st, 0, 0.0, 0.0);
  if (!nw.flag_h) {
    HIPCHK(hipHostMalloc((void**)&nw.flag_h, 2 * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
    nw.flag_h[0] = nw.flag_h[1] = 0;
    HIPCHK(hipHostGetDevicePointer((void**)&nw.flag_d, nw.flag_h, 0));
  }
  for (hipEvent_t& e : nw.ev)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  nw.ready = true;
  return nw;
}

// Band-kernel view of one array as the current iterate of a plain evaluation.
Bufs<double> nt_bufs(const Instance& I, const NewtonWork& nw, const double* X, double* O, const double* P, double* R,
                     double* G, const int* skip = nullptr) {
  Bufs<double> b;
  for (int k = 0; k < 3; ++k) {
    b.X[k] = const_cast<double*>(X);
    b.O[k] = O;
  }
  b.P = P;
  b.R_acc = R;
  b.R_rej = R;
  b.G = G;
  b.partials = nw.bpart;
  b.n_partials = I.n_partials;
  b.history = nullptr;
  b.fx_part = I.fx_part;
  b.fx_count = I.fx_count;
  b.ftr_part = I.ftr_part;
  b.skip = skip;
  return b;
}

// HV = 2 F^T (F V) + 2 gamma L V: forward product against zero data, then the transposed
// product's gradient mode on the result.  skip (may be null): both launches return at
// once while *skip != 0.
void nt_hessian(const ProbView& pv, const Instance& I, NewtonWork& nw, const double* V, double* HV, const int* skip,
                hipStream_t s) {
  const Bufs<double> b = nt_bufs(I, nw, V, nw.Oh, nw.Pz, nw.Rh, HV, skip);
  HIPCHK(launch_fx<double>(pv, b, nw.st, FX_EVAL, s));
  HIPCHK(launch_ftr<double>(pv, b, nw.st, FTR_GRAD, 0.0, s));
}

// f(X) into nw.st->f_eval and F X - P into nw.Rg (queued, not waited for)
void nt_eval(const ProbView& pv, const Instance& I, NewtonWork& nw, const double* X, hipStream_t s) {
  const Bufs<double> b = nt_bufs(I, nw, X, I.w64.O[0], I.P64, nw.Rg, nw.G);
  HIPCHK(launch_fx<double>(pv, b, nw.st, FX_EVAL, s));
  HIPCHK(launch_decide(nw.bpart, fx_num_waves(pv), nw.st, nullptr, DEC_EVAL, s));
}

// gradient at X into nw.G from the residual F X - P left in nw.Rg by nt_eval(X)
void nt_gradient(const ProbView& pv, const Instance& I, NewtonWork& nw, const double* X, hipStream_t s) {
  const Bufs<double> b = nt_bufs(I, nw, X, I.w64.O[0], I.P64, nw.Rg, nw.G);
  HIPCHK(launch_ftr<double>(pv, b, nw.st, FTR_GRAD, 0.0, s));
}

NewtonState nt_read(hipStream_t s, const NewtonWork& nw, double* f_eval = nullptr) {
  NewtonState h;
  HIPCHK(hipMemcpyAsync(&h, nw.ns, sizeof(h), hipMemcpyDeviceToHost, s));
  SolverState st;
  if (f_eval) HIPCHK(hipMemcpyAsync(&st, nw.st, sizeof(st), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (f_eval) *f_eval = st.f_eval;
  return h;
}

// One CG iteration of parity par: the Hessian product of the free part of p (skipped
// once the solve has stopped) and the three row kernels; the direction kernel reports
// the completion state to flag slot `slot`.
void enqueue_cg_iter(const ProbView& pv, const Instance& I, NewtonWork& nw, const NtRows& rows, int par, int slot,
                     hipStream_t s) {
  nt_hessian(pv, I, nw, nw.Vf, nw.Gh, &nw.ns->cg_done, s);
  HIPCHK(launch_nt_q(rows, nw.mask, nw.mi, I.hdiag, nw.p, nw.Gh, nw.q, nw.part, nw.ns, s));
  HIPCHK(launch_nt_update(rows, nw.mask, I.hdiag, nw.Dir, nw.res, nw.z, nw.p, nw.q, nw.part, nw.ns, par, s));
  HIPCHK(launch_nt_dir(rows, nw.mask, nw.mi, nw.z, nw.p, nw.Vf, nw.part, nw.ns, par, nw.flag_d + slot, s));
}

constexpr int kCgGraphIters = 4;  // CG iterations per captured launch (even: parities repeat)

// kCgGraphIters CG iterations of one stage reporting to one flag slot, recorded once per
// problem on the library's capture stream (dropped with the other graphs when the
// kernel grid changes)
hipGraphExec_t cg_graph(pdt_problem_s* pb, const ProbView& pv, const Instance& I, NewtonWork& nw,
                        const NtRows& rows, int slot) {
  hipGraphExec_t& ge = nw.cg_graph[rows.stage - 1][slot];
  if (ge) return ge;
  if (!pb->capture) HIPCHK(hipStreamCreateWithFlags(&pb->capture, hipStreamNonBlocking));
  hipStream_t cs = pb->capture;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  try {
    for (int j = 0; j < kCgGraphIters; ++j) enqueue_cg_iter(pv, I, nw, rows, j & 1, slot, cs);
  } catch (...) {
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPCHK(hipStreamEndCapture(cs, &g));
  hipGraphExec_t e_out = nullptr;
  const hipError_t e = hipGraphInstantiate(&e_out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e);
  ge = e_out;
  return ge;
}

// Direction of one Newton step at X (gradient in nw.G): codes, CG solve, result in
// nw.Dir (and the row maxima in nw.mi for stage 2).  Returns the CG iterations.  The
// iterations go out kCgGraphIters per graph launch (the last < kCgGraphIters one by
// one); the host reads the completion flag of the previous launch only, so the device
// always has the next one queued, and launches queued after the solve stopped return at
// once on the device flag.
int nt_direction(pdt_problem_s* pb, const ProbView& pv, const Instance& I, NewtonWork& nw, const NtRows& rows,
                 const double* X, double eps, double rtol, int cg_max, hipStream_t s) {
  HIPCHK(launch_nt_prep(rows, X, nw.G, I.hdiag, eps, nw.mask, nw.mi, nw.res, nw.z, nw.p, nw.Vf, nw.Dir, nw.part,
                        nw.ns, rtol, cg_max, s));
  int it = 0;
  for (int k = 0; it < cg_max; ++k) {
    const int slot = k & 1;
    if (cg_max - it >= kCgGraphIters) {
      HIPCHK(hipGraphLaunch(cg_graph(pb, pv, I, nw, rows, slot), s));
      it += kCgGraphIters;
    } else {
      for (; it < cg_max; ++it) enqueue_cg_iter(pv, I, nw, rows, it & 1, slot, s);
    }
    HIPCHK(hipEventRecord(nw.ev[slot], s));
    if (k >= 1) {
      HIPCHK(hipEventSynchronize(nw.ev[slot ^ 1]));
      if (nw.flag_h[slot ^ 1]) break;
    }
  }
  return nt_read(s, nw).cg_iter;
}

double nt_slope(const Instance& I, NewtonWork& nw, const NtRows& rows, const double* X, hipStream_t s) {
  HIPCHK(launch_nt_slope(rows, X, nw.Dir, nw.G, nw.mi, nw.part, nw.ns, s));
  (void)I;
  return nt_read(s, nw).out[0];
}

struct NewtonRun {
  int64_t n1 = 0, n2 = 0, cg = 0, trials = 0;
  double f = 0.0, kkt = 0.0;
  bool converged = false;
  std::vector<double> hist;
};

// Runs the method from the iterate in I.w64.X[0]; leaves the result there.
void newton_run(pdt_problem_s* pb, Instance& I, const pdt_newton_opts& o, NewtonRun& out) {
  hipStream_t s = pb->stream;
  const ProbView pv = view_var(I, VAR_FP64);
  NewtonWork& nw = ensure_newton(pb, I);
  double* X = I.w64.X[0];
  double* Xa = I.w64.X[1];
  const double mn = (double)I.M * (double)I.N;
  NtRows rows{(int)I.M, (int)I.N, (int)I.Npad, 1};
  double f = 0.0;
  nt_eval(pv, I, nw, X, s);
  (void)nt_read(s, nw, &f);
  out.hist.push_back(f);
  int stage = o.stage2_only ? 2 : 1;
  bool resid_ok = true;  // nw.Rg holds F X - P of the current X
  double kkt = 0.0;
  bool kkt_fresh = false;
  for (int64_t k = 0; k < o.max_newton; ++k) {
    if (!resid_ok) {
      nt_eval(pv, I, nw, X, s);
      resid_ok = true;
    }
    nt_gradient(pv, I, nw, X, s);
    rows.stage = stage;
    HIPCHK(launch_nt_measure(rows, X, nw.G, nw.part, nw.ns, s));
    NewtonState m = nt_read(s, nw);
    kkt = std::sqrt(m.out[0] / mn);
    kkt_fresh = true;
    if (stage == 2 && kkt <= o.eps_kkt) {
      out.converged = true;
      break;
    }
    const double eps = std::min(o.eps_cap > 0.0 ? o.eps_cap : 1e-9, std::sqrt(m.out[1]));
    out.cg += nt_direction(pb, pv, I, nw, rows, X, eps, o.cg_rtol, o.cg_max, s);
    double slope = nt_slope(I, nw, rows, X, s);
    if (slope >= 0.0) {
      HIPCHK(launch_nt_negrad(rows, nw.G, nw.mi, nw.Dir, s));
      slope = nt_slope(I, nw, rows, X, s);
    }
    if (stage == 1 && std::fabs(slope) <= o.stage_switch) {
      stage = 2;
      continue;
    }
    if (stage == 2 && slope == 0.0) break;
    if (stage == 1) ++out.n1;
    else ++out.n2;
    double a = 1.0;
    bool accepted = false;
    for (int t = 0; t < kNtMaxTrials; ++t) {
      HIPCHK(launch_nt_trial(rows, X, nw.Dir, nw.mi, a, Xa, nw.part, nw.ns, s));
      nt_eval(pv, I, nw, Xa, s);
      double fa = 0.0;
      const NewtonState tr = nt_read(s, nw, &fa);
      ++out.trials;
      const bool ok = stage == 1 || tr.out[1] == 0.0;
      if (ok && fa <= f + kNtArmijo * a * slope) {
        std::swap(X, Xa);
        f = fa;
        accepted = true;
        break;
      }
      a *= kNtBeta;
    }
    resid_ok = accepted;
    kkt_fresh = false;
    out.hist.push_back(f);
    if (accepted && o.f_star > 0.0 && f - o.f_star <= o.rel_obj_tol * o.f_star) {
      out.converged = true;
      break;
    }
    if (!accepted) {
      if (stage == 1) stage = 2;
      else break;
    }
  }
  if (!kkt_fresh) {
    if (!resid_ok) nt_eval(pv, I, nw, X, s);
    nt_gradient(pv, I, nw, X, s);
    rows.stage = 2;
    HIPCHK(launch_nt_measure(rows, X, nw.G, nw.part, nw.ns, s));
    kkt = std::sqrt(nt_read(s, nw).out[0] / mn);
    if (kkt <= o.eps_kkt) out.converged = true;
  }
  if (o.f_star > 0.0 && f - o.f_star <= o.rel_obj_tol * o.f_star) out.converged = true;
  if (X != I.w64.X[0])
    HIPCHK(hipMemcpyAsync(I.w64.X[0], X, (size_t)I.M * I.Npad * sizeof(double), hipMemcpyDeviceToDevice, s));
  out.f = f;
  out.kkt = kkt;
}

// copies a dense device [M][N] array into a padded device [M][Npad] one (zero pad)
void to_padded(const Instance& I, const double* src, double* dst, hipStream_t s) {
  const size_t Np = (size_t)I.Npad, N = (size_t)I.N;
  HIPCHK(hipMemsetAsync(dst, 0, (size_t)I.M * Np * sizeof(double), s));
  HIPCHK(hipMemcpy2DAsync(dst, Np * sizeof(double), src, N * sizeof(double), N * sizeof(double), (size_t)I.M,
                          hipMemcpyDeviceToDevice, s));
}

void from_padded(const Instance& I, const double* src, double* dst, hipStream_t s) {
  const size_t Np = (size_t)I.Npad, N = (size_t)I.N;
  HIPCHK(hipMemcpy2DAsync(dst, N * sizeof(double), src, Np * sizeof(double), N * sizeof(double), (size_t)I.M,
                          hipMemcpyDeviceToDevice, s));
}

}  // namespace

namespace {
template <typename T, typename TC = T>
void replay_impl(pdt_problem_s* pb, Instance& I, int kernel, int64_t reps) {
  hipStream_t s = pb->stream;
  const int var = std::is_same<T, float>::value ? VAR_FP32 : (std::is_same<T, TC>::value ? VAR_FP64 : VAR_MIXED);
  const ProbView pv = view_var(I, var);
  Bufs<T> b = bufs_of(I, work_of<T>(I), nullptr, nullptr, var == VAR_MIXED);
  SolverState s0;
  std::memset(&s0, 0, sizeof(s0));
  s0.ix_cur = 0;
  s0.ix_prev = 2;
  s0.ix_new = 1;
  s0.t = 3.0;
  s0.beta = 0.5;
  s0.sel_acc = 1;
  s0.f_cur = 1e300;
  s0.max_iters = LLONG_MAX;
  HIPCHK(hipMemcpyAsync(I.st_eval, &s0, sizeof(s0), hipMemcpyHostToDevice, s));
  const double step = 1.0 / I.L_hat;
  for (int64_t r = 0; r < reps; ++r) {
    const int fxmode = std::is_same<T, TC>::value ? FX_ITER : FX_DELTA;  // the mixed kernel is delta-only
    if (kernel == 0 || kernel == 3) HIPCHK((launch_ftr<T, TC>(pv, b, I.st_eval, FTR_STEP, step, s)));
    if (kernel == 1 || kernel == 3) HIPCHK((launch_fx<T, TC>(pv, b, I.st_eval, fxmode, s)));
    if (kernel == 2 || kernel == 3)
      HIPCHK(launch_decide(I.partials, fx_num_waves(pv), I.st_eval, nullptr, DEC_ITER, s));
  }
}

}  // namespace

namespace {
int learned_start(pdt_problem_s* pb, Instance& I, pdt_model_s* md);
}

extern "C" {

const char* pdt_last_error(void) { return g_last_error.c_str(); }

pdt_status pdt_make_problem(const pdt_problem_desc* descs, int64_t n_instances, void* stream,
                            pdt_problem_t* out) {
  if (!out) return set_err(PDT_ERR_INVALID_ARG, "out must not be NULL");
  *out = nullptr;
  if (!descs) return set_err(PDT_ERR_INVALID_ARG, "descs must not be NULL");
  if (n_instances < 1 || n_instances > 65536) return set_err(PDT_ERR_INVALID_ARG, "n_instances must be in [1, 65536]");
  pdt_problem_s* pb = nullptr;
  try {
    for (int64_t k = 0; k < n_instances; ++k) validate_desc(descs[k]);
    pb = new pdt_problem_s();
    pb->stream = static_cast<hipStream_t>(stream);
    HIPCHK(hipGetDevice(&pb->device));
    pb->inst.resize((size_t)n_instances);
    for (int64_t k = 0; k < n_instances; ++k) setup_instance(pb, pb->inst[(size_t)k], descs[k]);
    *out = pb;
    g_last_error.clear();
    return PDT_OK;
  } catch (...) {
    if (pb) {
      (void)hipStreamSynchronize(pb->stream);
      pb->arena.release();
      delete pb;
    }
    return status_of_current_exception();
  }
}

void pdt_destroy_problem(pdt_problem_t problem) {
  if (!problem) return;
  (void)hipStreamSynchronize(problem->stream);
  for (Instance& I : problem->inst) {
    drop_graphs(I);
    for (hipEvent_t& e : I.nw.ev)
      if (e) (void)hipEventDestroy(e);
    if (I.nw.flag_h) (void)hipHostFree(I.nw.flag_h);
  }
  for (int k = 0; k < 2; ++k) {
    if (problem->plan[k].graph) (void)hipGraphExecDestroy(problem->plan[k].graph);
    problem->plan_arena[k].release();
  }
  if (problem->capture) (void)hipStreamDestroy(problem->capture);
  problem->arena.release();
  delete problem;
}

pdt_status pdt_problem_bands(pdt_problem_t pb, int32_t* lo, int32_t* hi, double* tail, double* lipschitz,
                             int64_t* nnz) {
  if (!pb) return set_err(PDT_ERR_INVALID_ARG, "problem is NULL");
  const Instance& I = pb->inst[0];
  if (lo) std::memcpy(lo, I.lo_h.data(), I.lo_h.size() * sizeof(int32_t));
  if (hi) std::memcpy(hi, I.hi_h.data(), I.hi_h.size() * sizeof(int32_t));
  if (tail) std::memcpy(tail, I.tail_h.data(), I.tail_h.size() * sizeof(double));
  if (lipschitz) *lipschitz = I.L_hat;
  if (nnz) *nnz = I.nnz;
  return PDT_OK;
}

pdt_status pdt_problem_set_tiles(pdt_problem_t pb, int64_t instance, int precision, int ks_fx, int ks_ftr) {
  if (!pb) return set_err(PDT_ERR_INVALID_ARG, "problem is NULL");
  if (instance < 0 || instance >= (int64_t)pb->inst.size()) return set_err(PDT_ERR_INVALID_ARG, "bad instance");
  if (precision != PDT_FP64 && precision != PDT_FP32 && precision != PDT_MIXED)
    return set_err(PDT_ERR_INVALID_ARG, "precision not supported");
  auto ok = [](int k) { return k == 0 || k == 4 || k == 8; };
  if (!ok(ks_fx) || !ok(ks_ftr)) return set_err(PDT_ERR_INVALID_ARG, "waves per workgroup must be 0, 4 or 8");
  try {
    (void)hipStreamSynchronize(pb->stream);
    Instance& I = pb->inst[(size_t)instance];
    I.ks_force[precision][0] = ks_fx;
    I.ks_force[precision][1] = ks_ftr;
    drop_graphs(I);
    for (BatchPlan& P : pb->plan) {
      if (P.graph) (void)hipGraphExecDestroy(P.graph);
      P.graph = nullptr;
      P.prec = -1;
    }
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_problem_set_fx_split(pdt_problem_t pb, int64_t instance, int split) {
  if (!pb) return set_err(PDT_ERR_INVALID_ARG, "problem is NULL");
  if (instance < 0 || instance >= (int64_t)pb->inst.size()) return set_err(PDT_ERR_INVALID_ARG, "bad instance");
  if (split < 0 || split > kMaxFxSplit) return set_err(PDT_ERR_INVALID_ARG, "split must be in [0, 16]");
  try {
    Instance& I = pb->inst[(size_t)instance];
    HIPCHK(hipStreamSynchronize(pb->stream));
    drop_graphs(I);  // captured launches carry the old grid
    set_fx_split(pb->arena, I, split == 0 ? I.fx_split_auto : split);
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_problem_fx_split(pdt_problem_t pb, int64_t instance, int* split) {
  if (!pb || !split) return set_err(PDT_ERR_INVALID_ARG, "problem and split must not be NULL");
  if (instance < 0 || instance >= (int64_t)pb->inst.size()) return set_err(PDT_ERR_INVALID_ARG, "bad instance");
  *split = pb->inst[(size_t)instance].fx_split;
  return PDT_OK;
}

pdt_status pdt_problem_set_ftr_split(pdt_problem_t pb, int64_t instance, int split) {
  if (!pb) return set_err(PDT_ERR_INVALID_ARG, "problem is NULL");
  if (instance < 0 || instance >= (int64_t)pb->inst.size()) return set_err(PDT_ERR_INVALID_ARG, "bad instance");
  if (split < 0 || split > kMaxFtrSplit) return set_err(PDT_ERR_INVALID_ARG, "split must be in [0, 16]");
  try {
    Instance& I = pb->inst[(size_t)instance];
    HIPCHK(hipStreamSynchronize(pb->stream));
    drop_graphs(I);  // captured launches carry the old grid
    set_ftr_split(pb->arena, I, split == 0 ? I.ftr_split_auto : split);
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_problem_ftr_split(pdt_problem_t pb, int64_t instance, int* split) {
  if (!pb || !split) return set_err(PDT_ERR_INVALID_ARG, "problem and split must not be NULL");
  if (instance < 0 || instance >= (int64_t)pb->inst.size()) return set_err(PDT_ERR_INVALID_ARG, "bad instance");
  *split = pb->inst[(size_t)instance].ftr_split;
  return PDT_OK;
}

pdt_status pdt_problem_tiles(pdt_problem_t pb, int64_t instance, int precision, int* ks_fx, int* ks_ftr) {
  if (!pb) return set_err(PDT_ERR_INVALID_ARG, "problem is NULL");
  if (instance < 0 || instance >= (int64_t)pb->inst.size()) return set_err(PDT_ERR_INVALID_ARG, "bad instance");
  if (precision != PDT_FP64 && precision != PDT_FP32 && precision != PDT_MIXED)
    return set_err(PDT_ERR_INVALID_ARG, "precision not supported");
  const ProbView pv = view_var(pb->inst[(size_t)instance], precision);
  if (ks_fx) *ks_fx = pv.ks_fx;
  if (ks_ftr) *ks_ftr = pv.ks_ftr;
  return PDT_OK;
}

pdt_status pdt_problem_scaling(pdt_problem_t pb, double* hdiag, double* lipschitz_scaled) {
  if (!pb) return set_err(PDT_ERR_INVALID_ARG, "problem is NULL");
  try {
    Instance& I = pb->inst[0];
    if (hdiag) std::memcpy(hdiag, I.hdiag_h.data(), I.hdiag_h.size() * sizeof(double));
    if (lipschitz_scaled) *lipschitz_scaled = scaled_lipschitz(pb, I);
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

static pdt_status objective_impl(pdt_problem_t pb, const double* Pi, double* f_out, double* grad_out,
                                 double* kkt_out) {
  if (!pb || !Pi) return set_err(PDT_ERR_INVALID_ARG, "problem and Pi must not be NULL");
  try {
    Instance& I = pb->inst[0];
    hipStream_t s = pb->stream;
    ensure_work<double>(pb->arena, I, I.w64, I.P64);
    const size_t Np = (size_t)I.Npad, N = (size_t)I.N;
    HIPCHK(hipMemsetAsync(I.w64.X[0], 0, (size_t)I.M * Np * sizeof(double), s));
    HIPCHK(hipMemcpy2DAsync(I.w64.X[0], Np * sizeof(double), Pi, N * sizeof(double), N * sizeof(double),
                            (size_t)I.M, hipMemcpyDeviceToDevice, s));
    const double f = eval_fp64(pb, I, grad_out != nullptr, kkt_out);
    if (f_out) *f_out = f;
    if (grad_out) {
      HIPCHK(hipMemcpy2DAsync(grad_out, N * sizeof(double), I.w64.G, Np * sizeof(double), N * sizeof(double),
                              (size_t)I.M, hipMemcpyDeviceToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    return std::isfinite(f) ? PDT_OK : set_err(PDT_ERR_NUMERIC, "objective is not finite");
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_objective(pdt_problem_t pb, const double* Pi, double* f_out, double* grad_out) {
  return objective_impl(pb, Pi, f_out, grad_out, nullptr);
}

pdt_status pdt_kkt(pdt_problem_t pb, const double* Pi, double* kkt_out) {
  if (!kkt_out) return set_err(PDT_ERR_INVALID_ARG, "kkt_out must not be NULL");
  return objective_impl(pb, Pi, nullptr, nullptr, kkt_out);
}

pdt_status pdt_newton_solve(pdt_problem_t pb, double* Pi, const pdt_newton_opts* opts, pdt_newton_info* info) {
  if (!pb || !Pi || !opts) return set_err(PDT_ERR_INVALID_ARG, "problem, Pi and opts must not be NULL");
  const pdt_newton_opts o = *opts;
  if (o.max_newton < 0) return set_err(PDT_ERR_INVALID_ARG, "max_newton must be >= 0");
  if (!std::isfinite(o.eps_kkt) || o.eps_kkt < 0 || !std::isfinite(o.stage_switch) || o.stage_switch < 0 ||
      !std::isfinite(o.cg_rtol) || o.cg_rtol < 0)
    return set_err(PDT_ERR_INVALID_ARG, "eps_kkt, stage_switch and cg_rtol must be finite and >= 0");
  if (o.cg_max < 1) return set_err(PDT_ERR_INVALID_ARG, "cg_max must be >= 1");
  if (o.init != PDT_INIT_UNIFORM && o.init != PDT_INIT_USER)
    return set_err(PDT_ERR_INVALID_ARG, "init must be PDT_INIT_UNIFORM or PDT_INIT_USER");
  if (o.stage2_only != 0 && o.stage2_only != 1) return set_err(PDT_ERR_INVALID_ARG, "stage2_only must be 0 or 1");
  if (!std::isfinite(o.f_star) || !std::isfinite(o.rel_obj_tol) || o.rel_obj_tol < 0)
    return set_err(PDT_ERR_INVALID_ARG, "bad objective tolerance");
  if (!std::isfinite(o.eps_cap) || o.eps_cap < 0) return set_err(PDT_ERR_INVALID_ARG, "eps_cap must be >= 0");
  const auto t0 = std::chrono::steady_clock::now();
  try {
    Instance& I = pb->inst[0];
    hipStream_t s = pb->stream;
    ensure_work<double>(pb->arena, I, I.w64, I.P64);
    const size_t Np = (size_t)I.Npad, N = (size_t)I.N, M = (size_t)I.M;
    if (o.init == PDT_INIT_USER)
      HIPCHK(launch_project_rows<double>(Pi, I.w64.X[0], (long long)M, (int)N, (int)N, (int)Np, s));
    else
      HIPCHK(launch_fill_rows<double>(I.w64.X[0], (long long)M, (int)N, (int)Np, 1.0 / (double)N, s));
    NewtonRun r;
    newton_run(pb, I, o, r);
    from_padded(I, I.w64.X[0], Pi, s);
    HIPCHK(hipStreamSynchronize(s));
    if (o.history) std::memcpy(o.history, r.hist.data(), r.hist.size() * sizeof(double));
    if (info) {
      info->stage1_iters = r.n1;
      info->stage2_iters = r.n2;
      info->cg_iters = r.cg;
      info->line_trials = r.trials;
      info->objective = r.f;
      info->kkt = r.kkt;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      info->converged = r.converged ? 1 : 0;
    }
    if (!std::isfinite(r.f)) return set_err(PDT_ERR_NUMERIC, "objective is not finite");
    if (!r.converged) return set_err(PDT_ERR_NOT_CONVERGED, "stopped before the KKT or objective test held");
    g_last_error.clear();
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_hessian_apply(pdt_problem_t pb, const double* V, double* HV) {
  if (!pb || !V || !HV) return set_err(PDT_ERR_INVALID_ARG, "problem, V and HV must not be NULL");
  if (V == HV) return set_err(PDT_ERR_INVALID_ARG, "V and HV must be distinct");
  try {
    Instance& I = pb->inst[0];
    hipStream_t s = pb->stream;
    ensure_work<double>(pb->arena, I, I.w64, I.P64);
    NewtonWork& nw = ensure_newton(pb, I);
    const ProbView pv = view_var(I, VAR_FP64);
    to_padded(I, V, nw.Vf, s);
    nt_hessian(pv, I, nw, nw.Vf, nw.Gh, nullptr, s);
    from_padded(I, nw.Gh, HV, s);
    HIPCHK(hipStreamSynchronize(s));
    g_last_error.clear();
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_newton_direction(pdt_problem_t pb, int stage, const double* Pi, double eps, double cg_rtol,
                                int32_t cg_max, double* Dir, int32_t* row_max, int64_t* cg_iters, double* slope) {
  if (!pb || !Pi || !Dir) return set_err(PDT_ERR_INVALID_ARG, "problem, Pi and Dir must not be NULL");
  if (stage != 1 && stage != 2) return set_err(PDT_ERR_INVALID_ARG, "stage must be 1 or 2");
  if (!std::isfinite(eps) || eps < 0 || !std::isfinite(cg_rtol) || cg_rtol < 0)
    return set_err(PDT_ERR_INVALID_ARG, "eps and cg_rtol must be finite and >= 0");
  if (cg_max < 1) return set_err(PDT_ERR_INVALID_ARG, "cg_max must be >= 1");
  try {
    Instance& I = pb->inst[0];
    hipStream_t s = pb->stream;
    ensure_work<double>(pb->arena, I, I.w64, I.P64);
    NewtonWork& nw = ensure_newton(pb, I);
    const ProbView pv = view_var(I, VAR_FP64);
    double* X = I.w64.X[0];
    to_padded(I, Pi, X, s);
    nt_eval(pv, I, nw, X, s);
    nt_gradient(pv, I, nw, X, s);
    const NtRows rows{(int)I.M, (int)I.N, (int)I.Npad, stage};
    const int it = nt_direction(pb, pv, I, nw, rows, X, eps, cg_rtol, cg_max, s);
    const double sl = nt_slope(I, nw, rows, X, s);
    from_padded(I, nw.Dir, Dir, s);
    if (row_max && stage == 2)
      HIPCHK(hipMemcpyAsync(row_max, nw.mi, (size_t)I.M * sizeof(int), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (cg_iters) *cg_iters = it;
    if (slope) *slope = sl;
    g_last_error.clear();
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_solve(pdt_problem_t pb, double* Pi, const pdt_solve_opts* opts, pdt_solve_info* info) {
  if (!pb || !Pi || !opts) return set_err(PDT_ERR_INVALID_ARG, "problem, Pi and opts must not be NULL");
  const pdt_solve_opts o = *opts;
  if (o.max_iters < 0) return set_err(PDT_ERR_INVALID_ARG, "max_iters must be >= 0");
  if (!std::isfinite(o.step_L) || o.step_L < 0) return set_err(PDT_ERR_INVALID_ARG, "step_L must be >= 0");
  if (o.init != PDT_INIT_UNIFORM && o.init != PDT_INIT_USER && o.init != PDT_INIT_LEARNED)
    return set_err(PDT_ERR_INVALID_ARG, "bad init");
  if (o.precision != PDT_FP64 && o.precision != PDT_FP32 && o.precision != PDT_MIXED)
    return set_err(PDT_ERR_INVALID_ARG, "precision not supported");
  if (!std::isfinite(o.rel_obj_tol) || o.rel_obj_tol < 0 || !std::isfinite(o.f_star))
    return set_err(PDT_ERR_INVALID_ARG, "bad tolerance");
  if (!std::isfinite(o.kkt_tol) || o.kkt_tol < 0) return set_err(PDT_ERR_INVALID_ARG, "kkt_tol must be finite and >= 0");
  if (o.history_stride < 0) return set_err(PDT_ERR_INVALID_ARG, "history_stride must be >= 0");
  if (o.scaling != PDT_STEP_UNIFORM && o.scaling != PDT_STEP_DIAG) return set_err(PDT_ERR_INVALID_ARG, "bad scaling");
  if (o.restart != PDT_RESTART_FUNCTION && o.restart != PDT_RESTART_GRADIENT)
    return set_err(PDT_ERR_INVALID_ARG, "bad restart");
  const auto t0 = std::chrono::steady_clock::now();
  try {
    Instance& I = pb->inst[0];
    hipStream_t s = pb->stream;
    Arena& A = pb->arena;
    ensure_work<double>(A, I, I.w64, I.P64);
    const size_t Np = (size_t)I.Npad, N = (size_t)I.N, M = (size_t)I.M;
    const bool scaled = o.scaling == PDT_STEP_DIAG;
    const double L = o.step_L > 0 ? o.step_L : (scaled ? scaled_lipschitz(pb, I) : I.L_hat);
    const double step = 1.0 / L;
    const double* wrow = scaled ? I.wrow : nullptr;
    // starting point in X64[0]: 1/N, or the caller's Pi projected onto the constraints
    if (o.init == PDT_INIT_USER) {
      HIPCHK(launch_project_rows<double>(Pi, I.w64.X[0], (long long)M, (int)N, (int)N, (int)Np, s));
    } else if (o.init == PDT_INIT_LEARNED) {
      if (!o.model) return set_err(PDT_ERR_INVALID_ARG, "init = LEARNED needs a model");
    } else {
      HIPCHK(launch_fill_rows<double>(I.w64.X[0], (long long)M, (int)N, (int)Np, 1.0 / (double)N, s));
    }
    int fell_back = 0;
    if (o.init == PDT_INIT_LEARNED) fell_back = learned_start(pb, I, o.model);
    const double f_star = o.f_star > 0 ? o.f_star : 0.0;
    init_state(s, I.st, o.max_iters, f_star, o.rel_obj_tol, o.kkt_tol, (double)M * (double)N, o.history_stride);
    SolverState fin;
    int64_t refine_iters = 0;
    if (o.precision == PDT_FP64) {
      Bufs<double> b = bufs_of(I, I.w64, o.history, wrow, false, o.restart);
      start_from_x0<double>(pb, I, b, VAR_FP64, o.kkt_tol > 0);
      fin = run_chunks<double, double>(pb, I, VAR_FP64, b, step, 0.0, o.kkt_tol > 0);
    } else if (o.precision == PDT_MIXED) {
      run_mixed(pb, I, o, step, wrow, fin, refine_iters);
    } else {
      run_fp32(pb, I, o, step, wrow, fin, refine_iters);
    }
    if (o.precision != PDT_FP32 && fin.ix_cur != 0)
      HIPCHK(hipMemcpyAsync(I.w64.X[0], I.w64.X[fin.ix_cur], M * Np * sizeof(double), hipMemcpyDeviceToDevice, s));
    // the tests that decide convergence are re-evaluated in FP64 at the returned iterate
    double kkt = 0, fw = 0;
    const double f = eval_fp64(pb, I, true, &kkt, &fw);
    HIPCHK(hipMemcpy2DAsync(Pi, N * sizeof(double), I.w64.X[0], Np * sizeof(double), N * sizeof(double), M,
                            hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    const bool want_obj = f_star > 0 && o.rel_obj_tol > 0, want_kkt = o.kkt_tol > 0;
    const bool conv = (want_obj && f - f_star <= o.rel_obj_tol * f_star) || (want_kkt && kkt <= o.kkt_tol);
    pdt_status st = PDT_OK;
    if (!std::isfinite(f)) st = set_err(PDT_ERR_NUMERIC, "objective is not finite");
    else if ((want_obj || want_kkt) && !conv) st = set_err(PDT_ERR_NOT_CONVERGED, "max_iters reached before the tolerance");
    if (info) {
      info->iters = fin.iter;
      info->rejects = fin.rejects;
      info->objective = f;
      info->kkt = kkt;
      info->L_used = L;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      info->converged = conv ? 1 : 0;
      info->refine_iters = refine_iters;
      info->fell_back_to_cold = fell_back;
      info->fw_gap = fw;
      info->status = st;
    }
    if (st == PDT_OK) g_last_error.clear();
    return st;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_replay_kernel(pdt_problem_t pb, int kernel, int precision, int64_t reps) {
  if (!pb || kernel < 0 || kernel > 3 || reps < 0) return set_err(PDT_ERR_INVALID_ARG, "bad arguments");
  Instance& I = pb->inst[0];
  try {
    if (precision == PDT_FP64) {
      if (!I.w64.ready) return set_err(PDT_ERR_INVALID_ARG, "solve in FP64 once before replaying");
      replay_impl<double>(pb, I, kernel, reps);
    } else if (precision == PDT_FP32) {
      if (!I.w32.ready) return set_err(PDT_ERR_INVALID_ARG, "solve in FP32 once before replaying");
      replay_impl<float>(pb, I, kernel, reps);
    } else if (precision == PDT_MIXED) {
      if (!I.w64.ready || !I.w64.dX) return set_err(PDT_ERR_INVALID_ARG, "solve in mixed precision once before replaying");
      replay_impl<double, float>(pb, I, kernel, reps);
    } else {
      return set_err(PDT_ERR_INVALID_ARG, "precision not supported");
    }
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_smooth_rows(const double* Pi, double* out, int64_t M, int64_t N, int32_t divisor, int64_t skip,
                           void* stream) {
  if (!Pi || !out) return set_err(PDT_ERR_INVALID_ARG, "Pi and out must not be NULL");
  if (M < 1 || N < 1 || M * N > (int64_t)INT_MAX) return set_err(PDT_ERR_INVALID_ARG, "need M, N >= 1, M*N < 2^31");
  if (divisor < 1 || skip < 0) return set_err(PDT_ERR_INVALID_ARG, "need divisor >= 1, skip >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Arena tmp;
  try {
    double* scratch = tmp.alloc<double>((size_t)smooth_scratch_doubles((long long)M, (int)N));
    HIPCHK(launch_smooth_rows(Pi, out, (long long)M, (int)N, (int)divisor, (long long)skip, scratch, s));
    HIPCHK(hipStreamSynchronize(s));
    tmp.release();
    g_last_error.clear();
    return PDT_OK;
  } catch (...) {
    (void)hipStreamSynchronize(s);
    tmp.release();
    return status_of_current_exception();
  }
}

pdt_status pdt_project_simplex(const double* X, double* Y, int64_t rows, int64_t cols, void* stream) {
  if (rows == 0 && cols >= 1 && cols <= 1024) return PDT_OK;
  if (!X || !Y) return set_err(PDT_ERR_INVALID_ARG, "X and Y must not be NULL");
  if (rows < 0 || cols < 1 || cols > 1024) return set_err(PDT_ERR_INVALID_ARG, "need rows >= 0, 1 <= cols <= 1024");
  if (rows > (int64_t)INT_MAX) return set_err(PDT_ERR_INVALID_ARG, "too many rows");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_project_rows<double>(X, Y, (long long)rows, (int)cols, (int)cols, (int)cols, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_err(PDT_ERR_DEVICE, hipGetErrorString(e));
  return PDT_OK;
}

pdt_status pdt_project_simplex_f32(const float* X, float* Y, int64_t rows, int64_t cols, void* stream) {
  if (rows == 0 && cols >= 1 && cols <= 1024) return PDT_OK;
  if (!X || !Y) return set_err(PDT_ERR_INVALID_ARG, "X and Y must not be NULL");
  if (rows < 0 || cols < 1 || cols > 1024) return set_err(PDT_ERR_INVALID_ARG, "need rows >= 0, 1 <= cols <= 1024");
  if (rows > (int64_t)INT_MAX) return set_err(PDT_ERR_INVALID_ARG, "too many rows");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_project_rows<float>(X, Y, (long long)rows, (int)cols, (int)cols, (int)cols, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_err(PDT_ERR_DEVICE, hipGetErrorString(e));
  return PDT_OK;
}

}  // extern "C"

// =======================================================================================
// Warm-start network: FP32 master weights, BF16 copies for the MFMA GEMMs, Adam state.
// =======================================================================================
struct pdt_model_s {
  int64_t n_in = 0, hidden = 0, n_out = 0, nparam = 0;
  hipStream_t stream = nullptr;
  Arena arena, work;
  float* p = nullptr;
  __bf16* pb = nullptr;
  float* g = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  int t = 0;
  int64_t offW[4] = {0, 0, 0, 0}, offb[4] = {0, 0, 0, 0}, fin[4] = {0, 0, 0, 0}, fout[4] = {0, 0, 0, 0};
  int64_t cap = 0;  // batch capacity of the workspace
  __bf16* hb[4] = {nullptr, nullptr, nullptr, nullptr};
  float* z[3] = {nullptr, nullptr, nullptr};
  float* Xf = nullptr;
  float* Y = nullptr;
  float* dY = nullptr;
  __bf16* dYb = nullptr;
  float* dH = nullptr;
  float* dZ = nullptr;
  __bf16* dZb = nullptr;
  double* partials = nullptr;
};

namespace {

constexpr int kLossBlocks = 256;

void model_reserve(pdt_model_s* md, int64_t B) {
  if (B <= md->cap) return;
  md->work.release();
  const int64_t H = md->hidden;
  md->hb[0] = md->work.alloc<__bf16>((size_t)(B * md->n_in));
  for (int l = 1; l < 4; ++l) md->hb[l] = md->work.alloc<__bf16>((size_t)(B * H));
  for (int l = 0; l < 3; ++l) md->z[l] = md->work.alloc<float>((size_t)(B * H));
  md->Xf = md->work.alloc<float>((size_t)(B * md->n_in));
  md->Y = md->work.alloc<float>((size_t)(B * md->n_out));
  md->dY = md->work.alloc<float>((size_t)(B * md->n_out));
  md->dYb = md->work.alloc<__bf16>((size_t)(B * md->n_out));
  md->dH = md->work.alloc<float>((size_t)(B * H));
  md->dZ = md->work.alloc<float>((size_t)(B * H));
  md->dZb = md->work.alloc<__bf16>((size_t)(B * H));
  md->partials = md->work.alloc<double>(kLossBlocks);
  md->cap = B;
}

GemmArgs gemm(const __bf16* A, long long lda, int at, const __bf16* Bm, long long ldb, int bt, int M, int N, int K,
              long long ldc) {
  GemmArgs g{};
  g.A = A;
  g.B = Bm;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.a_trans = at;
  g.b_trans = bt;
  g.M = M;
  g.N = N;
  g.K = K;
  return g;
}

// forward of X (FP32 [B][n_in] on the device, or already BF16 in hb[0] when X == nullptr)
void model_forward(pdt_model_s* md, const float* X, int64_t B) {
  hipStream_t s = md->stream;
  model_reserve(md, B);
  if (X) HIPCHK(launch_f32_to_bf16(X, md->hb[0], B * md->n_in, s));
  for (int l = 0; l < 4; ++l) {
    GemmArgs g = gemm(md->hb[l], md->fin[l], 0, md->pb + md->offW[l], md->fin[l], 1, (int)B, (int)md->fout[l],
                      (int)md->fin[l], md->fout[l]);
    g.bias = md->p + md->offb[l];
    if (l < 3) {
      g.preact = md->z[l];
      g.gelu = 1;
      g.Cbf = md->hb[l + 1];
    } else {
      g.C = md->Y;
    }
    HIPCHK(launch_gemm_bf16(g, s));
  }
}

// gradients into md->g for dLoss/dY given in md->dY (FP32) and md->dYb (BF16)
void model_backward(pdt_model_s* md, int64_t B) {
  hipStream_t s = md->stream;
  const int H = (int)md->hidden;
  const float* dOut = md->dY;
  const __bf16* dOutB = md->dYb;
  for (int l = 3; l >= 0; --l) {
    const int fo = (int)md->fout[l], fi = (int)md->fin[l];
    if (l < 3) {
      // dZ = dH * gelu'(z_l)
      HIPCHK(launch_gelu_back(md->dH, md->z[l], B * H, md->dZ, md->dZb, s));
      dOut = md->dZ;
      dOutB = md->dZb;
    }
    // dW_l = dOut^T h_l   ([fo][fi], contraction over the batch)
    GemmArgs gw = gemm(dOutB, fo, 1, md->hb[l], fi, 0, fo, fi, (int)B, fi);
    gw.C = md->g + md->offW[l];
    HIPCHK(launch_gemm_bf16(gw, s));
    HIPCHK(launch_colsum(dOut, (int)B, fo, md->g + md->offb[l], s));
    if (l > 0) {
      // dH = dOut W_l  ([B][fi])
      GemmArgs gh = gemm(dOutB, fo, 0, md->pb + md->offW[l], fi, 0, (int)B, fi, fo, fi);
      gh.C = md->dH;
      HIPCHK(launch_gemm_bf16(gh, s));
    }
  }
}

pdt_status model_err(pdt_status st, const std::string& m) { return set_err(st, m); }

}  // namespace

extern "C" {

pdt_status pdt_model_create(int64_t n_in, int64_t hidden, int64_t n_out, const float* params, void* stream,
                            pdt_model_t* out) {
  if (!out) return model_err(PDT_ERR_INVALID_ARG, "out must not be NULL");
  *out = nullptr;
  if (n_in < 1 || hidden < 1 || n_out < 1 || n_in > (1 << 20) || hidden > (1 << 16) || n_out > (1 << 26))
    return model_err(PDT_ERR_INVALID_ARG, "bad network sizes");
  pdt_model_s* md = nullptr;
  try {
    md = new pdt_model_s();
    md->n_in = n_in;
    md->hidden = hidden;
    md->n_out = n_out;
    md->stream = static_cast<hipStream_t>(stream);
    const int64_t ins[4] = {n_in, hidden, hidden, hidden}, outs[4] = {hidden, hidden, hidden, n_out};
    int64_t off = 0;
    for (int l = 0; l < 4; ++l) {
      md->fin[l] = ins[l];
      md->fout[l] = outs[l];
      md->offW[l] = off;
      off += ins[l] * outs[l];
      md->offb[l] = off;
      off += outs[l];
    }
    md->nparam = off;
    md->p = md->arena.alloc<float>((size_t)off);
    md->pb = md->arena.alloc<__bf16>((size_t)off);
    md->g = md->arena.alloc<float>((size_t)off);
    md->m = md->arena.alloc<float>((size_t)off);
    md->v = md->arena.alloc<float>((size_t)off);
    hipStream_t s = md->stream;
    if (params) HIPCHK(hipMemcpyAsync(md->p, params, (size_t)off * sizeof(float), hipMemcpyHostToDevice, s));
    else HIPCHK(hipMemsetAsync(md->p, 0, (size_t)off * sizeof(float), s));
    HIPCHK(hipMemsetAsync(md->m, 0, (size_t)off * sizeof(float), s));
    HIPCHK(hipMemsetAsync(md->v, 0, (size_t)off * sizeof(float), s));
    HIPCHK(launch_f32_to_bf16(md->p, md->pb, off, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = md;
    return PDT_OK;
  } catch (...) {
    if (md) {
      (void)hipStreamSynchronize(md->stream);
      md->arena.release();
      delete md;
    }
    return status_of_current_exception();
  }
}

void pdt_model_destroy(pdt_model_t md) {
  if (!md) return;
  (void)hipStreamSynchronize(md->stream);
  md->work.release();
  md->arena.release();
  delete md;
}

int64_t pdt_model_num_params(pdt_model_t md) { return md ? md->nparam : 0; }

pdt_status pdt_model_get_params(pdt_model_t md, float* params_host) {
  if (!md || !params_host) return model_err(PDT_ERR_INVALID_ARG, "NULL argument");
  hipError_t e = hipMemcpyAsync(params_host, md->p, (size_t)md->nparam * sizeof(float), hipMemcpyDeviceToHost, md->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(md->stream);
  return e == hipSuccess ? PDT_OK : model_err(PDT_ERR_DEVICE, hipGetErrorString(e));
}

pdt_status pdt_model_forward(pdt_model_t md, const float* X, float* Y, int64_t B) {
  if (!md || !X || !Y || B < 1) return model_err(PDT_ERR_INVALID_ARG, "bad arguments");
  try {
    model_forward(md, X, B);
    HIPCHK(hipMemcpyAsync(Y, md->Y, (size_t)(B * md->n_out) * sizeof(float), hipMemcpyDeviceToDevice, md->stream));
    HIPCHK(hipStreamSynchronize(md->stream));
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_model_gradients(pdt_model_t md, const float* X, const float* dY, int64_t B, float* grads) {
  if (!md || !X || !dY || !grads || B < 1) return model_err(PDT_ERR_INVALID_ARG, "bad arguments");
  try {
    hipStream_t s = md->stream;
    model_forward(md, X, B);
    HIPCHK(hipMemcpyAsync(md->dY, dY, (size_t)(B * md->n_out) * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_f32_to_bf16(md->dY, md->dYb, B * md->n_out, s));
    model_backward(md, B);
    HIPCHK(hipMemcpyAsync(grads, md->g, (size_t)md->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_model_train_step(pdt_model_t md, const float* X, const float* T, int64_t B, float lr, double* loss) {
  if (!md || !X || !T || B < 1 || !(lr > 0)) return model_err(PDT_ERR_INVALID_ARG, "bad arguments");
  try {
    hipStream_t s = md->stream;
    model_forward(md, X, B);
    const long long n = B * md->n_out;
    HIPCHK(launch_mse_grad(md->Y, T, n, 2.0f / (float)n, md->dY, md->dYb, md->partials, kLossBlocks, s));
    model_backward(md, B);
    md->t += 1;
    HIPCHK(launch_adam(md->p, md->g, md->m, md->v, md->nparam, lr, 0.9f, 0.999f, 1e-8f, md->t, md->pb, md->nparam, s));
    if (loss) {
      double part[kLossBlocks];
      HIPCHK(hipMemcpyAsync(part, md->partials, sizeof(part), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double acc = 0;
      for (int k = 0; k < kLossBlocks; ++k) acc += part[k];
      *loss = acc / (double)n;
    }
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

pdt_status pdt_warmstart_features(pdt_problem_t pb, float* X, int64_t* bins_out) {
  if (!pb || !X) return model_err(PDT_ERR_INVALID_ARG, "bad arguments");
  const Instance& I = pb->inst[0];
  if (I.bins < 1) return model_err(PDT_ERR_INVALID_ARG, "the detector needs at least 2 outcomes");
  hipError_t e = launch_features(I.mu, I.P64, (int)I.D, (int)I.Npad, I.bins, 256, X, nullptr, pb->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(pb->stream);
  if (e != hipSuccess) return model_err(PDT_ERR_DEVICE, hipGetErrorString(e));
  if (bins_out) *bins_out = I.bins;
  return PDT_OK;
}

}  // extern "C"

namespace {

// Learned start: features of the real outcomes -> network -> columns of Pi -> row-wise
// projection.  Falls back to Pi = 1/N (returns 1) when the predicted start is not finite
// or not better than the uniform one.
int learned_start(pdt_problem_s* pb, Instance& I, pdt_model_s* md) {
  if (md->n_in != 258 || md->n_out != I.M) throw ArgError{"the model does not match the problem (n_in 258, n_out M)"};
  if (I.bins < 1) throw ArgError{"the detector needs at least 2 outcomes"};
  hipStream_t s = pb->stream;
  hipStream_t saved = md->stream;
  md->stream = s;
  const int64_t B = I.bins + 1;
  const size_t M = (size_t)I.M, Np = (size_t)I.Npad;
  try {
    model_reserve(md, B);
    HIPCHK(launch_features(I.mu, I.P64, (int)I.D, (int)I.Npad, I.bins, 256, md->Xf, md->hb[0], s));
    model_forward(md, nullptr, B);
    HIPCHK(launch_assemble(md->Y, (int)I.M, I.bins, (int)I.N, (int)I.Npad, I.w64.X[0], s));
    HIPCHK(launch_project_rows<double>(I.w64.X[0], I.w64.X[0], (long long)M, (int)I.N, (int)Np, (int)Np, s));
  } catch (...) {
    md->stream = saved;
    throw;
  }
  md->stream = saved;
  const double f_warm = eval_fp64(pb, I, false, nullptr);
  HIPCHK(hipMemcpyAsync(I.w64.X[1], I.w64.X[0], M * Np * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_fill_rows<double>(I.w64.X[0], (long long)M, (int)I.N, (int)Np, 1.0 / (double)I.N, s));
  const double f_cold = eval_fp64(pb, I, false, nullptr);
  if (std::isfinite(f_warm) && f_warm <= f_cold) {
    HIPCHK(hipMemcpyAsync(I.w64.X[0], I.w64.X[1], M * Np * sizeof(double), hipMemcpyDeviceToDevice, s));
    return 0;
  }
  return 1;
}

}  // namespace

// =======================================================================================
// Batched solve: every instance of the problem, one launch per phase and column-tile
// class over work lists of (instance, tile) items ordered by decreasing band work.
// =======================================================================================
namespace {

template <typename T>
constexpr int plan_slot() { return std::is_same<T, float>::value ? 1 : 0; }

template <typename T>
void build_plan(pdt_problem_s* pb, int scaling, int restart, const std::vector<double>& steps) {
  const int prec = std::is_same<T, float>::value ? PDT_FP32 : PDT_FP64;
  BatchPlan& P = pb->plan[plan_slot<T>()];
  Arena& PA = pb->plan_arena[plan_slot<T>()];
  if (P.prec == prec && P.scaling == scaling && P.restart == restart && P.steps == steps) return;
  if (P.graph) (void)hipGraphExecDestroy(P.graph);
  P = BatchPlan();
  PA.release();
  hipStream_t s = pb->stream;
  const size_t n = pb->inst.size();
  const int var = prec == PDT_FP32 ? VAR_FP32 : VAR_FP64;
  std::vector<BatchInst<T>> host(n);
  // per (column-tile class, workgroup shape): items with their band work as the cost.
  // Each instance keeps the workgroup shape its single solve would use, so the batch
  // reproduces the single solves bit for bit.
  auto key = [](int nt, int ks) { return 2 * nt + (ks == 8 ? 1 : 0); };
  std::vector<std::vector<std::pair<int64_t, int2>>> fx(2 * kMaxNT + 2), ftr(2 * kMaxNT + 2);
  for (size_t k = 0; k < n; ++k) {
    Instance& I = pb->inst[k];
    BatchInst<T> bi;
    bi.pv = view_var(I, var);
    bi.pv.fx_split = 1;  // batches run one workgroup per probe tile and per row tile
    bi.pv.ftr_split = 1;
    // a problem whose row tiles are all narrow runs its single solves' transposed product
    // with four waves (the narrow-only launch): the batch uses the same shape, so the
    // narrow contraction splits and sums its steps in the same order
    if (bi.pv.ftr_narrow_all) bi.pv.ks_ftr = 4;
    bi.b = bufs_of(I, work_of<T>(I), nullptr, scaling == PDT_STEP_DIAG ? I.wrow : nullptr, false, restart);
    bi.b.fx_part = nullptr;
    bi.b.fx_count = nullptr;
    bi.b.ftr_part = nullptr;
    bi.st = I.st;
    bi.step = steps[k];
    bi.n_dt = fx_num_tiles(bi.pv);
    bi.n_mt = ftr_num_waves(bi.pv);
    host[k] = bi;
    const int nt = (int)(I.Npad / 16);
    const int kfx = key(nt, bi.pv.ks_fx), kftr = key(nt, bi.pv.ks_ftr);
    for (int t = 0; t < bi.n_dt; ++t) {
      int64_t lo = INT64_MAX, hi = -1;
      for (int d = 16 * t; d < std::min<int64_t>(16 * t + 16, I.D); ++d) {
        if (I.lo_h[d] > I.hi_h[d]) continue;
        lo = std::min<int64_t>(lo, I.lo_h[d]);
        hi = std::max<int64_t>(hi, I.hi_h[d]);
      }
      fx[kfx].push_back({(hi >= lo ? hi - lo + 1 : 0) * nt, int2{(int)k, t}});
    }
    for (int t = 0; t < bi.n_mt; ++t) ftr[kftr].push_back({(int64_t)nt, int2{(int)k, t}});
  }
  P.insts = PA.alloc<BatchInst<T>>(n);
  HIPCHK(hipMemcpyAsync(P.insts, host.data(), n * sizeof(BatchInst<T>), hipMemcpyHostToDevice, s));
  auto by_cost = [](const std::pair<int64_t, int2>& a, const std::pair<int64_t, int2>& b) {
    return a.first > b.first;
  };
  auto upload = [&](std::vector<std::pair<int64_t, int2>>& v, int c, std::vector<LaunchList>& out) {
    if (v.empty()) return;
    std::stable_sort(v.begin(), v.end(), by_cost);
    std::vector<int2> items;
    for (auto& e : v) items.push_back(e.second);
    LaunchList L;
    L.nt = c / 2;
    L.ks = (c & 1) ? 8 : 4;
    L.n = (int)items.size();
    L.items = PA.alloc<int2>(items.size());
    HIPCHK(hipMemcpyAsync(L.items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    out.push_back(L);
  };
  for (int c = 0; c < 2 * kMaxNT + 2; ++c) {
    upload(fx[c], c, P.fx);
    upload(ftr[c], c, P.ftr);
  }
  HIPCHK(hipStreamSynchronize(s));
  P.prec = prec;
  P.scaling = scaling;
  P.restart = restart;
  P.steps = steps;
}

template <typename T>
void enqueue_batch_iters(pdt_problem_s* pb, int64_t iters, hipStream_t s) {
  BatchPlan& P = pb->plan[plan_slot<T>()];
  const BatchInst<T>* insts = static_cast<const BatchInst<T>*>(P.insts);
  const int n = (int)pb->inst.size();
  for (int64_t k = 0; k < iters; ++k) {
    for (const LaunchList& L : P.ftr)
      HIPCHK((launch_ftr_batch<T, T>(L.nt, L.ks, insts, L.items, L.n, FTR_STEP, s)));
    for (const LaunchList& L : P.fx) HIPCHK((launch_fx_batch<T, T>(L.nt, L.ks, insts, L.items, L.n, FX_ITER, s)));
    HIPCHK(launch_decide_batch<T>(insts, n, DEC_ITER, s));
  }
}

// Every instance's state, with one gather launch and one copy.
void read_batch_states(pdt_problem_s* pb, std::vector<SolverState>& out) {
  hipStream_t s = pb->stream;
  const int n = (int)pb->inst.size();
  out.resize(n);
  HIPCHK(launch_gather_states(pb->st_ptrs, n, pb->st_gather, s));
  HIPCHK(hipMemcpyAsync(out.data(), pb->st_gather, n * sizeof(SolverState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
}

// One phase of a batch from X[0] of every instance (storage T): exact products, f and
// fresh momentum, then chunks of kGraphIters iterations (one recorded graph) until every
// instance is done.  With stall > 0 an instance whose chunk lowered f by less than stall
// relative is stopped (its reduced-precision phase is over).
template <typename T>
void run_batch(pdt_problem_s* pb, double stall, std::vector<SolverState>& out) {
  hipStream_t s = pb->stream;
  BatchPlan& P = pb->plan[plan_slot<T>()];
  const BatchInst<T>* insts = static_cast<const BatchInst<T>*>(P.insts);
  const int n = (int)pb->inst.size();
  for (const LaunchList& L : P.fx) HIPCHK((launch_fx_batch<T, T>(L.nt, L.ks, insts, L.items, L.n, FX_INIT, s)));
  HIPCHK(launch_decide_batch<T>(insts, n, DEC_INIT, s));
  std::vector<SolverState> st;
  read_batch_states(pb, st);
  std::vector<int> flags(n, 0);
  for (;;) {
    int64_t left = 0;
    for (int k = 0; k < n; ++k)
      if (!st[k].done) left = std::max<int64_t>(left, st[k].max_iters - st[k].iter);
    if (left <= 0) break;
    if (left >= kGraphIters) {
      if (!P.graph) {
        if (!pb->capture) HIPCHK(hipStreamCreateWithFlags(&pb->capture, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(pb->capture, hipStreamCaptureModeThreadLocal));
        try {
          enqueue_batch_iters<T>(pb, kGraphIters, pb->capture);
        } catch (...) {
          (void)hipStreamEndCapture(pb->capture, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        HIPCHK(hipStreamEndCapture(pb->capture, &g));
        hipError_t e = hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
      }
      HIPCHK(hipGraphLaunch(P.graph, s));
    } else {
      enqueue_batch_iters<T>(pb, left, s);
    }
    std::vector<SolverState> prev = st;
    read_batch_states(pb, st);
    if (stall > 0) {
      bool any = false;
      for (int k = 0; k < n; ++k) {
        flags[k] = !st[k].done && prev[k].f_cur - st[k].f_cur <= stall * st[k].f_cur;
        any = any || flags[k];
      }
      if (any) {
        HIPCHK(hipMemcpyAsync(pb->st_flags, flags.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(launch_mark_done(pb->st_ptrs, pb->st_flags, n, s));
        read_batch_states(pb, st);
      }
    }
  }
  out = st;
}

}  // namespace

extern "C" {

pdt_status pdt_solve_batch(pdt_problem_t pb, double* const* Pi, const pdt_solve_opts* opts, const double* f_star,
                           pdt_solve_info* info) {
  if (!pb || !Pi || !opts) return set_err(PDT_ERR_INVALID_ARG, "problem, Pi and opts must not be NULL");
  const pdt_solve_opts o = *opts;
  const size_t n = pb->inst.size();
  if (o.max_iters < 0 || !std::isfinite(o.rel_obj_tol) || o.rel_obj_tol < 0)
    return set_err(PDT_ERR_INVALID_ARG, "bad max_iters or tolerance");
  if (o.precision != PDT_FP64 && o.precision != PDT_FP32) return set_err(PDT_ERR_INVALID_ARG, "batch precision must be FP64 or FP32");
  if (o.init != PDT_INIT_UNIFORM && o.init != PDT_INIT_USER) return set_err(PDT_ERR_INVALID_ARG, "bad init");
  if (o.history) return set_err(PDT_ERR_INVALID_ARG, "history is not supported for batches");
  if (o.kkt_tol != 0.0) return set_err(PDT_ERR_INVALID_ARG, "kkt_tol is not supported for batches");
  if (o.scaling != PDT_STEP_UNIFORM && o.scaling != PDT_STEP_DIAG) return set_err(PDT_ERR_INVALID_ARG, "bad scaling");
  if (o.restart != PDT_RESTART_FUNCTION && o.restart != PDT_RESTART_GRADIENT)
    return set_err(PDT_ERR_INVALID_ARG, "bad restart");
  for (size_t k = 0; k < n; ++k)
    if (!Pi[k]) return set_err(PDT_ERR_INVALID_ARG, "Pi[k] must not be NULL");
  const auto t0 = std::chrono::steady_clock::now();
  try {
    hipStream_t s = pb->stream;
    Arena& A = pb->arena;
    if (!pb->st_ptrs) {
      std::vector<SolverState*> ptrs(n);
      for (size_t k = 0; k < n; ++k) ptrs[k] = pb->inst[k].st;
      pb->st_ptrs = A.alloc<SolverState*>(n);
      pb->st_gather = A.alloc<SolverState>(n);
      pb->st_flags = A.alloc<int>(n);
      HIPCHK(hipMemcpyAsync(pb->st_ptrs, ptrs.data(), n * sizeof(SolverState*), hipMemcpyHostToDevice, s));
    }
    std::vector<double> steps(n), Ls(n);
    for (size_t k = 0; k < n; ++k) {
      Instance& I = pb->inst[k];
      ensure_work<double>(A, I, I.w64, I.P64);
      const size_t Np = (size_t)I.Npad, N = (size_t)I.N, M = (size_t)I.M;
      Ls[k] = o.step_L > 0 ? o.step_L : (o.scaling == PDT_STEP_DIAG ? scaled_lipschitz(pb, I) : I.L_hat);
      steps[k] = 1.0 / Ls[k];
      if (o.init == PDT_INIT_USER) HIPCHK(launch_project_rows<double>(Pi[k], I.w64.X[0], (long long)M, (int)N, (int)N, (int)Np, s));
      else HIPCHK(launch_fill_rows<double>(I.w64.X[0], (long long)M, (int)N, (int)Np, 1.0 / (double)N, s));
      const double fs = (f_star && f_star[k] > 0) ? f_star[k] : 0.0;
      init_state(s, I.st, o.max_iters, fs, o.rel_obj_tol, 0.0, (double)M * (double)N, 1);
      if (o.precision == PDT_FP32) {
        if (!I.P32) {
          I.P32 = A.alloc<float>((size_t)I.D * Np);
          HIPCHK(launch_convert_pad<double, float>(I.P64, I.P32, (long long)I.D, (int)Np, (int)Np, (int)Np, s));
        }
        ensure_work<float>(A, I, I.w32, I.P32);
        HIPCHK(launch_convert_pad<double, float>(I.w64.X[0], I.w32.X[0], (long long)M, (int)Np, (int)Np, (int)Np, s));
      }
    }
    std::vector<SolverState> fin, fin32;
    bool refined = false;
    if (o.precision == PDT_FP64) {
      build_plan<double>(pb, o.scaling, o.restart, steps);
      run_batch<double>(pb, 0.0, fin);
    } else {
      build_plan<float>(pb, o.scaling, o.restart, steps);
      run_batch<float>(pb, o.skip_refine ? 0.0 : kStallFp32, fin32);
      // the promoted FP32 iterates, in X64[0]
      for (size_t k = 0; k < n; ++k) {
        Instance& I = pb->inst[k];
        const size_t Np = (size_t)I.Npad;
        HIPCHK(launch_convert_pad<float, double>(I.w32.X[fin32[k].ix_cur], I.w64.X[0], (long long)I.M, (int)Np,
                                                 (int)Np, (int)Np, s));
      }
      fin = fin32;
      if (!o.skip_refine) {
        // as in a single solve: the instances with iterations left start the FP64 phase
        // from their projected iterate, the others keep the FP32 result as it is
        for (size_t k = 0; k < n; ++k) {
          Instance& I = pb->inst[k];
          if (fin32[k].iter < fin32[k].max_iters)
            HIPCHK(launch_project_rows<double>(I.w64.X[0], I.w64.X[0], (long long)I.M, (int)I.N, (int)I.Npad,
                                               (int)I.Npad, s));
        }
        // FP64 refinement of every instance together: each starts from its promoted
        // iterate with fresh momentum and its remaining iterations; an instance whose
        // exact objective already meets its tolerance (or that has none left) stops at once
        std::vector<SolverState> restart(n);
        for (size_t k = 0; k < n; ++k) {
          restart[k] = restart_state(fin32[k]);
          HIPCHK(hipMemcpyAsync(pb->inst[k].st, &restart[k], sizeof(SolverState), hipMemcpyHostToDevice, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        build_plan<double>(pb, o.scaling, o.restart, steps);
        run_batch<double>(pb, 0.0, fin);
        refined = true;
      }
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all_conv = true, all_finite = true;
    for (size_t k = 0; k < n; ++k) {
      Instance& I = pb->inst[k];
      const size_t Np = (size_t)I.Npad, N = (size_t)I.N, M = (size_t)I.M;
      if ((o.precision == PDT_FP64 || refined) && fin[k].ix_cur != 0)
        HIPCHK(hipMemcpyAsync(I.w64.X[0], I.w64.X[fin[k].ix_cur], M * Np * sizeof(double), hipMemcpyDeviceToDevice, s));
      double kkt = 0, fw = 0;
      const double f = eval_fp64(pb, I, true, &kkt, &fw);
      HIPCHK(hipMemcpy2DAsync(Pi[k], N * sizeof(double), I.w64.X[0], Np * sizeof(double), N * sizeof(double), M,
                              hipMemcpyDeviceToDevice, s));
      const double fs = (f_star && f_star[k] > 0) ? f_star[k] : 0.0;
      const bool want = fs > 0 && o.rel_obj_tol > 0;
      const bool conv = want && f - fs <= o.rel_obj_tol * fs;
      const int stk = !std::isfinite(f) ? PDT_ERR_NUMERIC : (want && !conv ? PDT_ERR_NOT_CONVERGED : PDT_OK);
      all_conv = all_conv && (conv || !want);
      all_finite = all_finite && std::isfinite(f);
      if (info) {
        info[k].iters = fin[k].iter;
        info[k].rejects = fin[k].rejects;
        info[k].objective = f;
        info[k].kkt = kkt;
        info[k].L_used = Ls[k];
        info[k].seconds = secs;
        info[k].converged = conv ? 1 : 0;
        info[k].refine_iters = refined ? fin[k].iter - fin32[k].iter : 0;
        info[k].fell_back_to_cold = 0;
        info[k].fw_gap = fw;
        info[k].status = stk;
      }
    }
    HIPCHK(hipStreamSynchronize(s));
    if (!all_finite) return set_err(PDT_ERR_NUMERIC, "objective is not finite for some instance");
    if (!all_conv) return set_err(PDT_ERR_NOT_CONVERGED, "max_iters reached before the tolerance for some instance");
    g_last_error.clear();
    return PDT_OK;
  } catch (...) {
    return status_of_current_exception();
  }
}

}  // extern "C"
