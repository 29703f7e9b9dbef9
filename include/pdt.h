/*
 * pdt.h -- C ABI of libpdt, an MI355X (gfx950) solver for phase-insensitive quantum
 * detector tomography (arXiv 2404.02844).
 *
 * Problem (Eq. min, Sec. 2.1, with the regulariser of Eq. regul, Sec. 3.2):
 *
 *     minimise   f(Pi) = ||F Pi - P||_F^2 + gamma * sum_n sum_{i<M-1} (Pi[i][n] - Pi[i+1][n])^2
 *     subject to Pi[i][n] >= 0,  sum_n Pi[i][n] = 1  for every photon number i,
 *
 * where Pi is the M x N POVM matrix (row i = photon number i, column n = outcome n),
 * P is the D x N matrix of measured outcome frequencies, and F is the D x M matrix of
 * coherent-probe photon-number distributions F[d][i] = mu_d^i exp(-mu_d) / i!
 * (Eq. Fmatrix).  F is never stored: the kernels regenerate it in its band, the
 * photon numbers where F[d][i] >= pmf_threshold.
 *
 * The solver is an accelerated projected-gradient method: a gradient step, the
 * row-wise Euclidean projection onto the probability simplex P_{S^M} (Eq. Mp1_proj,
 * App. B.1) and Nesterov momentum with a monotone restart (a rejected step resets the
 * momentum).  It is the first-order analogue of the paper's first stage (Algorithm 2).
 *
 * Conventions.  Every call returns a pdt_status; nothing throws across the ABI.  On a
 * non-OK status pdt_last_error() returns a thread-local message.  Matrices are dense
 * row-major FP64 at the boundary.  "device" pointers are HIP device memory on the
 * problem's device; "host" pointers are ordinary host memory.  The caller keeps
 * ownership of every array it passes; the library copies what it needs.  Calls that
 * take a stream enqueue their work on it and return after it has completed.
 */
#ifndef PDT_H
#define PDT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdt_problem_s* pdt_problem_t;

typedef enum {
  PDT_OK = 0,
  PDT_ERR_INVALID_ARG = 1,   /* bad sizes, NaN/Inf, mu < 0 or decreasing, gamma < 0, ... */
  PDT_ERR_OUT_OF_MEMORY = 2, /* a device allocation failed; nothing is leaked */
  PDT_ERR_DEVICE = 3,        /* a HIP runtime call or kernel launch failed */
  PDT_ERR_NOT_CONVERGED = 4, /* max_iters reached before the requested tolerance */
  PDT_ERR_NUMERIC = 5        /* the objective became NaN/Inf */
} pdt_status;

typedef enum {
  PDT_FP64 = 0,  /* products and iterates in FP64 (FP64 MFMA) */
  PDT_FP32 = 1,  /* products and iterates in FP32 (FP32 MFMA), FP64 objective; once a
                    64-iteration chunk lowers f by < 1e-6 relative (FP32 storage cannot
                    resolve smaller steps) the solve continues from the promoted iterate in
                    FP64 (the refinement sweep), unless opts.skip_refine */
  PDT_MIXED = 2  /* FP32 MFMA products on FP64 iterates: F X is kept in FP64 and updated by
                    F (X_new - X_cur) in FP32, resynchronised exactly every 64 iterations;
                    once a 64-iteration chunk lowers f by < 1e-10 relative the solve
                    continues in FP64 (the refinement sweep) to the requested tolerance */
} pdt_precision;

typedef enum {
  PDT_TAIL_TRUNCATE = 0, /* F[d][i] = Poisson(i; mu_d) for i < M, as printed in Eq. Fmatrix */
  PDT_TAIL_LUMP = 1      /* as TRUNCATE, but column M-1 holds P(X >= M-1): rows of F sum to 1 */
} pdt_tail_mode;

typedef enum {
  PDT_INIT_UNIFORM = 0, /* Pi = 1/N (the paper's start, Algorithm 1) */
  PDT_INIT_USER = 1,    /* start from the caller's Pi, projected onto the constraints first */
  PDT_INIT_LEARNED = 2  /* start predicted by a warm-start network (opts.model), projected;
                           falls back to 1/N when that start is not better */
} pdt_init_mode;

/*
 * Step of row m of Pi.  UNIFORM: 1/L with L = 1.05 lambda_max(H), H = 2 F^T F + 2 gamma
 * L_path.  DIAG: w_m / L_w with w_m = 1 / max(h_m, 1e-12 max h), h_m = 2 sum_d F[d][m]^2 +
 * 2 gamma L_path[m][m] the Hessian diagonal (the diagonal the paper uses to precondition
 * its CG solves, Table "ops" and App. B), and L_w = 1.05 lambda_max(W^(1/2) H W^(1/2)).
 * The diagonal is the same for every outcome column, so each row is scaled uniformly and
 * the projection stays the row-wise Euclidean one; the minimiser is unchanged.
 */
typedef enum {
  PDT_STEP_UNIFORM = 0,
  PDT_STEP_DIAG = 1
} pdt_step_scaling;

/*
 * Momentum restart.  FUNCTION: a step that raises f is rejected and the momentum reset
 * (t = 1), the monotone restart of the method as defined above.  GRADIENT: in addition,
 * an accepted step resets the momentum when it points against the gradient mapping,
 * sum_m (1 / w_m) sum_n (Y - X_new)[m][n] (X_new - X_cur)[m][n] > 0 (the adaptive
 * restart of O'Donoghue and Candes, 2015, in the metric of the step; w_m = 1 for the
 * uniform step).
 */
typedef enum {
  PDT_RESTART_FUNCTION = 0,
  PDT_RESTART_GRADIENT = 1
} pdt_restart;

typedef struct pdt_model_s* pdt_model_t;

/* One tomography instance (arguments follow Eq. min and Eq. Fmatrix). */
typedef struct {
  int64_t M;            /* Hilbert-space cutoff: photon numbers 0..M-1, M >= 1 */
  int64_t N;            /* detector outcomes, 1 <= N <= 192 */
  int64_t D;            /* probe states, D >= 1 */
  const double* mu;     /* host [D]: probe mean photon numbers |alpha_d|^2, finite, >= 0,
                           non-decreasing */
  const double* P;      /* [D*N] row-major outcome frequencies, finite, >= 0 (host memory,
                           or device memory when P_on_device != 0) */
  int P_on_device;
  double gamma;         /* regularisation weight of Eq. regul, finite, >= 0 */
  double pmf_threshold; /* keep F entries >= this (0: dense F), finite, in [0, 1) */
  int tail_mode;        /* pdt_tail_mode */
} pdt_problem_desc;

/*
 * Validates every instance, copies mu and P to device memory owned by the problem,
 * computes the F bands (per probe: first/last photon number with F >= threshold, and
 * the lumped tail mass) and the Lipschitz constant L = 1.05 * lambda_max(2 F^T F +
 * 2 gamma L_path) of the gradient by 100 FP64 power iterations.  stream: a hipStream_t
 * (NULL = the default stream); all later calls on the problem use it.  On error
 * nothing is allocated and *out is set to NULL.  n_instances >= 2 makes a batch
 * (descs[k] per instance) for pdt_solve_batch.
 */
pdt_status pdt_make_problem(const pdt_problem_desc* descs, int64_t n_instances, void* stream,
                            pdt_problem_t* out);

/* Frees all device memory of the problem.  NULL is a no-op. */
void pdt_destroy_problem(pdt_problem_t problem);

typedef struct {
  int precision;          /* pdt_precision */
  int init;               /* pdt_init_mode */
  int64_t max_iters;      /* iterations of the momentum method, >= 0 */
  double rel_obj_tol;     /* stop once f - f_star <= rel_obj_tol * f_star (needs f_star > 0) */
  double f_star;          /* known optimum value; <= 0 disables the tolerance test */
  double step_L;          /* overrides the Lipschitz constant of the step (L, or L_w with
                             scaling = DIAG); 0 uses the problem's own estimate */
  double* history;        /* optional device [ceil(max_iters / history_stride)]: f after
                             iteration k for k = 0, stride, 2 stride, ... (FP64) */
  pdt_model_t model;      /* warm-start network for init == PDT_INIT_LEARNED (n_in 258, n_out M) */
  int scaling;            /* pdt_step_scaling */
  double kkt_tol;         /* > 0: also stop once the KKT residual (see pdt_solve_info.kkt) of
                             the current iterate is <= kkt_tol; it is formed on the device
                             every 64 iterations (one gradient product) and needs no f_star */
  int skip_refine;        /* PDT_FP32 / PDT_MIXED: 0 (default) continue in FP64 once the
                             reduced-precision phase stalls or meets a tolerance on its own
                             inexact values; 1 stop at the reduced-precision result */
  int64_t history_stride; /* spacing of the history entries (0 or 1: every iteration) */
  int restart;            /* pdt_restart */
} pdt_solve_opts;

typedef struct {
  int64_t iters;          /* iterations performed */
  int64_t rejects;        /* candidate steps rejected (momentum restarts) */
  double objective;       /* f at the returned Pi, FP64 */
  double kkt;             /* KKT residual of App. B at the returned Pi, FP64:
                             sqrt(mean_{i,n} (Pi[i][n] (g[i][n] + lambda_i))^2), g = grad f,
                             lambda_i = -min_n g[i][n] */
  double L_used;          /* Lipschitz constant used for the step (L_w with scaling = DIAG) */
  double seconds;         /* wall time of the call */
  int converged;          /* 1 if a requested test holds at the returned Pi, evaluated in FP64
                             (f - f_star <= rel_obj_tol f_star, or kkt <= kkt_tol) */
  int64_t refine_iters;   /* PDT_FP32 / PDT_MIXED: iterations of the FP64 refinement
                             (included in iters) */
  int fell_back_to_cold;  /* PDT_INIT_LEARNED: 1 if the predicted start was rejected for 1/N */
  double fw_gap;          /* Frank-Wolfe gap sum_i (<g_i, Pi_i> - min_n g[i][n]) at the returned
                             Pi: an upper bound on f - f* (the objective is convex) */
  int status;             /* pdt_status of this instance (batches: per instance) */
} pdt_solve_info;

/*
 * Solves instance 0.  Pi: device [M*N] row-major FP64; read when init == USER, always
 * overwritten with the final iterate (rows on the simplex).  Returns
 * PDT_ERR_NOT_CONVERGED (with Pi and info filled) when a tolerance was requested and
 * did not hold at the returned Pi (evaluated in FP64) when max_iters ran out.
 */
pdt_status pdt_solve(pdt_problem_t problem, double* Pi, const pdt_solve_opts* opts,
                     pdt_solve_info* info);

/*
 * Solves every instance of a problem made with n_instances > 1 (uneven M and N allowed)
 * together: each phase of an iteration is one launch per column-tile class (16 * nt
 * outcome columns) over a work list of (instance, tile) items, ordered by decreasing
 * band work; 64 iterations are captured in one graph and replayed until every instance
 * reports done.  Pi: host array [n_instances] of device pointers, Pi[k] = [M_k * N_k].
 * f_star: host [n_instances] (nullable) per-instance optimum for the tolerance test.
 * info: host [n_instances] (nullable), each with its own status.  precision: PDT_FP64,
 * or PDT_FP32, whose batch (unless skip_refine) promotes every instance to FP64 once
 * each has stalled, met its tolerance on FP32 values or used its iterations, and
 * continues the unconverged ones together in FP64; no history, no kkt_tol.
 * pdt_solve, pdt_objective and pdt_kkt act on instance 0 of such a problem.
 */
pdt_status pdt_solve_batch(pdt_problem_t problem, double* const* Pi, const pdt_solve_opts* opts,
                           const double* f_star, pdt_solve_info* info);

/*
 * f(Pi) (FP64) and optionally its gradient 2 F^T (F Pi - P) + 2 gamma L_path Pi
 * (Table "ops": objective value and gradient).  Pi: device [M*N]; grad_out: device
 * [M*N] or NULL; f_out: host.  Pi is used as given (not projected).
 */
pdt_status pdt_objective(pdt_problem_t problem, const double* Pi, double* f_out, double* grad_out);

/*
 * KKT residual of App. B at Pi (device [M*N]): sqrt(mean((Pi * (grad + lambda))^2))
 * with lambda_i = -min_n grad[i][n].  Result in *kkt_out (host).
 */
pdt_status pdt_kkt(pdt_problem_t problem, const double* Pi, double* kkt_out);

/*
 * Row-wise Euclidean projection onto the probability simplex, P_{S^M} of Eq. Mp1_proj:
 * Y[r] = argmin_{y >= 0, sum y = 1} ||X[r] - y||.  X, Y: device [rows*cols] row-major
 * FP64 (X == Y allowed); 1 <= cols <= 1024.  stream: hipStream_t or NULL.
 */
pdt_status pdt_project_simplex(const double* X, double* Y, int64_t rows, int64_t cols, void* stream);

/*
 * Long-range smoothing before the paper's second, stage-2-only run (Sec. 3.2,
 * Eq. smoothing): out[i] = mean of Pi rows i - h .. i + h with h = min(floor(i /
 * divisor), M - 1 - i) (the paper: divisor 50), for i >= skip (the paper: ~100); rows
 * below skip are copied.  The window stays centred on i, shrinking at the top of the
 * range.  Pi, out: device [M*N] row-major FP64 (out == Pi allowed).  Window sums are
 * differences of compensated FP64 column prefix sums (temporary device memory of
 * 2 (M + 1 + M/256) N doubles).  stream: hipStream_t or NULL.
 */
pdt_status pdt_smooth_rows(const double* Pi, double* out, int64_t M, int64_t N, int32_t divisor, int64_t skip,
                           void* stream);

/*
 * pdt_smooth_rows without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as pdt_smooth_rows, but the window
 * sums use a fixed device array of PDT_SMOOTH_NOALLOC_MAX_DOUBLES doubles (64 MiB)
 * that the library holds on each GPU it runs on until the process ends, instead of
 * temporary memory.  Sizes with 2 (M + 1 + ceil(M / 256)) N above that limit are
 * rejected with PDT_ERR_INVALID_ARG (e.g. M = 16384 rows of N <= 255 outcomes fit).
 * The array's address on the current device is looked up on the first call on that
 * device; the call then uses the current device, so `stream` must belong to it.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * threads, other streams) race and give wrong results; serialise them.  No entry of
 * the array needs to start at zero (each pass writes what the next reads).
 */
#define PDT_SMOOTH_NOALLOC_MAX_DOUBLES (8ll << 20)
pdt_status pdt_smooth_rows_noalloc(const double* Pi, double* out, int64_t M, int64_t N, int32_t divisor,
                                   int64_t skip, void* stream);

/* Same, FP32. */
pdt_status pdt_project_simplex_f32(const float* X, float* Y, int64_t rows, int64_t cols, void* stream);

/* Problem facts for tests and reports: band edges (host int32 [D] each, nullable),
 * lumped tail mass (host [D], nullable), Lipschitz constant (host, nullable),
 * number of band entries sum_d (hi_d - lo_d + 1) (host, nullable). */
pdt_status pdt_problem_bands(pdt_problem_t problem, int32_t* lo, int32_t* hi, double* tail,
                             double* lipschitz, int64_t* nnz);

/* Row scaling of instance 0 (see pdt_step_scaling): Hessian diagonal h (host [M],
 * nullable) and L_w (host, nullable; 100 FP64 power iterations on first request). */
pdt_status pdt_problem_scaling(pdt_problem_t problem, double* hdiag, double* lipschitz_scaled);

/*
 * Workgroup shape of the two band kernels (not a quantity of the paper: a launch
 * parameter).  Each band product runs one workgroup per 16-row tile whose waves split
 * the tile's contraction; ks_fx / ks_ftr waves (4 or 8) for the forward / transposed
 * product of the given precision of one instance.  0 selects the tuning table, which
 * picks 8 for launches with few tiles (see pdt_tuning.h).  The waves' partial results
 * are summed in a fixed order, so a given shape is deterministic, while the two shapes
 * differ in rounding.  Changing the shape drops captured graphs and the batch plan.
 * A problem whose 16-row tiles all meet fewer than 32 probes runs its transposed product
 * as a dedicated four-wave launch without chunk staging (its ks_ftr is not used).
 */
pdt_status pdt_problem_set_tiles(pdt_problem_t problem, int64_t instance, int precision, int ks_fx, int ks_ftr);
/* The shape in effect (host int* outputs, nullable). */
pdt_status pdt_problem_tiles(pdt_problem_t problem, int64_t instance, int precision, int* ks_fx, int* ks_ftr);

/*
 * Split contraction of the forward band product (a launch parameter, not a quantity of
 * the paper).  With few 16-probe tiles and long photon-number ranges (the paper's
 * experiment: D = 1076 probes with bands ~1.8e4 wide) each tile's contraction is shared
 * by `split` workgroups whose partial tiles the last of them sums in a fixed order.
 * split in [1, 16], or 0 for the automatic choice made at setup (up to 16 workgroups
 * per tile, about 768 in all, when there are fewer than 256 tiles, at least 32 64-entry
 * chunks each; else 1).
 * Different splits differ in rounding only.  Drops captured graphs.
 */
pdt_status pdt_problem_set_fx_split(pdt_problem_t problem, int64_t instance, int split);
/* The split in effect (host int*). */
pdt_status pdt_problem_fx_split(pdt_problem_t problem, int64_t instance, int* split);

/*
 * Split contraction of the transposed band product F^T R (a launch parameter, not a
 * quantity of the paper).  Each 16-row tile's probe range (its 64-probe chunks) is cut
 * into `split` contiguous parts, one workgroup each, whose partial tiles a second
 * launch sums in part order before the projected step.  More workgroups fill
 * the GPU when row tiles are few against their probe ranges (M = 4096 rows: 256 tiles of
 * ~760 probes).  split in [1, 16], or 0 for the automatic choice made at setup (1).
 * Scratch: [ceil(M/16) * split * 16 * Npad] FP64, allocated on first use and kept.
 * Batched solves always run one workgroup per row tile.  Different splits differ in
 * rounding only.  Drops captured graphs.
 */
pdt_status pdt_problem_set_ftr_split(pdt_problem_t problem, int64_t instance, int split);
/* The split in effect (host int*). */
pdt_status pdt_problem_ftr_split(pdt_problem_t problem, int64_t instance, int* split);

/*
 * The paper's own solver: the two-stage two-metric projected truncated Newton method
 * of App. B (Algorithms 1-3) on instance 0.
 *
 * Stage 1 (Algorithm 2): binding set I = {Pi <= eps, df/dPi > 0} (Eq. 2metric_I) with
 * eps = min(eps_cap, ||Pi - P_S(Pi - grad)||) (eps_cap 1e-9 by default; stage 2 uses the
 * residual of the bound constraints); direction from D P = -grad, D the Hessian
 * 2 F^T F + 2 gamma L_path on the free entries and its diagonal on I, solved by
 * conjugate gradients preconditioned with the Hessian diagonal (Hessian products are
 * the band kernels of pdt_solve); Armijo search (beta 3/4, c 1/10) on
 * P_S(Pi + alpha P), slope phi'(0) the exact one-sided derivative of that path (the
 * projection of P onto the tangent cone of the simplex rows).
 * Switches to stage 2 once |phi'(0)| <= stage_switch (or when no trial is accepted).
 * Stage 2 (Algorithm 1): every row's largest entry m(i) is eliminated through the row
 * sum; the same two-metric step in the reduced variables (reduced Hessian T^T H T,
 * diagonal 2 h), trials max(Pi + alpha P, 0) with the eliminated entry from the sum,
 * accepted when Armijo holds and every eliminated entry is >= 0.  Stops once the KKT
 * residual with the clamped multiplier max(0, -min_n grad) is <= eps_kkt, or when no
 * trial is accepted.  A descent test failure (phi'(0) >= 0) falls back to -grad.
 *
 * Pi: device [M*N] row-major FP64, read when init == PDT_INIT_USER (projected onto the
 * simplex rows first), always overwritten with the final iterate.  history: host
 * [max_newton + 1] (nullable), f at the start and after every Newton step.
 * With f_star > 0 the solve also stops once f - f_star <= rel_obj_tol * f_star (the
 * comparison test of pdt_solve).  Returns PDT_ERR_NOT_CONVERGED (with Pi and info
 * filled) when the method stopped (max_newton reached, or no stage-2 trial accepted)
 * before either test held.
 * The first Newton call on a problem (this one, pdt_hessian_apply or
 * pdt_newton_direction) allocates the method's work arrays (eight [M*N] and four [D*N]
 * FP64 arrays, N padded to a multiple of 16, and a byte mask), two ints of pinned host memory mapped for the device (the CG
 * completion flags) and, on the first CG solve of each stage, two recorded graphs of
 * four CG iterations.  The problem keeps all of them until pdt_destroy_problem;
 * pdt_problem_set_tiles, pdt_problem_set_fx_split and pdt_problem_set_ftr_split drop
 * the graphs.
 */
typedef struct {
  int64_t max_newton;     /* Newton steps of both stages, >= 0 */
  double eps_kkt;         /* stage-2 stopping residual, >= 0 */
  double stage_switch;    /* |phi'(0)| of the stage transition (paper: 1e-4) */
  double cg_rtol;         /* CG stops at ||r|| <= cg_rtol ||r_0|| */
  int32_t cg_max;         /* CG iterations per Newton step, >= 1 */
  int32_t init;           /* PDT_INIT_UNIFORM or PDT_INIT_USER */
  int32_t stage2_only;    /* 1: start in stage 2 */
  double* history;        /* host [max_newton + 1] or NULL */
  double f_star;          /* known optimum value; <= 0 disables the objective test */
  double rel_obj_tol;     /* also stop once f - f_star <= rel_obj_tol * f_star */
  double eps_cap;         /* binding tolerance eps = min(eps_cap, w) (0: 1e-9) */
} pdt_newton_opts;

typedef struct {
  int64_t stage1_iters;   /* accepted or attempted stage-1 steps */
  int64_t stage2_iters;
  int64_t cg_iters;       /* CG iterations over all steps */
  int64_t line_trials;    /* objective evaluations of the line searches */
  double objective;       /* f at the returned Pi */
  double kkt;             /* KKT residual with the clamped multiplier */
  double seconds;
  int converged;          /* 1 if the KKT or the objective test was met */
} pdt_newton_info;

pdt_status pdt_newton_solve(pdt_problem_t problem, double* Pi, const pdt_newton_opts* opts,
                            pdt_newton_info* info);

/*
 * Hessian product HV = 2 F^T (F V) + 2 gamma L_path V of instance 0 (Table "ops",
 * Hessian products: the operator of the CG solves), by the band kernels.  V, HV: device [M*N]
 * row-major FP64 (distinct).
 */
pdt_status pdt_hessian_apply(pdt_problem_t problem, const double* V, double* HV);

/*
 * One Newton direction of the given stage (1 or 2) at Pi (device [M*N], used as given)
 * with binding tolerance eps >= 0: the CG solve of the two-metric system described at
 * pdt_newton_solve.  Dir: device [M*N], receives the direction (stage 2: the reduced
 * variables, 0 at the eliminated entries).  row_max: device int32 [M] (nullable),
 * receives m(i) in stage 2.  cg_iters, slope (host, nullable): CG iterations and
 * phi'(0) of the direction as the line search would use it.  No steepest-descent
 * fallback is applied.
 */
pdt_status pdt_newton_direction(pdt_problem_t problem, int stage, const double* Pi, double eps, double cg_rtol,
                                int32_t cg_max, double* Dir, int32_t* row_max, int64_t* cg_iters,
                                double* slope);

/*
 * Warm-start network (learned initial Pi; not in the paper, whose runs start from
 * Pi = 1/N and, for its smoothed second run, from a window average of a solution).
 * Four linear layers n_in -> hidden -> hidden -> hidden -> n_out with the tanh form of
 * GELU after the first three; weights [out][in] row-major, y = x W^T + b.  Products run
 * on BF16 MFMA with FP32 accumulation; master weights and Adam moments are FP32.
 * Parameter vector (FP32): W1, b1, W2, b2, W3, b3, W4, b4 in that order.
 * Features of outcome n of a detector whose outcomes 0..bins carry probability:
 * P[:, n] linearly interpolated at 256 equally spaced mean photon numbers from mu_0 to
 * mu_{D-1}, then n / bins and bins / 128 (n_in = 258).
 */
/* params: host [num_params] FP32 or NULL (zeros); stream: hipStream_t or NULL. */
pdt_status pdt_model_create(int64_t n_in, int64_t hidden, int64_t n_out, const float* params, void* stream,
                            pdt_model_t* out);
void pdt_model_destroy(pdt_model_t model);
int64_t pdt_model_num_params(pdt_model_t model);
/* params_host: host [num_params] FP32, receives the master weights. */
pdt_status pdt_model_get_params(pdt_model_t model, float* params_host);
/* X: device [B*n_in] FP32, Y: device [B*n_out] FP32. */
pdt_status pdt_model_forward(pdt_model_t model, const float* X, float* Y, int64_t B);
/* Gradient of a loss whose derivative w.r.t. the output is dY (device [B*n_out]) into
 * grads (device [num_params], same layout as the parameters). */
pdt_status pdt_model_gradients(pdt_model_t model, const float* X, const float* dY, int64_t B, float* grads);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on mean((Y - T)^2); X, T on the
 * device; *loss (host, nullable) receives the loss before the step. */
pdt_status pdt_model_train_step(pdt_model_t model, const float* X, const float* T, int64_t B, float lr,
                                double* loss);
/* Features of the problem's real outcomes: X device [(bins+1)*258]; *bins_out host. */
pdt_status pdt_warmstart_features(pdt_problem_t problem, float* X, int64_t* bins_out);

/*
 * Measurement hook: enqueues `reps` launches of one kernel of the iteration on the
 * problem's stream and returns without waiting, so the caller can bracket them with
 * its own HIP events.  kernel: 0 = transposed band product + projected step,
 * 1 = forward band product + objective partials, 2 = accept/reject decision,
 * 3 = one whole iteration (0, 1, 2).  Requires an earlier pdt_solve in the same
 * precision (it works on that solve's buffers, whose contents it overwrites).
 */
pdt_status pdt_replay_kernel(pdt_problem_t problem, int kernel, int precision, int64_t reps);

/* Thread-local message of the last failing call ("" if none). */
const char* pdt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PDT_H */
