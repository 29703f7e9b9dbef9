// Row kernels of the two-stage two-metric projected truncated Newton method (App. B,
// Algorithms 1-3): binding sets and right-hand sides of the two-metric system, the
// diagonally preconditioned conjugate-gradient updates around the band-kernel Hessian
// products, the line-search slope, and the trial points of both stages.
//
// One wave per row of Pi (column c = 64 v + lane, V = ceil(Npad / 64) values per lane),
// rows dealt round-robin over a fixed grid so that every reduction adds its per-wave
// partials in one order: per block in wave order, then over the blocks in block order.
// HBM-bound elementwise work: each kernel streams a few [M][Npad] arrays once.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "pdt_decide.h"
#include "pdt_device.h"
#include "pdt_newton.h"

namespace pdt {

namespace {

constexpr int kWavesPerBlock = 4;

__device__ __forceinline__ double diag_of(const double* h, int m, int stage) {
  const double d = stage == 1 ? h[m] : 2.0 * h[m];
  return d > 0.0 ? d : 1.0;  // a row no probe reaches with gamma = 0 keeps a unit diagonal
}

// lowest column index of the row maximum over the real columns (every lane gets it)
template <int V>
__device__ __forceinline__ int row_argmax(const double (&x)[V], int N, int lane) {
  double bv = -INFINITY;
  int bi = INT_MAX;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = 64 * v + lane;
    if (c < N && x[v] > bv) {
      bv = x[v];
      bi = c;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  return bi;
}

// value of column c0 of a row held one column per (v, lane) (exact: one term is nonzero)
template <int V>
__device__ __forceinline__ double row_pick(const double (&x)[V], int c0, int lane) {
  double s = 0.0;
#pragma unroll
  for (int v = 0; v < V; ++v) s += (64 * v + lane == c0) ? x[v] : 0.0;
  return group_sum<64>(s);
}

// per-block partial sums of K quantities in a fixed order
template <int K>
__device__ __forceinline__ void block_partials(double (&acc)[K], double* part, int nb) {
  __shared__ double sh[K][kWavesPerBlock];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double t = group_sum<64>(acc[k]);
    if (lane == 0) sh[k][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWavesPerBlock; ++w) t += sh[k][w];
      part[(size_t)k * nb + blockIdx.x] = t;
    }
  }
}

// fixed-order sum of nb block partials by one block of 256 threads: strided per-thread
// sums, an xor butterfly per wave (every lane, and every block given the same partials,
// ends with the same bits), then the wave sums in wave order
__device__ __forceinline__ double sum_partials(const double* part, int nb) {
  __shared__ double sh[kWavesPerBlock];
  double s = strided_sum256(part, nb, threadIdx.x);
  s = group_sum<64>(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) r += sh[w];
  __syncthreads();
  return r;
}

#define NT_ROWS(r)                                                      \
  const int lane = threadIdx.x & 63;                                    \
  const int wave0 = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);   \
  const int nwaves = gridDim.x * kWavesPerBlock;                        \
  for (int m = wave0; m < (r).M; m += nwaves)

// ---- KKT residual with the clamped multiplier, and the residual w of the binding-set
// tolerance eps = min(cap, w) (cap: the eps_cap option, 1e-9 by default) ------------------
template <int V>
__global__ __launch_bounds__(256) void nt_measure_kernel(NtRows r, const double* X, const double* G, double* part) {
  double acc[2] = {0.0, 0.0};
  NT_ROWS(r) {
    const size_t base = (size_t)m * r.Npad;
    double x[V], g[V];
    double gmin = INFINITY;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      x[v] = c < r.N ? X[base + c] : 0.0;
      g[v] = c < r.N ? G[base + c] : 0.0;
      if (c < r.N) gmin = fmin(gmin, g[v]);
    }
    gmin = group_min<64>(gmin);
    const double lam = fmax(-gmin, 0.0);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double e = x[v] * (g[v] + lam);
      acc[0] += (64 * v + lane < r.N) ? e * e : 0.0;
    }
    if (r.stage == 1) {
      // ||Pi - P_S(Pi - g)||
      double z[1][V];
#pragma unroll
      for (int v = 0; v < V; ++v) z[0][v] = (64 * v + lane < r.N) ? x[v] - g[v] : neg_huge<double>();
      double tau[1];
      simplex_threshold<double, 64, V, 1, 8>(z, tau);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double e = x[v] - fmax(z[0][v] - tau[0], 0.0);
        acc[1] += (64 * v + lane < r.N) ? e * e : 0.0;
      }
    } else {
      // ||min(Pi, reduced gradient)|| over the reduced variables
      const int mi = row_argmax<V>(x, r.N, lane);
      const double gm = row_pick<V>(g, mi, lane);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int c = 64 * v + lane;
        const double e = fmin(x[v], g[v] - gm);
        acc[1] += (c < r.N && c != mi) ? e * e : 0.0;
      }
    }
  }
  block_partials<2>(acc, part, gridDim.x);
}

// ---- two-metric system: codes, right-hand side, first CG residual and direction -------
template <int V>
__global__ __launch_bounds__(256) void nt_prep_kernel(NtRows r, const double* X, const double* G, const double* h,
                                                      double eps, uint8_t* mask, int* mi_out, double* res,
                                                      double* z, double* p, double* Vf, double* Dir, double* part) {
  double acc[2] = {0.0, 0.0};
  NT_ROWS(r) {
    const size_t base = (size_t)m * r.Npad;
    double x[V], g[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      x[v] = c < r.N ? X[base + c] : 0.0;
      g[v] = c < r.N ? G[base + c] : 0.0;
    }
    int mi = -1;
    double gm = 0.0;
    if (r.stage == 2) {
      mi = row_argmax<V>(x, r.N, lane);
      gm = row_pick<V>(g, mi, lane);
      if (lane == 0) mi_out[m] = mi;
    }
    const double dg = diag_of(h, m, r.stage);
    double vf[V];
    double vsum = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      const bool var = c < r.N && c != mi;
      const double gr = g[v] - gm;
      const bool bind = var && x[v] <= eps && gr > 0.0;
      const double rr = var ? -gr : 0.0;
      const double zz = var ? rr / dg : 0.0;
      vf[v] = (var && !bind) ? zz : 0.0;
      vsum += vf[v];
      acc[0] += rr * rr;
      acc[1] += rr * zz;
      if (c < r.Npad) {
        mask[base + c] = (uint8_t)(!var ? 2 : (bind ? 1 : 0));
        res[base + c] = rr;
        z[base + c] = zz;
        p[base + c] = zz;
        Dir[base + c] = 0.0;
      }
    }
    if (r.stage == 2) {
      vsum = group_sum<64>(vsum);
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (64 * v + lane == mi) vf[v] = -vsum;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      if (c < r.Npad) Vf[base + c] = vf[v];
    }
  }
  block_partials<2>(acc, part, gridDim.x);
}

__global__ __launch_bounds__(256) void nt_cginit_kernel(const double* part, int nb, NewtonState* ns, double rtol,
                                                        int cg_max) {
  const double rr0 = sum_partials(part, nb);
  const double rz = sum_partials(part + nb, nb);
  if (threadIdx.x != 0) return;
  ns->nr0 = sqrt(rr0);
  ns->rz[0] = rz;
  ns->rtol = rtol;
  ns->cg_iter = 0;
  ns->cg_max = cg_max;
  ns->cg_done = (rr0 == 0.0 || cg_max <= 0) ? 1 : 0;
}

// ---- q = D p from the Hessian product Gh = H (free part of p, expanded) --------------
template <int V>
__global__ __launch_bounds__(256) void nt_q_kernel(NtRows r, const uint8_t* mask, const int* mi_in, const double* h,
                                                   const double* p, const double* Gh, double* q, double* part,
                                                   const NewtonState* ns) {
  if (ns->cg_done) return;
  double acc[1] = {0.0};
  NT_ROWS(r) {
    const size_t base = (size_t)m * r.Npad;
    const double gm = r.stage == 2 ? Gh[base + mi_in[m]] : 0.0;
    const double dg = diag_of(h, m, r.stage);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      if (c < r.Npad) {
        const int code = mask[base + c];
        const double pv = p[base + c];
        const double qq = code == 0 ? Gh[base + c] - gm : (code == 1 ? dg * pv : 0.0);
        q[base + c] = qq;
        acc[0] += pv * qq;
      }
    }
  }
  block_partials<1>(acc, part, gridDim.x);
}

// CG step of iteration k (par = k % 2): every block forms p'q from the q kernel's
// partials in the same fixed order, so all blocks take the same alpha = r'z / p'q and
// the same decision; block 0 records it.  r'z of iteration k sits in rz[par].
template <int V>
__global__ __launch_bounds__(256) void nt_update_kernel(NtRows r, const uint8_t* mask, const double* h, double* Dir,
                                                        double* res, double* z, const double* p, const double* q,
                                                        const double* part_pq, double* part, NewtonState* ns,
                                                        int par) {
  if (ns->cg_done) return;
  const double pq = sum_partials(part_pq, gridDim.x);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ns->cg_iter += 1;
    if (!(pq > 0.0)) ns->cg_done = 1;  // D is not positive definite along p: keep the current solution
  }
  if (!(pq > 0.0)) return;
  const double alpha = ns->rz[par] / pq;
  double acc[2] = {0.0, 0.0};
  NT_ROWS(r) {
    const size_t base = (size_t)m * r.Npad;
    const double dg = diag_of(h, m, r.stage);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      if (c < r.Npad && mask[base + c] != 2) {
        Dir[base + c] += alpha * p[base + c];
        const double rr = res[base + c] - alpha * q[base + c];
        const double zz = rr / dg;
        res[base + c] = rr;
        z[base + c] = zz;
        acc[0] += rr * rr;
        acc[1] += rr * zz;
      }
    }
  }
  block_partials<2>(acc, part, gridDim.x);
}

// Next search direction: every block forms r'r and r'z from the update's partials in the
// same fixed order and takes the same stopping decision and beta = r'z_new / r'z; block 0
// records r'z_new in rz[par ^ 1] (rz[par] stays readable for the other blocks) and stores
// the solve's completion state in *flag (host memory mapped for the device).
template <int V>
__global__ __launch_bounds__(256) void nt_dir_kernel(NtRows r, const uint8_t* mask, const int* mi_in, const double* z,
                                                     double* p, double* Vf, const double* part, NewtonState* ns,
                                                     int par, int* flag) {
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (ns->cg_done) {
    if (lead) {
      *flag = 1;
      __threadfence_system();
    }
    return;
  }
  const double rr = sum_partials(part, gridDim.x);
  const double rzn = sum_partials(part + gridDim.x, gridDim.x);
  const bool stop = sqrt(rr) <= ns->rtol * ns->nr0 || ns->cg_iter >= ns->cg_max;
  if (lead) {
    if (stop) ns->cg_done = 1;
    else ns->rz[par ^ 1] = rzn;
    *flag = stop ? 1 : 0;
    __threadfence_system();
  }
  if (stop) return;
  const double beta = rzn / ns->rz[par];
  NT_ROWS(r) {
    const size_t base = (size_t)m * r.Npad;
    const int mi = r.stage == 2 ? mi_in[m] : -1;
    double vf[V];
    double vsum = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      vf[v] = 0.0;
      if (c < r.Npad) {
        const int code = mask[base + c];
        const double pn = code == 2 ? 0.0 : z[base + c] + beta * p[base + c];
        p[base + c] = pn;
        vf[v] = code == 0 ? pn : 0.0;
      }
      vsum += vf[v];
    }
    if (r.stage == 2) {
      vsum = group_sum<64>(vsum);
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (64 * v + lane == mi) vf[v] = -vsum;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      if (c < r.Npad) Vf[base + c] = vf[v];
    }
  }
}

// ---- slope phi'(0) of the line search: the exact one-sided derivative at alpha = 0 ----
// Stage 1: for a row x on the simplex, d/dalpha P_S(x + alpha d) at 0+ is d_n - t on the
// support and max(d_n - t, 0) on the zero entries, with t the shift that keeps the row
// sum: the threshold is grown over the entries above it until that set stops changing
// (at most N passes: every pass that continues drops an entry).  Stage 2: the bound
// projection moves entry (i, n) by Dir unless Pi = 0 and Dir < 0, and the row maximum
// takes minus the sum of the others.
template <int V>
__global__ __launch_bounds__(256) void nt_slope_kernel(NtRows r, const double* X, const double* Dir, const double* G,
                                                       const int* mi_in, double* part) {
  double acc[1] = {0.0};
  NT_ROWS(r) {
    const size_t base = (size_t)m * r.Npad;
    double x[V], d[V], g[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      x[v] = c < r.N ? X[base + c] : 0.0;
      d[v] = c < r.N ? Dir[base + c] : 0.0;
      g[v] = c < r.N ? G[base + c] : 0.0;
    }
    if (r.stage == 1) {
      bool zero[V], active[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int c = 64 * v + lane;
        zero[v] = c < r.N && x[v] == 0.0;
        active[v] = c < r.N;
      }
      double t = 0.0;
      for (int pass = 0; pass <= r.N; ++pass) {
        double s = 0.0;
        int cnt = 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          s += active[v] ? d[v] : 0.0;
          cnt += active[v] ? 1 : 0;
        }
        s = group_sum<64>(s);
        cnt = group_isum<64>(cnt);
        t = s / (double)cnt;
        int dropped = 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const bool keep = !zero[v] || d[v] > t;
          dropped += (active[v] && !keep) ? 1 : 0;
          active[v] = active[v] && keep;
        }
        if (group_isum<64>(dropped) == 0) break;
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double tv = zero[v] ? fmax(d[v] - t, 0.0) : d[v] - t;
        acc[0] += (64 * v + lane < r.N) ? g[v] * tv : 0.0;
      }
    } else {
      const int mi = mi_in[m];
      double s = 0.0;
      double u[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int c = 64 * v + lane;
        u[v] = (c < r.N && c != mi && (x[v] > 0.0 || d[v] > 0.0)) ? d[v] : 0.0;
        s += u[v];
      }
      s = group_sum<64>(s);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int c = 64 * v + lane;
        acc[0] += g[v] * (c == mi ? -s : u[v]);
      }
    }
  }
  block_partials<1>(acc, part, gridDim.x);
}

// steepest-descent replacement of a direction that does not descend
template <int V>
__global__ __launch_bounds__(256) void nt_negrad_kernel(NtRows r, const double* G, const int* mi_in, double* Dir) {
  NT_ROWS(r) {
    const size_t base = (size_t)m * r.Npad;
    double g[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      g[v] = c < r.N ? G[base + c] : 0.0;
    }
    const int mi = r.stage == 2 ? mi_in[m] : -1;
    const double gm = r.stage == 2 ? row_pick<V>(g, mi, lane) : 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      if (c < r.Npad) Dir[base + c] = (c < r.N && c != mi) ? -(g[v] - gm) : 0.0;
    }
  }
}

// ---- trial points: P_S(Pi + alpha Dir) (stage 1); bounds projection of the reduced
// variables and the row maximum from the sum constraint (stage 2), counting the rows
// whose eliminated entry turns negative -------------------------------------------------
template <int V>
__global__ __launch_bounds__(256) void nt_trial_kernel(NtRows r, const double* X, const double* Dir, const int* mi_in,
                                                       double alpha, double* Xa, double* part) {
  double acc[1] = {0.0};
  NT_ROWS(r) {
    const size_t base = (size_t)m * r.Npad;
    double z[1][V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = 64 * v + lane;
      z[0][v] = c < r.N ? X[base + c] + alpha * Dir[base + c] : neg_huge<double>();
    }
    if (r.stage == 1) {
      double tau[1];
      simplex_threshold<double, 64, V, 1, 8>(z, tau);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int c = 64 * v + lane;
        if (c < r.Npad) Xa[base + c] = c < r.N ? fmax(z[0][v] - tau[0], 0.0) : 0.0;
      }
    } else {
      const int mi = mi_in[m];
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int c = 64 * v + lane;
        z[0][v] = (c < r.N && c != mi) ? fmax(z[0][v], 0.0) : 0.0;
        s += z[0][v];
      }
      s = group_sum<64>(s);
      const double xm = 1.0 - s;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int c = 64 * v + lane;
        if (c < r.Npad) Xa[base + c] = c == mi ? xm : z[0][v];
      }
      if (lane == 0 && xm < 0.0) acc[0] += 1.0;
    }
  }
  block_partials<1>(acc, part, gridDim.x);
}

// K consecutive arrays of nb partials -> ns->out[slot + k]
template <int K>
__global__ __launch_bounds__(256) void nt_sum_kernel(const double* part, int nb, NewtonState* ns, int slot) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double t = sum_partials(part + (size_t)k * nb, nb);
    if (threadIdx.x == 0) ns->out[slot + k] = t;
  }
}

int nt_blocks(const NtRows& r) {
  const int need = (r.M + kWavesPerBlock - 1) / kWavesPerBlock;
  return need < kNtBlocks ? (need > 0 ? need : 1) : kNtBlocks;
}

#define NT_V_SWITCH(r, CALL)                     \
  switch (((r).Npad + 63) / 64) {                \
    case 1: CALL(1); break;                      \
    case 2: CALL(2); break;                      \
    case 3: CALL(3); break;                      \
    default: return hipErrorInvalidValue;        \
  }

}  // namespace

hipError_t launch_nt_measure(const NtRows& r, const double* X, const double* G, double* part, NewtonState* ns,
                             hipStream_t s) {
  const int nb = nt_blocks(r);
#define K_(V) hipLaunchKernelGGL((nt_measure_kernel<V>), dim3(nb), dim3(256), 0, s, r, X, G, part)
  NT_V_SWITCH(r, K_)
#undef K_
  hipLaunchKernelGGL((nt_sum_kernel<2>), dim3(1), dim3(256), 0, s, part, nb, ns, 0);
  return hipGetLastError();
}

hipError_t launch_nt_prep(const NtRows& r, const double* X, const double* G, const double* h, double eps,
                          uint8_t* mask, int* mi, double* res, double* z, double* p, double* Vf, double* Dir,
                          double* part, NewtonState* ns, double rtol, int cg_max, hipStream_t s) {
  const int nb = nt_blocks(r);
#define K_(V)                                                                                                 \
  hipLaunchKernelGGL((nt_prep_kernel<V>), dim3(nb), dim3(256), 0, s, r, X, G, h, eps, mask, mi, res, z, p, Vf, \
                     Dir, part)
  NT_V_SWITCH(r, K_)
#undef K_
  hipLaunchKernelGGL(nt_cginit_kernel, dim3(1), dim3(256), 0, s, part, nb, ns, rtol, cg_max);
  return hipGetLastError();
}

hipError_t launch_nt_q(const NtRows& r, const uint8_t* mask, const int* mi, const double* h, const double* p,
                       const double* Gh, double* q, double* part, NewtonState* ns, hipStream_t s) {
  const int nb = nt_blocks(r);
#define K_(V) hipLaunchKernelGGL((nt_q_kernel<V>), dim3(nb), dim3(256), 0, s, r, mask, mi, h, p, Gh, q, part, ns)
  NT_V_SWITCH(r, K_)
#undef K_
  return hipGetLastError();
}

hipError_t launch_nt_update(const NtRows& r, const uint8_t* mask, const double* h, double* Dir, double* res,
                            double* z, const double* p, const double* q, double* part, NewtonState* ns, int par,
                            hipStream_t s) {
  const int nb = nt_blocks(r);
  // p'q partials of the q kernel in part[0, nb); r'r and r'z partials into part[2 kNtBlocks, ...)
#define K_(V)                                                                                                    \
  hipLaunchKernelGGL((nt_update_kernel<V>), dim3(nb), dim3(256), 0, s, r, mask, h, Dir, res, z, p, q, part,      \
                     part + 2 * kNtBlocks, ns, par)
  NT_V_SWITCH(r, K_)
#undef K_
  return hipGetLastError();
}

hipError_t launch_nt_dir(const NtRows& r, const uint8_t* mask, const int* mi, const double* z, double* p,
                         double* Vf, double* part, NewtonState* ns, int par, int* flag, hipStream_t s) {
  if (!flag) return hipErrorInvalidValue;
  const int nb = nt_blocks(r);
#define K_(V)                                                                                                    \
  hipLaunchKernelGGL((nt_dir_kernel<V>), dim3(nb), dim3(256), 0, s, r, mask, mi, z, p, Vf, part + 2 * kNtBlocks, \
                     ns, par, flag)
  NT_V_SWITCH(r, K_)
#undef K_
  return hipGetLastError();
}

hipError_t launch_nt_slope(const NtRows& r, const double* X, const double* Dir, const double* G, const int* mi,
                           double* part, NewtonState* ns, hipStream_t s) {
  const int nb = nt_blocks(r);
#define K_(V) hipLaunchKernelGGL((nt_slope_kernel<V>), dim3(nb), dim3(256), 0, s, r, X, Dir, G, mi, part)
  NT_V_SWITCH(r, K_)
#undef K_
  hipLaunchKernelGGL((nt_sum_kernel<1>), dim3(1), dim3(256), 0, s, part, nb, ns, 0);
  return hipGetLastError();
}

hipError_t launch_nt_negrad(const NtRows& r, const double* G, const int* mi, double* Dir, hipStream_t s) {
  const int nb = nt_blocks(r);
#define K_(V) hipLaunchKernelGGL((nt_negrad_kernel<V>), dim3(nb), dim3(256), 0, s, r, G, mi, Dir)
  NT_V_SWITCH(r, K_)
#undef K_
  return hipGetLastError();
}

hipError_t launch_nt_trial(const NtRows& r, const double* X, const double* Dir, const int* mi, double alpha,
                           double* Xa, double* part, NewtonState* ns, hipStream_t s) {
  const int nb = nt_blocks(r);
#define K_(V) hipLaunchKernelGGL((nt_trial_kernel<V>), dim3(nb), dim3(256), 0, s, r, X, Dir, mi, alpha, Xa, part)
  NT_V_SWITCH(r, K_)
#undef K_
  hipLaunchKernelGGL((nt_sum_kernel<1>), dim3(1), dim3(256), 0, s, part, nb, ns, 1);
  return hipGetLastError();
}

}  // namespace pdt
