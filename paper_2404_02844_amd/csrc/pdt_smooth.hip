// Long-range smoothing of a POVM (Sec. 3.2, Eq. smoothing): row i >= skip becomes the
// mean of rows i - h .. i + h, h = min(floor(i / divisor), M - 1 - i) (a window centred
// on i that shrinks symmetrically at the top of the range); rows below skip are copied.
//
// Window sums are differences of column prefix sums S[i][n] = sum_{k < i} Pi[k][n],
// carried as compensated pairs (hi, lo) (Neumaier's running sum with Knuth's TwoSum), so
// that a difference keeps the accuracy of the window sum itself rather than of the
// prefix sums, whose magnitude reaches the column sum (~1e4 for a million rows):
//   1. per block of kRowsPerBlk rows, its compensated column sums;
//   2. an exclusive compensated scan of those block sums down each column (a wave per
//      column, 64 blocks per step);
//   3. the in-block prefixes, written as (S_hi, S_lo) (M + 1 rows);
//   4. every output row from two rows of S.
// Each pass streams the [M][N] array once (HBM-bound).  Step 4 reads only S and its own
// entry, so the output may overwrite the input.
#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>
#include <string>

#include "pdt.h"
#include "pdt_internal.h"

namespace pdt {

namespace {

constexpr int kRowsPerBlk = 256;

// hi + lo += x, with the rounding error of the high part kept in lo
__device__ __forceinline__ void comp_add(double& hi, double& lo, double x) {
  const double s = hi + x;
  const double bb = s - hi;
  lo += (hi - (s - bb)) + (x - bb);
  hi = s;
}

__global__ __launch_bounds__(256) void smooth_blocksum_kernel(const double* Pi, long long M, int N, long long nblk,
                                                              double* Bh, double* Bl) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= nblk * N) return;
  const long long b = t / N;
  const int n = (int)(t % N);
  const long long r0 = b * kRowsPerBlk;
  const long long r1 = r0 + kRowsPerBlk < M ? r0 + kRowsPerBlk : M;
  double hi = 0.0, lo = 0.0;
  for (long long r = r0; r < r1; ++r) comp_add(hi, lo, Pi[r * N + n]);
  Bh[b * N + n] = hi;
  Bl[b * N + n] = lo;
}

// (hi, lo) += (h2, l2): one compensated pair added to another
__device__ __forceinline__ void pair_add(double& hi, double& lo, double h2, double l2) {
  comp_add(hi, lo, h2);
  lo += l2;
}

// Exclusive compensated scan of the block sums down each column, one wave per column:
// 64 blocks per step, scanned across the lanes (Hillis-Steele, earlier blocks added to
// later ones), on top of the carry of the steps before.
__global__ __launch_bounds__(256) void smooth_scan_kernel(double* Bh, double* Bl, long long nblk, int N) {
  const int lane = threadIdx.x & 63;
  const int n = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= N) return;
  double ch = 0.0, cl = 0.0;  // sum of the blocks before this step
  for (long long b0 = 0; b0 < nblk; b0 += 64) {
    const long long b = b0 + lane;
    double ih = 0.0, il = 0.0;
    if (b < nblk) {
      ih = Bh[b * N + n];
      il = Bl[b * N + n];
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double oh = __shfl_up(ih, off, 64), ol = __shfl_up(il, off, 64);
      if (lane >= off) {
        double h = oh, l = ol;
        pair_add(h, l, ih, il);
        ih = h;
        il = l;
      }
    }
    // exclusive prefix of this lane's block within the step, then the carry
    double eh = __shfl_up(ih, 1, 64), el = __shfl_up(il, 1, 64);
    if (lane == 0) eh = el = 0.0;
    double h = ch, l = cl;
    pair_add(h, l, eh, el);
    if (b < nblk) {
      Bh[b * N + n] = h;
      Bl[b * N + n] = l;
    }
    pair_add(ch, cl, __shfl(ih, 63, 64), __shfl(il, 63, 64));
  }
}

__global__ __launch_bounds__(256) void smooth_prefix_kernel(const double* Pi, long long M, int N, long long nblk,
                                                            const double* Bh, const double* Bl, double* Sh,
                                                            double* Sl) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= nblk * N) return;
  const long long b = t / N;
  const int n = (int)(t % N);
  const long long r0 = b * kRowsPerBlk;
  const long long r1 = r0 + kRowsPerBlk < M ? r0 + kRowsPerBlk : M;
  double hi = Bh[b * N + n], lo = Bl[b * N + n];
  for (long long r = r0; r < r1; ++r) {
    Sh[r * N + n] = hi;
    Sl[r * N + n] = lo;
    comp_add(hi, lo, Pi[r * N + n]);
  }
  if (r1 == M) {
    Sh[M * N + n] = hi;
    Sl[M * N + n] = lo;
  }
}

__global__ __launch_bounds__(256) void smooth_apply_kernel(const double* Pi, const double* Sh, const double* Sl,
                                                           long long M, int N, int divisor, long long skip,
                                                           double* out) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= M * N) return;
  const long long i = t / N;
  const int n = (int)(t % N);
  if (i < skip) {
    out[t] = Pi[t];
    return;
  }
  const long long hw = i / divisor;
  const long long h = hw < M - 1 - i ? hw : M - 1 - i;
  const long long a = (i + h + 1) * N + n, c = (i - h) * N + n;
  const double w = (Sh[a] - Sh[c]) + (Sl[a] - Sl[c]);
  out[t] = w / (double)(2 * h + 1);
}

unsigned grid_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

long long smooth_scratch_doubles(long long M, int N) {
  const long long nblk = (M + kRowsPerBlk - 1) / kRowsPerBlk;
  return 2 * ((M + 1) * N + nblk * N);
}

hipError_t launch_smooth_rows(const double* Pi, double* out, long long M, int N, int divisor, long long skip,
                              double* scratch, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const long long nblk = (M + kRowsPerBlk - 1) / kRowsPerBlk;
  double* Sh = scratch;
  double* Sl = Sh + (M + 1) * N;
  double* Bh = Sl + (M + 1) * N;
  double* Bl = Bh + nblk * N;
  hipLaunchKernelGGL(smooth_blocksum_kernel, dim3(grid_for(nblk * N)), dim3(256), 0, s, Pi, M, N, nblk, Bh, Bl);
  hipLaunchKernelGGL(smooth_scan_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, Bh, Bl, nblk, N);
  hipLaunchKernelGGL(smooth_prefix_kernel, dim3(grid_for(nblk * N)), dim3(256), 0, s, Pi, M, N, nblk, Bh, Bl, Sh,
                     Sl);
  hipLaunchKernelGGL(smooth_apply_kernel, dim3(grid_for(M * N)), dim3(256), 0, s, Pi, Sh, Sl, M, N, divisor, skip,
                     out);
  return hipGetLastError();
}

}  // namespace pdt

// ---------------------------------------------------------------------------------------
// Allocation-free smoothing: the same kernels on a fixed device array instead of memory
// allocated per call.  Each GPU the library runs on holds its own copy of the array
// until the process ends; in host code the array's name is not a device address, so
// its address is looked up once per device and only that address is handed to kernels.
// ---------------------------------------------------------------------------------------
constexpr long long kNoAllocScratchDoubles = PDT_SMOOTH_NOALLOC_MAX_DOUBLES;  // 64 MiB

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (the current device), looked up on
// the first call on that device.
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

pdt_status pdt_smooth_rows_noalloc(const double* Pi, double* out, int64_t M, int64_t N, int32_t divisor,
                                   int64_t skip, void* stream) {
  if (!Pi || !out) {
    pdt::set_last_error("Pi and out must not be NULL");
    return PDT_ERR_INVALID_ARG;
  }
  if (M < 1 || N < 1 || M * N > (int64_t)INT_MAX) {
    pdt::set_last_error("need M, N >= 1, M*N < 2^31");
    return PDT_ERR_INVALID_ARG;
  }
  if (divisor < 1 || skip < 0) {
    pdt::set_last_error("need divisor >= 1, skip >= 0");
    return PDT_ERR_INVALID_ARG;
  }
  const long long need = pdt::smooth_scratch_doubles((long long)M, (int)N);
  if (need > kNoAllocScratchDoubles) {
    pdt::set_last_error(("scratch of " + std::to_string(need) + " doubles exceeds the fixed " +
                    std::to_string(kNoAllocScratchDoubles) + " (2 (M + 1 + ceil(M / 256)) N must be <= that)")
                       .c_str());
    return PDT_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* buf = nullptr;
  hipError_t e = scratch_address(&buf);
  if (e == hipSuccess) e = pdt::launch_smooth_rows(Pi, out, (long long)M, (int)N, (int)divisor, (long long)skip, buf, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    pdt::set_last_error(hipGetErrorString(e));
    return PDT_ERR_DEVICE;
  }
  pdt::set_last_error("");
  return PDT_OK;
}

}  // extern "C"
