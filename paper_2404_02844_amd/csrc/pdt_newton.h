// Row kernels of the two-stage two-metric projected truncated Newton method (App. B,
// Algorithms 1-3).  The Hessian products of its conjugate-gradient solves are the band
// kernels of pdt_band.h (forward product without the data, then the transposed product
// with the regulariser term); everything else is row-local and lives here.
//
// Per-entry codes of the two-metric system (mask, [M][Npad] bytes):
//   0  free: coupled through the Hessian;
//   1  bound (the set I of Eq. 2metric_I): only the Hessian diagonal acts on it;
//   2  inactive: a padding column, or in stage 2 the eliminated row maximum m(i).
// Stage 2 works in the reduced variables: a vector v of them (zero at m(i)) stands for
// the change T v of Pi with (T v)[i][m(i)] = -sum_{n != m(i)} v[i][n].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdt {

// Device-resident scalars of one conjugate-gradient solve.
struct NewtonState {
  double rz[2];     // r . z of the current residual (iteration k keeps it in rz[k % 2])
  double nr0;       // ||r_0||
  double rtol;      // stop at ||r|| <= rtol ||r_0||
  double out[4];    // sums handed to the host
  int cg_iter;      // CG iterations started
  int cg_max;
  int cg_done;
  int pad_;
};

constexpr int kNtBlocks = 1024;  // fixed grid of the row kernels: reductions add in one order

struct NtRows {
  int M, N, Npad, stage;
};

hipError_t launch_nt_measure(const NtRows& r, const double* X, const double* G, double* part, NewtonState* ns,
                             hipStream_t s);
hipError_t launch_nt_prep(const NtRows& r, const double* X, const double* G, const double* h, double eps,
                          uint8_t* mask, int* mi, double* res, double* z, double* p, double* Vf, double* Dir,
                          double* part, NewtonState* ns, double rtol, int cg_max, hipStream_t s);
hipError_t launch_nt_q(const NtRows& r, const uint8_t* mask, const int* mi, const double* h, const double* p,
                       const double* Gh, double* q, double* part, NewtonState* ns, hipStream_t s);
// part: [4 kNtBlocks] (p'q partials first, r'r and r'z partials from 2 kNtBlocks on);
// par = CG iteration % 2; flag: device address of a host-mapped int that the direction
// kernel sets to 1 once the solve has stopped, else 0
hipError_t launch_nt_update(const NtRows& r, const uint8_t* mask, const double* h, double* Dir, double* res,
                            double* z, const double* p, const double* q, double* part, NewtonState* ns, int par,
                            hipStream_t s);
hipError_t launch_nt_dir(const NtRows& r, const uint8_t* mask, const int* mi, const double* z, double* p,
                         double* Vf, double* part, NewtonState* ns, int par, int* flag, hipStream_t s);
hipError_t launch_nt_slope(const NtRows& r, const double* X, const double* Dir, const double* G, const int* mi,
                           double* part, NewtonState* ns, hipStream_t s);
hipError_t launch_nt_negrad(const NtRows& r, const double* G, const int* mi, double* Dir, hipStream_t s);
hipError_t launch_nt_trial(const NtRows& r, const double* X, const double* Dir, const int* mi, double alpha,
                           double* Xa, double* part, NewtonState* ns, hipStream_t s);

}  // namespace pdt
