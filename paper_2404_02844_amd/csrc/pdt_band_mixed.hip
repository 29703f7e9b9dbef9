// Band-product kernels, storage double / MFMA operands float: every column-tile class and
// both workgroup shapes (compiled on their own so that builds run in parallel).
#include "pdt_band.h"

namespace pdt {

template hipError_t launch_fx<double, float>(const ProbView&, const Bufs<double>&, SolverState*, int, hipStream_t);
template hipError_t launch_ftr<double, float>(const ProbView&, const Bufs<double>&, SolverState*, int, double,
                                           hipStream_t);

}  // namespace pdt
