// Band-product kernels, storage float / MFMA operands float: every column-tile class and
// both workgroup shapes (compiled on their own so that builds run in parallel).
#include "pdt_band.h"

namespace pdt {

template hipError_t launch_fx<float, float>(const ProbView&, const Bufs<float>&, SolverState*, int, hipStream_t);
template hipError_t launch_ftr<float, float>(const ProbView&, const Bufs<float>&, SolverState*, int, double,
                                           hipStream_t);

}  // namespace pdt
