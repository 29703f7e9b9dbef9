// Batched band-product kernels (work lists of (instance, tile) items), FP64 and FP32.
#include "pdt_band.h"

namespace pdt {

template hipError_t launch_fx_batch<double, double>(int, int, const BatchInst<double>*, const int2*, int, int,
                                                    hipStream_t);
template hipError_t launch_fx_batch<float, float>(int, int, const BatchInst<float>*, const int2*, int, int,
                                                  hipStream_t);
template hipError_t launch_ftr_batch<double, double>(int, int, const BatchInst<double>*, const int2*, int, int,
                                                     hipStream_t);
template hipError_t launch_ftr_batch<float, float>(int, int, const BatchInst<float>*, const int2*, int, int,
                                                   hipStream_t);

}  // namespace pdt
