// 2D fused kernels of Cahn-Hilliard, FP32 storage: one
// (precision, kind) pair of the launchers in pf_fused2d_kind.h, instantiated in
// a file of its own.
#include "pf_fused2d_kind.h"

namespace pf {

template hipError_t launch_fused2d_kind<float, kCH>(const Launch &, const StepArgs<float> &, int32_t, int32_t, int,
                                                 int, hipStream_t);
template hipError_t launch_fused2d_batched_kind<float, kCH>(const Launch &, const BatchTable<float> &, int32_t,
                                                         int32_t, int, hipStream_t);

}  // namespace pf
