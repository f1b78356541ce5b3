// Radii of the 2D fused kernels and the per-(precision, kind) launchers:
// defined in pf_fused2d_kind.h and instantiated once per pair in
// kernels_f2d_<kind>_<precision>.hip, so that the pairs compile in
// parallel; kernels_fused2d.hip plans and dispatches.
#pragma once

#include "pf_dispatch.h"
#include "pf_internal.h"

namespace pf {

using Fused2DRadii = RList<1, 2, 3, 4>;
using TimeBlockRadii = RList<1, 2>;  // radii with a two-step (TB = 2) kernel

template <typename T, int KIND>
hipError_t launch_fused2d_kind(const Launch &L, const StepArgs<T> &a, int32_t blocks, int32_t threads,
                               int red, int tb, hipStream_t s);
// (not for the direct biharmonic, which the server does not take)
template <typename T, int KIND>
hipError_t launch_fused2d_batched_kind(const Launch &L, const BatchTable<T> &t, int32_t k, int32_t blocks,
                                       int tb, hipStream_t s);

}  // namespace pf
