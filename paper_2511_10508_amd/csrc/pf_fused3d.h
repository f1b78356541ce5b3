// Layout traits of the 3D fused kernels and the per-(precision, kind)
// launchers: the launchers are defined in pf_fused3d_kind.h and instantiated
// once per pair in kernels_f3d_<kind>_<precision>.hip, so that the pairs
// compile in parallel; kernels_fused3d.hip plans and dispatches.
#pragma once

#include "pf_dispatch.h"
#include "pf_march3d.h"

namespace pf {

// Gray-Scott and Allen-Cahn: r <= 4; Cahn-Hilliard (halo 2r): r <= 3.  The
// direct biharmonic runs its own kernels (kernels_chd3d.hip).
using Fused3DRadii = RList<1, 2, 3, 4>;
using Fused3DRadiiCH = RList<1, 2, 3>;

template <int KIND, typename F>
bool dispatch_r3d(int r, F &&f)
{
    if constexpr (KIND == kCH)
        return dispatch_r(r, Fused3DRadiiCH{}, f);
    else
        return dispatch_r(r, Fused3DRadii{}, f);
}

using TimeBlockRadii3D = RList<1>;  // radii with a two-step (TB = 2) 3D kernel

// One row per wave is built besides two for FP64 Allen-Cahn with r <= 2 and
// FP64 Gray-Scott with r = 1, where it measures faster (and is the default).
// Four rows per wave (8-wave workgroups: two per CU at up to 128 registers,
// up to 256 registers with one; 12 waves for Cahn-Hilliard with r = 3) for
// Cahn-Hilliard and Model C, Gray-Scott
// with r >= 2 and Allen-Cahn with r = 4: an autotuner candidate, and the
// default where two rows per wave would spill hundreds of bytes a lane.
template <typename T, int KIND, int R>
constexpr bool has_one_row_per_wave()
{
    return std::is_same<T, double>::value && ((KIND == kAC && R <= 2) || (KIND == kGS && R == 1));
}
template <typename T, int KIND, int R>
constexpr bool has_four_rows_per_wave()
{
    return KIND == kCH || KIND == kMC || (KIND == kGS && R >= 2) || (KIND == kAC && R == 4);
}

template <typename T, int KIND>
hipError_t launch_fused3d_kind(const Launch &L, const StepArgs<T> &a, int32_t blocks, int32_t threads,
                               int red, int tb, int rpw, T *mu, hipStream_t s);
template <typename T, int KIND>
hipError_t launch_fused3d_batched_kind(const Launch &L, const BatchTable<T> &t, int32_t k, int32_t blocks,
                                       int tb, hipStream_t s);

}  // namespace pf
