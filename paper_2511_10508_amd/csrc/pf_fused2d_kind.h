// Definitions of the per-(precision, kind) 2D launchers (declared in
// pf_fused2d.h); included only by the kernels_f2d_<kind>_<precision>.hip
// files, each of which instantiates one pair.
#pragma once

#include "pf_fused2d.h"
#include "pf_march2d.h"

namespace pf {

template <typename T, int KIND>
hipError_t launch_fused2d_kind(const Launch &L, const StepArgs<T> &a, int32_t blocks, int32_t threads,
                               int red, int tb, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (tb == 2) {
        if constexpr (KIND != kCHD) {  // the direct biharmonic has no two-step kernel
            dispatch_r(L.r, TimeBlockRadii{}, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                if (red)
                    hipLaunchKernelGGL((k_step2d<T, KIND, R, true, 2>), dim3(blocks), dim3(threads), 0, s, a);
                else
                    hipLaunchKernelGGL((k_step2d<T, KIND, R, false, 2>), dim3(blocks), dim3(threads), 0, s, a);
                err = hipGetLastError();
            });
        }
        return err;
    }
    dispatch_r(L.r, Fused2DRadii{}, [&](auto rc) {
        constexpr int R = decltype(rc)::value;
        if (red)
            hipLaunchKernelGGL((k_step2d<T, KIND, R, true, 1>), dim3(blocks), dim3(threads), 0, s, a);
        else
            hipLaunchKernelGGL((k_step2d<T, KIND, R, false, 1>), dim3(blocks), dim3(threads), 0, s, a);
        err = hipGetLastError();
    });
    return err;
}

template <typename T, int KIND>
hipError_t launch_fused2d_batched_kind(const Launch &L, const BatchTable<T> &t, int32_t k, int32_t blocks,
                                       int tb, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (tb == 2) {
        dispatch_r(L.r, TimeBlockRadii{}, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            hipLaunchKernelGGL((k_step2d_batched<T, KIND, R, 2>), dim3(blocks), dim3(64 * kWaves2D), 0, s, t, k);
            err = hipGetLastError();
        });
        return err;
    }
    dispatch_r(L.r, Fused2DRadii{}, [&](auto rc) {
        constexpr int R = decltype(rc)::value;
        hipLaunchKernelGGL((k_step2d_batched<T, KIND, R, 1>), dim3(blocks), dim3(64 * kWaves2D), 0, s, t, k);
        err = hipGetLastError();
    });
    return err;
}

}  // namespace pf
