// Definitions of the per-(precision, kind) 3D launchers (declared in
// pf_fused3d.h); included only by the kernels_f3d_<kind>_<precision>.hip
// files, each of which instantiates one pair.
#pragma once

#include "pf_fused3d.h"

namespace pf {

template <typename T, int KIND, int R, int TB, int RPW>
static hipError_t launch3d(const StepArgs<T> &a, int32_t blocks, int32_t threads, int red,
                           hipStream_t s)
{
    if (red)
        hipLaunchKernelGGL((k_step3d<T, KIND, R, true, TB, RPW>), dim3(blocks), dim3(threads), 0, s, a);
    else
        hipLaunchKernelGGL((k_step3d<T, KIND, R, false, TB, RPW>), dim3(blocks), dim3(threads), 0, s, a);
    return hipGetLastError();
}

// Two-pass step: the mu pass writes mu into the mu buffer through the output
// slot of field 0 (and reduces c); the update pass reads mu as field 0 and c
// as field 1 and writes c through the output slot of field 0.
template <typename T, int R>
static hipError_t launch3d_two_pass(const StepArgs<T> &a, T *mu, int32_t blocks, int32_t threads,
                                    int red, hipStream_t s)
{
    const int p = a.parity;
    StepArgs<T> a1 = a;
    a1.buf[0][p ^ 1] = mu;
    hipError_t err = launch3d<T, kCHMU, R, 1, 2>(a1, blocks, threads, red, s);
    if (err != hipSuccess) return err;
    StepArgs<T> a2 = a;
    a2.buf[0][p] = mu;
    a2.buf[1][p] = a.buf[0][p];
    a2.red = 0;
    hipLaunchKernelGGL((k_step3d<T, kCHUP, R, false, 1, 2>), dim3(blocks), dim3(threads), 0, s, a2);
    return hipGetLastError();
}

template <typename T, int KIND>
hipError_t launch_fused3d_kind(const Launch &L, const StepArgs<T> &a, int32_t blocks, int32_t threads,
                               int red, int tb, int rpw, T *mu, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    auto one = [&](auto rc, auto tbc) {
        constexpr int R = decltype(rc)::value, TB = decltype(tbc)::value;
        if constexpr (KIND == kCH && TB == 1) {
            if (mu) {
                err = launch3d_two_pass<T, R>(a, mu, blocks, threads, red, s);
                return;
            }
        }
        if constexpr (has_one_row_per_wave<T, KIND, R>()) {
            if (rpw == 1) {
                err = launch3d<T, KIND, R, TB, 1>(a, blocks, threads, red, s);
                return;
            }
        }
        if constexpr (has_four_rows_per_wave<T, KIND, R>()) {
            if (rpw == 4) {
                err = launch3d<T, KIND, R, TB, 4>(a, blocks, threads, red, s);
                return;
            }
        }
        err = launch3d<T, KIND, R, TB, 2>(a, blocks, threads, red, s);
    };
    if (tb == 2)
        dispatch_r(L.r, TimeBlockRadii3D{}, [&](auto rc) { one(rc, std::integral_constant<int, 2>{}); });
    else if (tb == 1)
        dispatch_r3d<KIND>(L.r, [&](auto rc) { one(rc, std::integral_constant<int, 1>{}); });
    return err;
}

template <typename T, int KIND>
hipError_t launch_fused3d_batched_kind(const Launch &L, const BatchTable<T> &t, int32_t k, int32_t blocks,
                                       int tb, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (tb == 2) {
        dispatch_r(L.r, TimeBlockRadii3D{}, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            constexpr int NW = Tile3D<T, KIND, R, 2, batched_rpw<KIND, R>()>::NW;
            hipLaunchKernelGGL((k_step3d_batched<T, KIND, R, 2>), dim3(blocks), dim3(64 * NW), 0, s, t, k);
            err = hipGetLastError();
        });
        return err;
    }
    dispatch_r3d<KIND>(L.r, [&](auto rc) {
        constexpr int R = decltype(rc)::value;
        constexpr int NW = Tile3D<T, KIND, R, 1, batched_rpw<KIND, R>()>::NW;
        hipLaunchKernelGGL((k_step3d_batched<T, KIND, R, 1>), dim3(blocks), dim3(64 * NW), 0, s, t, k);
        err = hipGetLastError();
    });
    return err;
}

}  // namespace pf
