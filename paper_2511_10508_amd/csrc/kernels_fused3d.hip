// Instantiations and launchers of the 3D fused marching kernels.
#include "pf_device.h"
#include "pf_dispatch.h"

namespace pf {

// Gray-Scott and Allen-Cahn: r <= 4; Cahn-Hilliard (halo 2r): r <= 3.
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

bool plan_fused3d(const Launch &L, int64_t nx, int64_t ny, int64_t nz, int32_t clen, int tb,
                  int32_t *strips, int32_t *ow, int32_t *ytiles, int32_t *chunks, int32_t *items,
                  int32_t *blocks, int32_t *threads)
{
    bool ok = false;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        dispatch_kind(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            ok = dispatch_r3d<KIND>(L.r, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                constexpr int V = Shape<T, KIND, R>::V;
                const int owmax = tb == 2 ? Shape<T, KIND, R, 2>::OWMAX : Shape<T, KIND, R, 1>::OWMAX;
                const int h = tb == 2 ? Shape<T, KIND, R, 2>::H : Shape<T, KIND, R, 1>::H;
                const int64_t st = cdiv(nx, owmax);
                *strips = (int32_t)st;
                *ow = (int32_t)(cdiv(cdiv(nx, st), V) * V);
                *ytiles = (int32_t)cdiv(ny, kWaves3D - 2 * h);
                *chunks = (int32_t)cdiv(nz, clen);
                const int64_t it = st * (int64_t)*ytiles * *chunks;
                *items = (int32_t)it;
                *blocks = (int32_t)it;
                *threads = 64 * kWaves3D;
            });
        });
    });
    return ok;
}

hipError_t launch_fused3d(const Launch &L, const void *args, int32_t blocks, int32_t threads,
                          int red, int tb, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        dispatch_kind(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            if (tb == 2) {
                dispatch_r(L.r, TimeBlockRadii3D{}, [&](auto rc) {
                    constexpr int R = decltype(rc)::value;
                    if (red)
                        hipLaunchKernelGGL((k_step3d<T, KIND, R, true, 2>), dim3(blocks), dim3(threads), 0, s, a);
                    else
                        hipLaunchKernelGGL((k_step3d<T, KIND, R, false, 2>), dim3(blocks), dim3(threads), 0, s, a);
                    err = hipGetLastError();
                });
                return;
            }
            dispatch_r3d<KIND>(L.r, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                if (red)
                    hipLaunchKernelGGL((k_step3d<T, KIND, R, true, 1>), dim3(blocks), dim3(threads), 0, s, a);
                else
                    hipLaunchKernelGGL((k_step3d<T, KIND, R, false, 1>), dim3(blocks), dim3(threads), 0, s, a);
                err = hipGetLastError();
            });
        });
    });
    return err;
}

hipError_t launch_fused3d_batched(const Launch &L, const void *table, int32_t k, int32_t blocks,
                                  hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const BatchTable<T> &tb = *static_cast<const BatchTable<T> *>(table);
        dispatch_kind(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            dispatch_r3d<KIND>(L.r, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                hipLaunchKernelGGL((k_step3d_batched<T, KIND, R>), dim3(blocks), dim3(64 * kWaves3D), 0, s, tb, k);
                err = hipGetLastError();
            });
        });
    });
    return err;
}

}  // namespace pf
