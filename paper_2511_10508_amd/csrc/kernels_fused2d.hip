// Planning and dispatch of the 2D fused marching kernels (their launchers
// are instantiated per precision and kind in kernels_f2d_*.hip).
#include "pf_device.h"
#include "pf_fused2d.h"

namespace pf {

bool time_block_available(const Launch &L)
{
    if (L.ndim == 1) return L.r >= 1 && L.r <= 4;  // every fused 1D kernel has a two-step form
    if (L.kind == kCHD) return false;
    return (L.ndim == 2 && (L.r == 1 || L.r == 2)) || (L.ndim == 3 && L.r == 1);
}

bool plan_fused2d(const Launch &L, int64_t nx, int64_t ny, int32_t clen, int tb, int32_t *strips,
                  int32_t *ow, int32_t *chunks, int32_t *items, int32_t *blocks, int32_t *threads)
{
    bool ok = false;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        dispatch_kind_all(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            ok = dispatch_r(L.r, Fused2DRadii{}, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                const int owmax = tb == 2 ? Shape<T, KIND, R, 2>::OWMAX : Shape<T, KIND, R, 1>::OWMAX;
                constexpr int V = Shape<T, KIND, R>::V;
                const int64_t st = cdiv(nx, owmax);
                int64_t w = cdiv(cdiv(nx, st), V) * V;
                *strips = (int32_t)st;
                *ow = (int32_t)w;
                *chunks = (int32_t)cdiv(ny, clen);
                const int64_t it = st * *chunks;
                *items = (int32_t)it;
                *blocks = (int32_t)cdiv(it, kWaves2D);
                *threads = 64 * kWaves2D;
            });
        });
    });
    return ok;
}

hipError_t launch_fused2d(const Launch &L, const void *args, int32_t blocks, int32_t threads,
                          int red, int tb, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        dispatch_kind_all(L.kind, [&](auto kc) {
            err = launch_fused2d_kind<T, decltype(kc)::value>(L, *static_cast<const StepArgs<T> *>(args), blocks,
                                                              threads, red, tb, s);
        });
    });
    return err;
}

hipError_t launch_fused2d_batched(const Launch &L, const void *table, int32_t k, int32_t blocks,
                                  int tb, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (tb == 2 && !time_block_available(L)) return err;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        dispatch_kind(L.kind, [&](auto kc) {
            err = launch_fused2d_batched_kind<T, decltype(kc)::value>(
                L, *static_cast<const BatchTable<T> *>(table), k, blocks, tb, s);
        });
    });
    return err;
}

}  // namespace pf
