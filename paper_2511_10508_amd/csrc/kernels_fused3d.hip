// Planning and dispatch of the 3D fused marching kernels (their launchers
// are instantiated per precision and kind in kernels_f3d_*.hip).
#include "pf_fused3d.h"

namespace pf {

// Calls f(T, KIND, R, TB) for the instantiated 3D kernel of L and tb.
template <typename F>
bool dispatch3d(const Launch &L, int tb, F &&f)
{
    bool ok = false;
    dispatch_prec(L.fp32, [&](auto tz) {
        dispatch_kind(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            if (tb == 2) {
                ok = dispatch_r(L.r, TimeBlockRadii3D{}, [&](auto rc) {
                    f(tz, kc, rc, std::integral_constant<int, 2>{});
                });
            }
            else if (tb == 1)
                ok = dispatch_r3d<KIND>(L.r, [&](auto rc) {
                    f(tz, kc, rc, std::integral_constant<int, 1>{});
                });
        });
    });
    return ok;
}

bool rows_per_wave_available(const Launch &L, int tb, int rpw)
{
    if (L.kind == kCHD) return chd3d_available(L) && tb == 1 && (rpw == 2 || rpw == 4);
    bool has1 = false, has4 = false;
    if (!dispatch3d(L, tb, [&](auto tz, auto kc, auto rc, auto) {
            has1 = has_one_row_per_wave<decltype(tz), decltype(kc)::value, decltype(rc)::value>();
            has4 = has_four_rows_per_wave<decltype(tz), decltype(kc)::value, decltype(rc)::value>();
        }))
        return false;
    return rpw == 2 || (rpw == 1 && has1) || (rpw == 4 && has4);
}

int rows_per_wave_batched(const Launch &L)
{
    int rpw = 2;
    dispatch_kind(L.kind, [&](auto kc) {
        dispatch_r3d<decltype(kc)::value>(L.r, [&](auto rc) {
            rpw = batched_rpw<decltype(kc)::value, decltype(rc)::value>();
        });
    });
    return rpw;
}

int rows_per_wave_default(const Launch &L, int tb)
{
    if (rows_per_wave_available(L, tb, 1)) return 1;
    // four rows where two would spill hundreds of bytes a lane (Gray-Scott and
    // Model C with r >= 3: 3-6x faster on 512^3) or 88 (FP32 Cahn-Hilliard
    // with r = 3, whose 48-row tiles of 12 waves run 1.5x faster on 512^3);
    // the direct biharmonic's march (its other layout is the column tiles:
    // 1.0-2.8x slower on 512^3)
    const bool heavy = ((L.kind == kGS || L.kind == kMC) && L.r >= 3) || (L.kind == kCH && L.r == 3 && L.fp32) ||
                       L.kind == kCHD;
    return heavy && rows_per_wave_available(L, tb, 4) ? 4 : 2;
}

bool two_pass_available(const Launch &L)
{
    return L.ndim == 3 && L.kind == kCH && L.r >= 1 && L.r <= 3;
}

bool plan_fused3d(const Launch &L, int64_t nx, int64_t ny, int64_t nz, int32_t clen, int tb,
                  int rpw, int passes, int32_t *strips, int32_t *ow, int32_t *ytiles,
                  int32_t *chunks, int32_t *items, int32_t *blocks, int32_t *threads)
{
    if (passes == 2 && !(two_pass_available(L) && tb == 1 && rpw == 2)) return false;
    if (!rows_per_wave_available(L, tb, rpw)) return false;
    if (L.kind == kCHD)
        return passes == 1 &&
               plan_chd3d(L, nx, ny, nz, clen, rpw, strips, ow, ytiles, chunks, items, blocks, threads);
    return dispatch3d(L, tb, [&](auto tz, auto kc, auto rc, auto tbc) {
        using T = decltype(tz);
        constexpr int KIND = decltype(kc)::value, R = decltype(rc)::value;
        constexpr int TB = decltype(tbc)::value;
        auto plan = [&](auto tl) {
            using TL = decltype(tl);
            const int64_t st = cdiv(nx, TL::OWMAX);
            *strips = (int32_t)st;
            *ow = (int32_t)(cdiv(cdiv(nx, st), TL::V) * TL::V);
            *ytiles = (int32_t)cdiv(ny, TL::NR - 2 * TL::H);
            *chunks = (int32_t)cdiv(nz, clen);
            const int64_t it = st * (int64_t)*ytiles * *chunks;
            *items = (int32_t)it;
            *blocks = (int32_t)it;
            *threads = 64 * TL::NW;
        };
        if constexpr (has_one_row_per_wave<T, KIND, R>()) {
            if (rpw == 1) {
                plan(Tile3D<T, KIND, R, TB, 1>{});
                return;
            }
        }
        if constexpr (has_four_rows_per_wave<T, KIND, R>()) {
            if (rpw == 4) {
                plan(Tile3D<T, KIND, R, TB, 4>{});
                return;
            }
        }
        if constexpr (KIND == kCH && TB == 1) {
            if (passes == 2) {  // both passes share the tiles of one radius-r stage
                plan(Tile3D<T, kCHMU, R, 1, 2>{});
                return;
            }
        }
        plan(Tile3D<T, KIND, R, TB, 2>{});
    });
}

hipError_t launch_fused3d(const Launch &L, const void *args, int32_t blocks, int32_t threads,
                          int red, int tb, int rpw, void *mu, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (!rows_per_wave_available(L, tb, rpw)) return err;
    if (mu && !(two_pass_available(L) && tb == 1 && rpw == 2)) return err;
    if (L.kind == kCHD) return launch_chd3d(L, args, blocks, threads, red, rpw, s);
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        dispatch_kind(L.kind, [&](auto kc) {
            err = launch_fused3d_kind<T, decltype(kc)::value>(L, *static_cast<const StepArgs<T> *>(args), blocks,
                                                              threads, red, tb, rpw, static_cast<T *>(mu), s);
        });
    });
    return err;
}

hipError_t launch_fused3d_batched(const Launch &L, const void *table, int32_t k, int32_t blocks,
                                  int tb, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (tb == 2 && !time_block_available(L)) return err;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        dispatch_kind(L.kind, [&](auto kc) {
            err = launch_fused3d_batched_kind<T, decltype(kc)::value>(
                L, *static_cast<const BatchTable<T> *>(table), k, blocks, tb, s);
        });
    });
    return err;
}

}  // namespace pf
