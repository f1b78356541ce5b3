// Instantiations and launchers of the 3D fused marching kernels.
#include "pf_march3d.h"
#include "pf_dispatch.h"

namespace pf {

// Gray-Scott and Allen-Cahn: r <= 4; Cahn-Hilliard (halo 2r): r <= 3.  The
// direct biharmonic runs its own column-tile kernel (kernels_chd3d.hip).
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

hipError_t launch_fused3d(const Launch &L, const void *args, int32_t blocks, int32_t threads,
                          int red, int tb, int rpw, void *mu, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (!rows_per_wave_available(L, tb, rpw)) return err;
    if (mu && !(two_pass_available(L) && tb == 1 && rpw == 2)) return err;
    if (L.kind == kCHD) return launch_chd3d(L, args, blocks, threads, red, rpw, s);
    dispatch3d(L, tb, [&](auto tz, auto kc, auto rc, auto tbc) {
        using T = decltype(tz);
        constexpr int KIND = decltype(kc)::value, R = decltype(rc)::value;
        constexpr int TB = decltype(tbc)::value;
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        if constexpr (KIND == kCH && TB == 1) {
            if (mu) {
                err = launch3d_two_pass<T, R>(a, static_cast<T *>(mu), blocks, threads, red, s);
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
        const BatchTable<T> &t = *static_cast<const BatchTable<T> *>(table);
        dispatch_kind(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            if (tb == 2) {
                dispatch_r(L.r, TimeBlockRadii3D{}, [&](auto rc) {
                    constexpr int R = decltype(rc)::value;
                    constexpr int NW = Tile3D<T, KIND, R, 2, batched_rpw<KIND, R>()>::NW;
                    hipLaunchKernelGGL((k_step3d_batched<T, KIND, R, 2>), dim3(blocks), dim3(64 * NW), 0, s, t,
                                       k);
                    err = hipGetLastError();
                });
                return;
            }
            dispatch_r3d<KIND>(L.r, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                constexpr int NW = Tile3D<T, KIND, R, 1, batched_rpw<KIND, R>()>::NW;
                hipLaunchKernelGGL((k_step3d_batched<T, KIND, R, 1>), dim3(blocks), dim3(64 * NW), 0, s, t, k);
                err = hipGetLastError();
            });
        });
    });
    return err;
}

}  // namespace pf
