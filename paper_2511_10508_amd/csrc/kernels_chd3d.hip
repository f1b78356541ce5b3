// Cahn-Hilliard with the direct biharmonic stencil on 3D grids, one z-marching
// pass (the fused family's 3D kernels for PF_BIHARMONIC_DIRECT), in two tile
// layouts: the 3D march of the other models with four rows per wave
// (k_step3d<T, kCHD, r, RED, 1, 4>, pf_march3d.h: halo r + 1, x-neighbours
// by lane shifts, the default) and the column tiles below (layout 2).
//
// c' = c + dt (sum_a D2_a mu_a - sum_a D4_a c), mu_a = g - sum_{b != a} D2_b c,
// g = c2 c^3 - c1 c.  Column tiles: a workgroup owns an x-y tile of output columns plus a
// halo of 2r and marches along z over a chunk of planes, one column per
// thread.  When plane t of c arrives:
//   mu_x, mu_y and mu_z at plane t - r (tile + r halo): x-y neighbours of c
//   from its LDS plane, z neighbours from the thread's z-window of c;
//   the update at q = t - 2r: the D2 pairs of mu_x (x) and mu_y (y) and the
//   D4 pairs of c (x, y) from LDS planes, those of mu_z and of c (z) from
//   z-windows in registers;
// so no mu reaches HBM and c is read once and written once per step (up to
// the re-read tile halos), with the loads two planes ahead in alternating
// register sets and one barrier per plane (double-buffered LDS).  Every value
// is formed with the per-site kernel's functions in its order (pairs x,
// then y, then z), so the fields are bitwise those of the two-pass per-site
// kernel.  The fused reductions (mass, energy, non-finite count of the state
// at the start of the step) follow the other fused kernels: one compensated
// partial per wave, in the slots of 16 waves per work item.
#include "pf_dispatch.h"
#include "pf_march3d.h"

namespace pf {

namespace {

// Output columns of a tile: 32 x 16; 16 x 16 at r = 3, where the 2r halo
// would need more than 1024 threads, and 16 x 8 for FP64 at r = 3, whose
// windows need more than the 128 registers a lane of a 13-wave workgroup
// has (a 9-wave workgroup gets 168).
template <typename T, int R>
struct CHD3Tile {
    static constexpr int TX = R == 3 ? 16 : 32;
    static constexpr int TY = (R == 3 && std::is_same<T, double>::value) ? 8 : 16;
    static constexpr int G = 2 * R;                      // staged halo (>= r + 1 for the D4 pairs)
    static constexpr int LX = TX + 2 * G, LY = TY + 2 * G;
    static constexpr int NT = LX * LY;                   // columns (threads that load)
    static constexpr int NW = (NT + 63) / 64;            // waves
    static constexpr int THREADS = NW * 64;
    static constexpr int ZC = 3 * R + 2;                 // z-window of c
    static constexpr int ZM = 2 * R + 1;                 // z-window of mu_z
    static constexpr int ZA = R + 1;                     // z-windows of mu_x, mu_y
    static_assert(NW <= kWaves3D, "reduction slots hold 16 waves per item");
};

// LDS planes per buffer: c at the mu plane, then c, mu_x and mu_y at the
// update plane.
enum { kCp = 0, kCq = 1, kMx = 2, kMy = 3, kCPlanes = 4 };

template <typename T, int R, bool RED>
__global__ void __launch_bounds__((CHD3Tile<T, R>::THREADS)) k_chd3d(StepArgs<T> a)
{
    using TL = CHD3Tile<T, R>;
    constexpr int G = TL::G, LX = TL::LX, LY = TL::LY, ZC = TL::ZC, ZM = TL::ZM, ZA = TL::ZA;
    constexpr int R4 = R + 1;
    __shared__ T L[2][kCPlanes][LY][LX];

    const int32_t item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= a.items) return;  // uniform over the workgroup
    const int32_t tx = item % a.strips, rest = item / a.strips;
    const int32_t ty = rest % a.ytiles, chunk = rest / a.ytiles;
    const int32_t nz = (int32_t)a.nz;
    const int32_t z0 = chunk * a.clen, z1 = min(z0 + a.clen, nz);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool col = tid < TL::NT;  // threads past the tile's columns only take part in barriers
    const int lx = col ? tid % LX : 0, ly = col ? tid / LX : 0;
    const int64_t x0 = (int64_t)tx * TL::TX, y0 = (int64_t)ty * TL::TY;
    const int64_t coff = wrap_any(y0 - G + ly, a.ny) * a.pitch + wrap_any(x0 - G + lx, a.nx);
    const bool mu_col = col && lx >= R && lx < LX - R && ly >= R && ly < LY - R;
    const bool out_col = col && lx >= G && lx < LX - G && ly >= G && ly < LY - G &&
                         x0 + lx - G < a.nx && y0 + ly - G < a.ny;
    const int par = a.parity;
    const T *__restrict__ in = a.buf[0][par];
    T *__restrict__ out = a.buf[0][par ^ 1];

    // z-windows: cw[i] holds c at plane t - (3r + 1) + i; mz[i] mu_z at plane
    // t - 3r + i and mx / my[i] mu_x / mu_y at plane t - 2r + i once this
    // plane's mu is shifted in (one plane older before).  pc: c of the next
    // two planes in flight, in two alternating register sets.
    T cw[ZC], mz[ZM], mx[ZA], my[ZA], pc[2];
#pragma unroll
    for (int i = 0; i < ZC; ++i) cw[i] = T(0);
#pragma unroll
    for (int i = 0; i < ZM; ++i) mz[i] = T(0);
#pragma unroll
    for (int i = 0; i < ZA; ++i) mx[i] = my[i] = T(0);
    RedState red;
    const int32_t t0 = z0 - G, tend = z1 + G;
    auto load = [&](int32_t t, T &v) { v = col ? in[(int64_t)wrap32(t, nz) * a.plane + coff] : T(0); };
    load(t0, pc[0]);
    load(t0 + 1, pc[1]);

    auto phase = [&](int32_t t, auto parc) {
        constexpr int PH = decltype(parc)::value;
        const int32_t age = t - t0;
#pragma unroll
        for (int i = 0; i < ZC - 1; ++i) cw[i] = cw[i + 1];
        cw[ZC - 1] = pc[PH];
        load(t + 2, pc[PH]);
        // centre planes: c at t - r (index 2r + 1) and at q = t - 2r (index r + 1);
        // mu_x, mu_y at q (index 1 until this plane's mu is shifted in)
        auto &B = L[t & 1];
        if (col) {
            B[kCp][ly][lx] = cw[2 * R + 1];
            B[kCq][ly][lx] = cw[R + 1];
            B[kMx][ly][lx] = mx[1];
            B[kMy][ly][lx] = my[1];
        }
        __syncthreads();
        // mu_x, mu_y, mu_z of plane t - r
        T nx_ = T(0), ny_ = T(0), nz_ = T(0);
        if (age >= 2 * R && mu_col) {
            constexpr int C = 2 * R + 1;
            const T c0 = cw[C];
            T Sx[R], Sy[R], Sz[R];
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                const T px = B[kCp][ly][lx + j] + B[kCp][ly][lx - j];
                const T py = B[kCp][ly + j][lx] + B[kCp][ly - j][lx];
                const T pz = cw[C + j] + cw[C - j];
                Sx[j - 1] = py + pz;  // mu_x: the pairs of the other axes, y then z
                Sy[j - 1] = px + pz;
                Sz[j - 1] = px + py;
            }
            nx_ = ch_mu<T, R>(a, c0, Sx, c0 * T(4));
            ny_ = ch_mu<T, R>(a, c0, Sy, c0 * T(4));
            nz_ = ch_mu<T, R>(a, c0, Sz, c0 * T(4));
        }
#pragma unroll
        for (int i = 0; i < ZM - 1; ++i) mz[i] = mz[i + 1];
        mz[ZM - 1] = nz_;
#pragma unroll
        for (int i = 0; i < ZA - 1; ++i) {
            mx[i] = mx[i + 1];
            my[i] = my[i + 1];
        }
        mx[ZA - 1] = nx_;
        my[ZA - 1] = ny_;
        // the update of plane q = t - 2r
        if (age >= 4 * R && out_col) {
            constexpr int C = R + 1;
            const int32_t q = t - 2 * R;
            const T c0 = cw[C];
            T Sm[R], S4[R4];
#pragma unroll
            for (int j = 1; j <= R; ++j)
                Sm[j - 1] = ((B[kMx][ly][lx + j] + B[kMx][ly][lx - j]) + (B[kMy][ly + j][lx] + B[kMy][ly - j][lx])) +
                            (mz[R + j] + mz[R - j]);
#pragma unroll
            for (int j = 1; j <= R4; ++j)
                S4[j - 1] = ((B[kCq][ly][lx + j] + B[kCq][ly][lx - j]) + (B[kCq][ly + j][lx] + B[kCq][ly - j][lx])) +
                            (cw[C + j] + cw[C - j]);
            const T musum = (B[kMx][ly][lx] + B[kMy][ly][lx]) + mz[R];
            out[(int64_t)wrap32(q, nz) * a.plane + coff] = chd_update<T, R>(a, c0, Sm, musum * T(2), S4, c0 * T(6));
            if constexpr (RED) {
                const double x = (double)c0;
                double e;
                if constexpr (std::is_same<T, double>::value) {
                    // the full chemical potential: (mu_x + mu_y + mu_z - g) / 2
                    e = energy_from_mu(a.c2, x, 0.5 * (musum - chd_g(a, c0)));
                } else {
                    double Pn[R];
#pragma unroll
                    for (int j = 1; j <= R; ++j)
                        Pn[j - 1] = ((double)B[kCq][ly][lx + j] + (double)B[kCq][ly + j][lx]) + (double)cw[C + j];
                    e = energy_by_parts<R>(a.c1, a.c2, a.w64, 3.0 * a.w64sum, x, Pn);
                }
                if (!(finite_val(x) && finite_val(e))) red.bad += finite_val(x) ? 0u : 1u;
                acc_add(red.q0, x);
                acc_add(red.q1, e);
            }
        }
    };
    // two planes per iteration: the register sets alternate at compile time
    // (the trip count is uniform over the workgroup, so every thread reaches
    // the same barriers)
    int32_t t = t0;
    for (; t + 1 < tend; t += 2) {
        phase(t, std::integral_constant<int, 0>{});
        phase(t + 1, std::integral_constant<int, 1>{});
    }
    if (t < tend) phase(t, std::integral_constant<int, 0>{});
    if constexpr (RED) {
        const int64_t slot0 = (int64_t)item * kWaves3D;
        red_flush(red, a.part, a.pstride, slot0 + w, lane);
        if constexpr (TL::NW < kWaves3D) {
            constexpr int M = kWaves3D - TL::NW;  // the slots of waves this tile does not have
            if (tid < kNumQ * M)
                a.part[(int64_t)(tid / M) * a.pstride + slot0 + TL::NW + tid % M] = make_double2(0.0, 0.0);
        }
    }
}

template <typename T, int R>
hipError_t launch_chd3d_r(const StepArgs<T> &a, int32_t blocks, int red, hipStream_t s)
{
    if (red)
        hipLaunchKernelGGL((k_chd3d<T, R, true>), dim3(blocks), dim3(CHD3Tile<T, R>::THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((k_chd3d<T, R, false>), dim3(blocks), dim3(CHD3Tile<T, R>::THREADS), 0, s, a);
    return hipGetLastError();
}

}  // namespace

bool chd3d_available(const Launch &L) { return L.kind == kCHD && L.ndim == 3 && L.r >= 1 && L.r <= 3; }

bool plan_chd3d(const Launch &L, int64_t nx, int64_t ny, int64_t nz, int32_t clen, int rpw,
                int32_t *strips, int32_t *ow, int32_t *ytiles, int32_t *chunks, int32_t *items,
                int32_t *blocks, int32_t *threads)
{
    if (!chd3d_available(L) || clen < 1) return false;
    bool ok = false;
    dispatch_prec(L.fp32, [&](auto tz) {
        dispatch_r(L.r, RList<1, 2, 3>{}, [&](auto rc) {
            using T = decltype(tz);
            constexpr int R = decltype(rc)::value;
            auto plan = [&](auto tl) {  // the 3D march's tiles
                using TS = decltype(tl);
                const int64_t st = cdiv(nx, TS::OWMAX);
                const int64_t it = st * cdiv(ny, TS::NR - 2 * TS::H) * cdiv(nz, clen);
                if (it > (int64_t)INT32_MAX) return;
                *strips = (int32_t)st;
                *ow = (int32_t)(cdiv(cdiv(nx, st), TS::V) * TS::V);
                *ytiles = (int32_t)cdiv(ny, TS::NR - 2 * TS::H);
                *chunks = (int32_t)cdiv(nz, clen);
                *items = (int32_t)it;
                *blocks = (int32_t)it;
                *threads = 64 * TS::NW;
                ok = true;
            };
            if (rpw == 4) {
                plan(Tile3D<T, kCHD, R, 1, 4>{});
                return;
            }
            if (rpw != 2) return;
            using TL = CHD3Tile<T, R>;
            const int64_t tx = cdiv(nx, TL::TX), ty = cdiv(ny, TL::TY), ch = cdiv(nz, clen);
            const int64_t it = tx * ty * ch;
            if (it > (int64_t)INT32_MAX) return;
            *strips = (int32_t)tx;
            *ow = TL::TX;
            *ytiles = (int32_t)ty;
            *chunks = (int32_t)ch;
            *items = (int32_t)it;
            *blocks = (int32_t)it;
            *threads = TL::THREADS;
            ok = true;
        });
    });
    return ok;
}

template <typename T, int R, int RPW>
hipError_t launch_chd3d_march(const StepArgs<T> &a, int32_t blocks, int32_t threads, int red, hipStream_t s)
{
    if (threads != 64 * Tile3D<T, kCHD, R, 1, RPW>::NW) return hipErrorInvalidValue;
    if (red)
        hipLaunchKernelGGL((k_step3d<T, kCHD, R, true, 1, RPW>), dim3(blocks), dim3(threads), 0, s, a);
    else
        hipLaunchKernelGGL((k_step3d<T, kCHD, R, false, 1, RPW>), dim3(blocks), dim3(threads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_chd3d(const Launch &L, const void *args, int32_t blocks, int32_t threads, int red,
                        int rpw, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (!chd3d_available(L)) return err;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        dispatch_r(L.r, RList<1, 2, 3>{}, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            if (rpw == 4)
                err = launch_chd3d_march<T, R, 4>(a, blocks, threads, red, s);
            else if (rpw == 2 && threads == CHD3Tile<T, R>::THREADS)
                err = launch_chd3d_r<T, R>(a, blocks, red, s);
        });
    });
    return err;
}

}  // namespace pf
