// Model H (Eq. model-h, transverse projector one) on 3D grids in one pass.
//
// A workgroup owns an x-y tile of output columns and marches along z
// over a chunk of planes.  Each thread holds one column of the tile plus a
// halo of 2r on each side (the columns of mu's own neighbours): for every
// plane it keeps z-windows of m, j_x, j_y, j_z (3r + 1 planes) and of mu
// (2r + 1 planes) in registers, and the centre planes the x-y neighbours
// come from in LDS (double-buffered, one barrier per plane).  When plane t
// arrives:
//   mu at plane t - r   = c2 m^3 - c1 m - L m            (tile + r halo)
//   the update at q = t - 2r:
//     m'   = m + dt L mu - dt c3 div(m j)
//     j_a' = j_a + dt L j_a + dt c3 m D1_a mu
// so mu never reaches HBM, each field is read once and written once per
// step (up to the re-read tile halos), and the loads of plane t + 2 are in
// flight while plane t is computed.  Every value is formed with the
// per-site kernel's functions in its order (pairs x, then y, then z;
// divergence x, then y, then z), so the fields are bitwise those of the
// two-pass per-site kernel.
#include "pf_device.h"
#include "pf_dispatch.h"

namespace pf {

namespace {

constexpr int kMH3Items = 2048;  // work items a launch aims for (z chunks)

// Output columns of a tile: 32 x 16, or 16 x 16 for FP64 with r = 2, whose
// windows need more than the 128 registers a lane of a 15-wave workgroup
// has (a 9-wave workgroup gets 168).
template <typename T, int R>
struct MH3Tile {
    static constexpr int TX = (std::is_same<T, double>::value && R == 2) ? 16 : 32, TY = 16;
    static constexpr int G = 2 * R;                      // staged halo
    static constexpr int LX = TX + 2 * G, LY = TY + 2 * G;
    static constexpr int NT = LX * LY;                   // columns (threads that load)
    static constexpr int THREADS = (NT + 63) / 64 * 64;
    static constexpr int ZW = 3 * R + 1;                 // z-window of the fields
    static constexpr int MW = 2 * R + 1;                 // z-window of mu
};

// Planes in LDS per buffer: m at the mu plane, then m, j_x, j_y, j_z and mu
// at the update plane.
enum { kLm = 0, kLmq = 1, kLjx = 2, kLjy = 3, kLjz = 4, kLmu = 5, kLPlanes = 6 };

template <typename T, int R>
__global__ void __launch_bounds__((MH3Tile<T, R>::THREADS)) k_mh3d(StepArgs<T> a, int32_t tiles_x,
                                                             int32_t tiles_y, int32_t clen)
{
    using TL = MH3Tile<T, R>;
    constexpr int G = TL::G, LX = TL::LX, LY = TL::LY, ZW = TL::ZW, MW = TL::MW;
    __shared__ T L[2][kLPlanes][LY][LX];

    const int32_t item = xcd_item(blockIdx.x, gridDim.x);
    const int32_t tx = item % tiles_x, rest = item / tiles_x;
    const int32_t ty = rest % tiles_y, chunk = rest / tiles_y;
    const int32_t nz = (int32_t)a.nz;
    const int32_t z0 = chunk * clen, z1 = min(z0 + clen, nz);
    const int tid = threadIdx.x;
    const bool col = tid < TL::NT;  // threads past the tile's columns only take part in barriers
    const int lx = col ? tid % LX : 0, ly = col ? tid / LX : 0;
    const int64_t x0 = (int64_t)tx * TL::TX, y0 = (int64_t)ty * TL::TY;
    const int64_t coff = wrap_any(y0 - G + ly, a.ny) * a.pitch + wrap_any(x0 - G + lx, a.nx);
    const bool mu_col = col && lx >= R && lx < LX - R && ly >= R && ly < LY - R;
    const bool out_col = col && lx >= G && lx < LX - G && ly >= G && ly < LY - G &&
                         x0 + lx - G < a.nx && y0 + ly - G < a.ny;
    const int par = a.parity;
    const T *__restrict__ in[4] = {a.buf[0][par], a.buf[1][par], a.buf[2][par], a.buf[3][par]};
    T *__restrict__ out[4] = {a.buf[0][par ^ 1], a.buf[1][par ^ 1], a.buf[2][par ^ 1], a.buf[3][par ^ 1]};
    const T ctr = T(6);

    // z-windows: fm[i] holds m at plane t - 3r + i (i <= 3r), fj[c][i] j_c at
    // plane t - 3r + i (i <= 2r; j is first needed r planes after m), mu[i]
    // mu at plane t - 3r + i (before this plane's mu is shifted in).  Loads
    // run two planes ahead into pm / pj, alternating between two register
    // sets so that a value is first touched two planes after its load.
    T fm[ZW], fj[3][MW], mu[MW], pm[2], pj[2][3];
#pragma unroll
    for (int i = 0; i < ZW; ++i) fm[i] = T(0);
#pragma unroll
    for (int i = 0; i < MW; ++i) {
        mu[i] = T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) fj[c][i] = T(0);
    }
    const int32_t t0 = z0 - G, tend = z1 + G;
    auto off_of = [&](int32_t t) { return (int64_t)wrap32(t, nz) * a.plane + coff; };
    auto load_m = [&](int32_t t, T &v) { v = col ? in[0][off_of(t)] : T(0); };
    auto load_j = [&](int32_t t, T (&v)[3]) {
        const int64_t off = off_of(t);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = col ? in[1 + c][off] : T(0);
    };
    load_m(t0, pm[0]);
    load_j(t0 - R, pj[0]);
    load_m(t0 + 1, pm[1]);
    load_j(t0 + 1 - R, pj[1]);

    auto phase = [&](int32_t t, auto parc) {
        constexpr int PH = decltype(parc)::value;
        const int32_t age = t - t0;
        // shift the windows by one plane: m of plane t and j of plane t - r
        // enter; m of t + 2 and j of t + 2 - r are requested
#pragma unroll
        for (int i = 0; i < ZW - 1; ++i) fm[i] = fm[i + 1];
        fm[ZW - 1] = pm[PH];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int i = 0; i < MW - 1; ++i) fj[c][i] = fj[c][i + 1];
            fj[c][MW - 1] = pj[PH][c];
        }
        load_m(t + 2, pm[PH]);
        load_j(t + 2 - R, pj[PH]);
        // centre planes: m at t - r (index 2r), m / j / mu at q = t - 2r (index r;
        // mu(q) is mu[r + 1] until this plane's mu is shifted in)
        auto &B = L[t & 1];
        if (col) {
            B[kLm][ly][lx] = fm[2 * R];
            B[kLmq][ly][lx] = fm[R];
            B[kLjx][ly][lx] = fj[0][R];
            B[kLjy][ly][lx] = fj[1][R];
            B[kLjz][ly][lx] = fj[2][R];
            B[kLmu][ly][lx] = mu[R + 1];
        }
        __syncthreads();
        // mu of plane t - r
        T mnew = T(0);
        if (age >= 2 * R && mu_col) {
            T S[R];
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                T acc = B[kLm][ly][lx + j] + B[kLm][ly][lx - j];
                acc = acc + (B[kLm][ly + j][lx] + B[kLm][ly - j][lx]);
                acc = acc + (fm[2 * R + j] + fm[2 * R - j]);
                S[j - 1] = acc;
            }
            const T c0 = fm[2 * R];
            mnew = ch_mu<T, R>(a, c0, S, c0 * ctr);
        }
#pragma unroll
        for (int i = 0; i < MW - 1; ++i) mu[i] = mu[i + 1];
        mu[MW - 1] = mnew;  // now mu[i] holds plane t - 3r + i: mu(q) = mu[r]
        // the update of plane q = t - 2r
        if (age >= 4 * R && out_col) {
            const int32_t q = t - 2 * R;
            const T m0 = fm[R], mu0 = B[kLmu][ly][lx];
            T Sm[R];
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                T acc = B[kLmu][ly][lx + j] + B[kLmu][ly][lx - j];
                acc = acc + (B[kLmu][ly + j][lx] + B[kLmu][ly - j][lx]);
                acc = acc + (mu[R + j] + mu[R - j]);
                Sm[j - 1] = acc;
            }
            T div = T(0);
#pragma unroll
            for (int k = 1; k <= R; ++k)
                div = fma(a.w1[k - 1], B[kLmq][ly][lx + k] * B[kLjx][ly][lx + k] -
                                           B[kLmq][ly][lx - k] * B[kLjx][ly][lx - k], div);
#pragma unroll
            for (int k = 1; k <= R; ++k)
                div = fma(a.w1[k - 1], B[kLmq][ly + k][lx] * B[kLjy][ly + k][lx] -
                                           B[kLmq][ly - k][lx] * B[kLjy][ly - k][lx], div);
#pragma unroll
            for (int k = 1; k <= R; ++k)
                div = fma(a.w1[k - 1], fm[R + k] * fj[2][R + k] - fm[R - k] * fj[2][R - k], div);
            const int64_t off = off_of(q);
            out[0][off] = fma(-a.k2, div, ch_update<T, R>(a, m0, Sm, mu0 * ctr));
            const T km = a.k2 * m0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int pl = kLjx + ax;
                T Sj[R];
                T grad = T(0);
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    T acc = B[pl][ly][lx + j] + B[pl][ly][lx - j];
                    acc = acc + (B[pl][ly + j][lx] + B[pl][ly - j][lx]);
                    acc = acc + (fj[ax][R + j] + fj[ax][R - j]);
                    Sj[j - 1] = acc;
                }
#pragma unroll
                for (int k = 1; k <= R; ++k) {
                    T d;
                    if (ax == 0)
                        d = B[kLmu][ly][lx + k] - B[kLmu][ly][lx - k];
                    else if (ax == 1)
                        d = B[kLmu][ly + k][lx] - B[kLmu][ly - k][lx];
                    else
                        d = mu[R + k] - mu[R - k];
                    grad = fma(a.w1[k - 1], d, grad);
                }
                const T j0 = fj[ax][R];
                out[1 + ax][off] = fma(km, grad, ch_update<T, R>(a, j0, Sj, j0 * ctr));
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
}

}  // namespace

bool mh3d_available(const Launch &L) { return L.kind == kMH && L.ndim == 3 && L.r >= 1 && L.r <= 2; }

hipError_t launch_mh3d(const Launch &L, const void *args, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (!mh3d_available(L)) return err;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        dispatch_r(L.r, RList<1, 2>{}, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            using TL = MH3Tile<T, R>;
            const int64_t tx = cdiv(a.nx, TL::TX), ty = cdiv(a.ny, TL::TY);
            const int64_t tiles = tx * ty;
            // z chunks: enough work items to fill the chip, at least 16 planes each
            const int64_t chunks =
                std::max<int64_t>(1, std::min<int64_t>(cdiv(kMH3Items, tiles), a.nz / 16));
            const int64_t clen = cdiv(a.nz, chunks);
            const int64_t items = tiles * cdiv(a.nz, clen);
            if (items > (int64_t)INT32_MAX || tx > INT32_MAX || ty > INT32_MAX) return;
            hipLaunchKernelGGL((k_mh3d<T, R>), dim3((unsigned)items), dim3(TL::THREADS), 0, s, a,
                               (int32_t)tx, (int32_t)ty, (int32_t)clen);
            err = hipGetLastError();
        });
    });
    return err;
}

}  // namespace pf
