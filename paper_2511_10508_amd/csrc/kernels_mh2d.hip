// Model H (Eq. model-h, transverse projector one) on 2D grids in one pass.
//
// A workgroup of 256 threads owns a strip of 256 - 4r output columns plus a
// halo of 2r on each side and marches along y over a chunk of rows, one
// column per thread.  Each thread keeps y-windows of m (3r + 1 rows), j_x,
// j_y and mu (2r + 1 rows) in registers; the rows the x neighbours come from
// are in LDS (double-buffered, one barrier per row).  When row t arrives:
//   mu at row t - r   = c2 m^3 - c1 m - L m            (strip + r halo)
//   the update at q = t - 2r:
//     m'   = m + dt L mu - dt c3 div(m j)
//     j_a' = j_a + dt L j_a + dt c3 m D1_a mu
// so mu never reaches HBM, each field is read once and written once per
// step (up to the 4r re-read halo columns of a strip), and the loads of row
// t + 2 are in flight while row t is computed.  Every value is formed with
// the per-site kernel's functions in its order (pairs x, then y; divergence
// x, then y), so the fields are bitwise those of the two-pass per-site
// kernel.
#include "pf_device.h"
#include "pf_dispatch.h"

namespace pf {

namespace {

constexpr int kMH2Threads = 256;
constexpr int kMH2Items = 4096;  // work items a launch aims for (y chunks)

template <int R>
struct MH2Strip {
    static constexpr int G = 2 * R;                      // staged halo
    static constexpr int LX = kMH2Threads;               // loaded columns
    static constexpr int OW = LX - 2 * G;                // output columns
    static constexpr int ZW = 3 * R + 1;                 // y-window of m
    static constexpr int MW = 2 * R + 1;                 // y-windows of j and mu
};

// Rows in LDS per buffer: m at the mu row, then m, j_x, j_y and mu at the
// update row.
enum { kRm = 0, kRmq = 1, kRjx = 2, kRjy = 3, kRmu = 4, kRRows = 5 };

template <typename T, int R>
__global__ void __launch_bounds__(kMH2Threads) k_mh2d(StepArgs<T> a, int32_t strips, int32_t clen)
{
    using SL = MH2Strip<R>;
    constexpr int G = SL::G, LX = SL::LX, ZW = SL::ZW, MW = SL::MW;
    __shared__ T L[2][kRRows][LX];

    const int32_t item = xcd_item(blockIdx.x, gridDim.x);
    const int32_t sx = item % strips, chunk = item / strips;
    const int32_t ny = (int32_t)a.ny;
    const int32_t y0 = chunk * clen, y1 = min(y0 + clen, ny);
    const int lx = threadIdx.x;
    const int64_t x0 = (int64_t)sx * SL::OW;
    const int64_t cx = wrap_any(x0 - G + lx, a.nx);
    const bool mu_col = lx >= R && lx < LX - R;
    const bool out_col = lx >= G && lx < LX - G && x0 + lx - G < a.nx;
    const int par = a.parity;
    const T *__restrict__ in[3] = {a.buf[0][par], a.buf[1][par], a.buf[2][par]};
    T *__restrict__ out[3] = {a.buf[0][par ^ 1], a.buf[1][par ^ 1], a.buf[2][par ^ 1]};
    const T ctr = T(4);

    // y-windows: fm[i] holds m at row t - 3r + i (i <= 3r), fj[c][i] j_c at row
    // t - 3r + i (i <= 2r; j is first needed r rows after m), mu[i] mu at row
    // t - 3r + i (before this row's mu is shifted in).  Loads run two rows
    // ahead into pm / pj, alternating between two register sets so that a
    // value is first touched two rows after its load.
    T fm[ZW], fj[2][MW], mu[MW], pm[2], pj[2][2];
#pragma unroll
    for (int i = 0; i < ZW; ++i) fm[i] = T(0);
#pragma unroll
    for (int i = 0; i < MW; ++i) {
        mu[i] = T(0);
        fj[0][i] = fj[1][i] = T(0);
    }
    const int32_t t0 = y0 - G, tend = y1 + G;
    auto off_of = [&](int32_t t) { return (int64_t)wrap32(t, ny) * a.pitch + cx; };
    auto load_m = [&](int32_t t, T &v) { v = in[0][off_of(t)]; };
    auto load_j = [&](int32_t t, T (&v)[2]) {
        const int64_t off = off_of(t);
        v[0] = in[1][off];
        v[1] = in[2][off];
    };
    load_m(t0, pm[0]);
    load_j(t0 - R, pj[0]);
    load_m(t0 + 1, pm[1]);
    load_j(t0 + 1 - R, pj[1]);

    auto phase = [&](int32_t t, auto parc) {
        constexpr int PH = decltype(parc)::value;
        const int32_t age = t - t0;
        // shift the windows by one row: m of row t and j of row t - r enter;
        // m of t + 2 and j of t + 2 - r are requested
#pragma unroll
        for (int i = 0; i < ZW - 1; ++i) fm[i] = fm[i + 1];
        fm[ZW - 1] = pm[PH];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int i = 0; i < MW - 1; ++i) fj[c][i] = fj[c][i + 1];
            fj[c][MW - 1] = pj[PH][c];
        }
        load_m(t + 2, pm[PH]);
        load_j(t + 2 - R, pj[PH]);
        // LDS rows: m at t - r (index 2r), m / j / mu at q = t - 2r (index r;
        // mu(q) is mu[r + 1] until this row's mu is shifted in)
        auto &B = L[t & 1];
        B[kRm][lx] = fm[2 * R];
        B[kRmq][lx] = fm[R];
        B[kRjx][lx] = fj[0][R];
        B[kRjy][lx] = fj[1][R];
        B[kRmu][lx] = mu[R + 1];
        __syncthreads();
        // mu of row t - r
        T mnew = T(0);
        if (age >= 2 * R && mu_col) {
            T S[R];
#pragma unroll
            for (int j = 1; j <= R; ++j)
                S[j - 1] = (B[kRm][lx + j] + B[kRm][lx - j]) + (fm[2 * R + j] + fm[2 * R - j]);
            const T c0 = fm[2 * R];
            mnew = ch_mu<T, R>(a, c0, S, c0 * ctr);
        }
#pragma unroll
        for (int i = 0; i < MW - 1; ++i) mu[i] = mu[i + 1];
        mu[MW - 1] = mnew;  // now mu[i] holds row t - 3r + i: mu(q) = mu[r]
        // the update of row q = t - 2r
        if (age >= 4 * R && out_col) {
            const int32_t q = t - 2 * R;
            const T m0 = fm[R], mu0 = mu[R];
            T Sm[R], Sx[R], Sy[R];
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                Sm[j - 1] = (B[kRmu][lx + j] + B[kRmu][lx - j]) + (mu[R + j] + mu[R - j]);
                Sx[j - 1] = (B[kRjx][lx + j] + B[kRjx][lx - j]) + (fj[0][R + j] + fj[0][R - j]);
                Sy[j - 1] = (B[kRjy][lx + j] + B[kRjy][lx - j]) + (fj[1][R + j] + fj[1][R - j]);
            }
            T div = T(0);
#pragma unroll
            for (int k = 1; k <= R; ++k)
                div = fma(a.w1[k - 1], B[kRmq][lx + k] * B[kRjx][lx + k] - B[kRmq][lx - k] * B[kRjx][lx - k], div);
#pragma unroll
            for (int k = 1; k <= R; ++k)
                div = fma(a.w1[k - 1], fm[R + k] * fj[1][R + k] - fm[R - k] * fj[1][R - k], div);
            T gx = T(0), gy = T(0);
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                gx = fma(a.w1[k - 1], B[kRmu][lx + k] - B[kRmu][lx - k], gx);
                gy = fma(a.w1[k - 1], mu[R + k] - mu[R - k], gy);
            }
            const int64_t off = off_of(q);
            out[0][off] = fma(-a.k2, div, ch_update<T, R>(a, m0, Sm, mu0 * ctr));
            const T km = a.k2 * m0;
            const T jx0 = fj[0][R], jy0 = fj[1][R];
            out[1][off] = fma(km, gx, ch_update<T, R>(a, jx0, Sx, jx0 * ctr));
            out[2][off] = fma(km, gy, ch_update<T, R>(a, jy0, Sy, jy0 * ctr));
        }
    };
    // two rows per iteration: the register sets alternate at compile time
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

bool mh2d_available(const Launch &L) { return L.kind == kMH && L.ndim == 2 && L.r >= 1 && L.r <= 2; }

hipError_t launch_mh2d(const Launch &L, const void *args, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (!mh2d_available(L)) return err;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        dispatch_r(L.r, RList<1, 2>{}, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            const int64_t strips = cdiv(a.nx, MH2Strip<R>::OW);
            // y chunks: enough work items to fill the chip, at least 16 rows each
            const int64_t chunks =
                std::max<int64_t>(1, std::min<int64_t>(cdiv(kMH2Items, strips), a.ny / 16));
            const int64_t clen = cdiv(a.ny, chunks);
            const int64_t items = strips * cdiv(a.ny, clen);
            if (items > (int64_t)INT32_MAX) return;
            hipLaunchKernelGGL((k_mh2d<T, R>), dim3((unsigned)items), dim3(kMH2Threads), 0, s, a,
                               (int32_t)strips, (int32_t)clen);
            err = hipGetLastError();
        });
    });
    return err;
}

}  // namespace pf
