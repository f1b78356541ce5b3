// Model H (Eq. model-h, transverse projector one) on 2D grids in one pass.
//
// A workgroup of 256 threads owns a tile of 32 x 32 output sites.  It stages
// m, j_x and j_y on the tile plus a halo of 2r (periodic wrap on load) in LDS,
// forms mu = c2 m^3 - c1 m - L m on the tile plus a halo of r in LDS, then
// the coupled update of its outputs:
//   m'   = m + dt L mu - dt c3 div(m j)
//   j_a' = j_a + dt L j_a + dt c3 m D1_a mu
// Every value is formed with the per-site kernel's functions in its order
// (x pair, then y pair; divergence x then y), so the fields are bitwise those
// of the two-pass per-site kernel, without its mu buffer in HBM.
#include "pf_device.h"
#include "pf_dispatch.h"

namespace pf {

namespace {

constexpr int kTileMH = 32;

template <typename T, int R>
__global__ void __launch_bounds__(256) k_mh2d(StepArgs<T> a, int32_t tiles_x)
{
    constexpr int TX = kTileMH, TY = kTileMH, H2 = 2 * R;
    constexpr int LX = TX + 2 * H2, LY = TY + 2 * H2;  // staged fields
    constexpr int MX = TX + 2 * R, MY = TY + 2 * R;    // mu
    __shared__ T sm[LY][LX], sjx[LY][LX], sjy[LY][LX];
    __shared__ T smu[MY][MX];
    const int32_t bx = blockIdx.x % tiles_x, by = blockIdx.x / tiles_x;
    const int64_t x0 = (int64_t)bx * TX, y0 = (int64_t)by * TY;
    const int par = a.parity;
    const T *__restrict__ pm = a.buf[0][par];
    const T *__restrict__ px = a.buf[1][par];
    const T *__restrict__ py = a.buf[2][par];
    for (int i = threadIdx.x; i < LX * LY; i += 256) {
        const int ly = i / LX, lx = i % LX;
        const int64_t gx = wrap_any(x0 - H2 + lx, a.nx), gy = wrap_any(y0 - H2 + ly, a.ny);
        const int64_t off = gy * a.pitch + gx;
        sm[ly][lx] = pm[off];
        sjx[ly][lx] = px[off];
        sjy[ly][lx] = py[off];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < MX * MY; i += 256) {
        const int my = i / MX, mx = i % MX;
        const int ly = my + R, lx = mx + R;
        T S[R];
#pragma unroll
        for (int j = 1; j <= R; ++j)
            S[j - 1] = (sm[ly][lx + j] + sm[ly][lx - j]) + (sm[ly + j][lx] + sm[ly - j][lx]);
        const T c0 = sm[ly][lx];
        smu[my][mx] = ch_mu<T, R>(a, c0, S, c0 * T(4));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TX * TY; i += 256) {
        const int oy = i / TX, ox = i % TX;
        const int64_t gx = x0 + ox, gy = y0 + oy;
        if (gx >= a.nx || gy >= a.ny) continue;
        const int ly = oy + H2, lx = ox + H2;  // staged coordinates
        const int my = oy + R, mx = ox + R;    // mu coordinates
        const T m0 = sm[ly][lx], mu0 = smu[my][mx];
        T Sm[R], Sx[R], Sy[R];
        T div = T(0), gxm = T(0), gym = T(0);
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            Sm[j - 1] = (smu[my][mx + j] + smu[my][mx - j]) + (smu[my + j][mx] + smu[my - j][mx]);
            Sx[j - 1] = (sjx[ly][lx + j] + sjx[ly][lx - j]) + (sjx[ly + j][lx] + sjx[ly - j][lx]);
            Sy[j - 1] = (sjy[ly][lx + j] + sjy[ly][lx - j]) + (sjy[ly + j][lx] + sjy[ly - j][lx]);
        }
#pragma unroll
        for (int k = 1; k <= R; ++k)
            div = fma(a.w1[k - 1], sm[ly][lx + k] * sjx[ly][lx + k] - sm[ly][lx - k] * sjx[ly][lx - k], div);
#pragma unroll
        for (int k = 1; k <= R; ++k)
            div = fma(a.w1[k - 1], sm[ly + k][lx] * sjy[ly + k][lx] - sm[ly - k][lx] * sjy[ly - k][lx], div);
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            gxm = fma(a.w1[k - 1], smu[my][mx + k] - smu[my][mx - k], gxm);
            gym = fma(a.w1[k - 1], smu[my + k][mx] - smu[my - k][mx], gym);
        }
        const int64_t off = gy * a.pitch + gx;
        a.buf[0][par ^ 1][off] = fma(-a.k2, div, ch_update<T, R>(a, m0, Sm, mu0 * T(4)));
        const T jx0 = sjx[ly][lx], jy0 = sjy[ly][lx];
        a.buf[1][par ^ 1][off] = fma(a.k2 * m0, gxm, ch_update<T, R>(a, jx0, Sx, jx0 * T(4)));
        a.buf[2][par ^ 1][off] = fma(a.k2 * m0, gym, ch_update<T, R>(a, jy0, Sy, jy0 * T(4)));
    }
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
        const int64_t tx = cdiv(a.nx, kTileMH), ty = cdiv(a.ny, kTileMH);
        if (tx * ty > (int64_t)INT32_MAX) return;
        dispatch_r(L.r, RList<1, 2>{}, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            hipLaunchKernelGGL((k_mh2d<T, R>), dim3((unsigned)(tx * ty)), dim3(256), 0, s, a, (int32_t)tx);
            err = hipGetLastError();
        });
    });
    return err;
}

}  // namespace pf
