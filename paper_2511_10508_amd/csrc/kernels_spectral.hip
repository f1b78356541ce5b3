// Element-wise kernels of the semi-implicit Fourier spectral step: the
// explicit real-space term and the implicit update of the half spectrum.
// The transforms themselves are hipFFT calls (spectral.cpp).
#include <algorithm>
#include <type_traits>

#include "pf_device.h"
#include "pf_dispatch.h"

namespace pf {

namespace {

// The element-wise kernels walk rows: blockIdx.x covers 256 columns of a row,
// blockIdx.y strides over the rows (ny nz < 2^30), so the index arithmetic is
// 32-bit and the row's division happens once per row.

// Explicit real-space term of the state buf[0][parity] into g (same pitched
// layout): Model A N = c1 u - c2 u^3, Model B g = c2 u^3 - c1 u.
template <typename T, int KIND>
__global__ void __launch_bounds__(256) k_spec_nonlinear(StepArgs<T> a, T *__restrict__ g)
{
    const int32_t x = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (x >= (int32_t)a.nx) return;
    const int32_t ny = (int32_t)a.ny, rows = ny * (int32_t)a.nz;
    const T c1 = (T)a.c1, c2 = (T)a.c2;
    const T *__restrict__ u = a.buf[0][a.parity];
    for (int32_t row = blockIdx.y; row < rows; row += gridDim.y) {
        const int64_t off = (int64_t)(row / ny) * a.plane + (int64_t)(row % ny) * a.pitch + x;
        const T v = u[off];
        const T v3 = (v * v) * v;
        g[off] = KIND == kAC ? c1 * v - c2 * v3 : c2 * v3 - c1 * v;
    }
}

// Implicit update of the half spectrum from the explicit term's spectrum nh:
//   Model A: s <- (u_scale uh + dt nh / N) / (1 + dt K2)
//   Model B: s <- (u_scale uh - dt K2 nh / N) / (1 + dt K2^2)
// K2 = sum_a (m_a s_a)^2, m_a the signed frequency, s_a = 2 pi / (n_a dx);
// the factors are formed in FP64 for both storage precisions.  The result is
// the spectrum of the next state divided by N (the inverse transform is
// unnormalised): it is kept in uh for the next step (u_scale = 1 then; 1/N
// for a spectrum fresh from the forward transform) and also written over nh,
// the input the inverse transform may overwrite.
template <typename T, int KIND>
__global__ void __launch_bounds__(256) k_spec_update(SpecArgs a)
{
    using C = typename std::conditional<std::is_same<T, double>::value, double2, float2>::type;
    const int32_t x = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (x >= (int32_t)a.nxh) return;
    C *__restrict__ uh = static_cast<C *>(a.uh);
    C *__restrict__ nh = static_cast<C *>(a.nh);
    const int32_t ny = (int32_t)a.ny, nz = (int32_t)a.nz, rows = ny * nz;
    const double kx = (double)x * a.sx;
    for (int32_t row = blockIdx.y; row < rows; row += gridDim.y) {
        const int32_t y = row % ny, z = row / ny;
        const double ky = (double)(2 * y <= ny ? y : y - ny) * a.sy;
        const double kz = (double)(2 * z <= nz ? z : z - nz) * a.sz;
        const double K2 = kx * kx + ky * ky + kz * kz;
        const int64_t i = (int64_t)row * a.nxh + x;
        const C u = uh[i], n = nh[i];
        C o;
        if constexpr (KIND == kAC) {
            const double f = 1.0 / (1.0 + a.dt * K2), d = a.dt * a.inv_n;
            o.x = (T)((a.u_scale * (double)u.x + d * (double)n.x) * f);
            o.y = (T)((a.u_scale * (double)u.y + d * (double)n.y) * f);
        } else {
            const double f = 1.0 / (1.0 + a.dt * K2 * K2), d = a.dt * K2 * a.inv_n;
            o.x = (T)((a.u_scale * (double)u.x - d * (double)n.x) * f);
            o.y = (T)((a.u_scale * (double)u.y - d * (double)n.y) * f);
        }
        uh[i] = o;
        nh[i] = o;
    }
}

dim3 grid_rows(int64_t cols, int64_t rows)
{
    return dim3((unsigned)cdiv(cols, 256), (unsigned)std::min<int64_t>(std::max<int64_t>(rows, 1), 65535));
}

}  // namespace

hipError_t launch_spectral_nonlinear(const Launch &L, const void *args, void *g, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        const dim3 grid = grid_rows(a.nx, a.ny * a.nz);
        if (L.kind == kAC)
            hipLaunchKernelGGL((k_spec_nonlinear<T, kAC>), grid, dim3(256), 0, s, a, static_cast<T *>(g));
        else if (L.kind == kCH)
            hipLaunchKernelGGL((k_spec_nonlinear<T, kCH>), grid, dim3(256), 0, s, a, static_cast<T *>(g));
        else
            return;
        err = hipGetLastError();
    });
    return err;
}

hipError_t launch_spectral_update(const Launch &L, const SpecArgs &a, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const dim3 grid = grid_rows(a.nxh, a.ny * a.nz);
        if (L.kind == kAC)
            hipLaunchKernelGGL((k_spec_update<T, kAC>), grid, dim3(256), 0, s, a);
        else if (L.kind == kCH)
            hipLaunchKernelGGL((k_spec_update<T, kCH>), grid, dim3(256), 0, s, a);
        else
            return;
        err = hipGetLastError();
    });
    return err;
}

}  // namespace pf
