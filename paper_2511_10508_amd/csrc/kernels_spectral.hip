// Element-wise kernels of the semi-implicit Fourier spectral step: the
// explicit real-space term and the implicit update of the half spectrum.
// The transforms themselves are hipFFT calls (spectral.cpp).
#include <algorithm>
#include <type_traits>

#include "pf_device.h"
#include "pf_dispatch.h"

namespace pf {

namespace {

// Explicit real-space term of the state buf[0][parity] into g (same pitched
// layout): Model A N = c1 u - c2 u^3, Model B g = c2 u^3 - c1 u.
template <typename T, int KIND>
__global__ void __launch_bounds__(256) k_spec_nonlinear(StepArgs<T> a, T *__restrict__ g)
{
    const int64_t N = a.nx * a.ny * a.nz;
    const T c1 = (T)a.c1, c2 = (T)a.c2;
    const T *__restrict__ u = a.buf[0][a.parity];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % a.nx, q = i / a.nx;
        const int64_t off = (q / a.ny) * a.plane + (q % a.ny) * a.pitch + x;
        const T v = u[off];
        const T v3 = (v * v) * v;
        g[off] = KIND == kAC ? c1 * v - c2 * v3 : c2 * v3 - c1 * v;
    }
}

// Implicit update of the half spectrum uh from the explicit term's spectrum
// nh, scaled by 1/N (the inverse transform is unnormalised):
//   Model A: uh <- (uh + dt nh) / (1 + dt K2)
//   Model B: uh <- (uh - dt K2 nh) / (1 + dt K2^2)
// K2 = sum_a (m_a s_a)^2, m_a the signed frequency, s_a = 2 pi / (n_a dx);
// the factors are formed in FP64 for both storage precisions.
template <typename T, int KIND>
__global__ void __launch_bounds__(256) k_spec_update(SpecArgs a)
{
    using C = typename std::conditional<std::is_same<T, double>::value, double2, float2>::type;
    C *__restrict__ uh = static_cast<C *>(a.uh);
    const C *__restrict__ nh = static_cast<const C *>(a.nh);
    const int64_t M = a.nxh * a.ny * a.nz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % a.nxh, q = i / a.nxh;
        const int64_t y = q % a.ny, z = q / a.ny;
        const double kx = (double)x * a.sx;
        const double ky = (double)(2 * y <= a.ny ? y : y - a.ny) * a.sy;
        const double kz = (double)(2 * z <= a.nz ? z : z - a.nz) * a.sz;
        const double K2 = kx * kx + ky * ky + kz * kz;
        const C u = uh[i], n = nh[i];
        C o;
        if constexpr (KIND == kAC) {
            const double f = a.inv_n / (1.0 + a.dt * K2);
            o.x = (T)(((double)u.x + a.dt * (double)n.x) * f);
            o.y = (T)(((double)u.y + a.dt * (double)n.y) * f);
        } else {
            const double f = a.inv_n / (1.0 + a.dt * K2 * K2), d = a.dt * K2;
            o.x = (T)(((double)u.x - d * (double)n.x) * f);
            o.y = (T)(((double)u.y - d * (double)n.y) * f);
        }
        uh[i] = o;
    }
}

unsigned grid_for(int64_t n)
{
    return (unsigned)std::min<int64_t>(std::max<int64_t>(cdiv(n, 256), 1), 16384);
}

}  // namespace

hipError_t launch_spectral_nonlinear(const Launch &L, const void *args, void *g, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        const unsigned grid = grid_for(a.nx * a.ny * a.nz);
        if (L.kind == kAC)
            hipLaunchKernelGGL((k_spec_nonlinear<T, kAC>), dim3(grid), dim3(256), 0, s, a, static_cast<T *>(g));
        else if (L.kind == kCH)
            hipLaunchKernelGGL((k_spec_nonlinear<T, kCH>), dim3(grid), dim3(256), 0, s, a, static_cast<T *>(g));
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
        const unsigned grid = grid_for(a.nxh * a.ny * a.nz);
        if (L.kind == kAC)
            hipLaunchKernelGGL((k_spec_update<T, kAC>), dim3(grid), dim3(256), 0, s, a);
        else if (L.kind == kCH)
            hipLaunchKernelGGL((k_spec_update<T, kCH>), dim3(grid), dim3(256), 0, s, a);
        else
            return;
        err = hipGetLastError();
    });
    return err;
}

}  // namespace pf
