// Per-site generic step kernels (any radius, 2D and 3D), standalone
// reductions, the fixed-order finaliser, initial conditions and the copy probe.
#include "pf_device.h"
#include "pf_dispatch.h"

namespace pf {

using GenericRadii = RList<1, 2, 3, 4, 5, 6, 7, 8>;

namespace {

struct Site {
    int64_t x, y, z;
};

__device__ __forceinline__ Site site_of(int64_t i, int64_t nx, int64_t ny)
{
    Site s;
    s.x = i % nx;
    const int64_t q = i / nx;
    s.y = q % ny;
    s.z = q / ny;
    return s;
}

// Neighbour pair sums S[j-1] at site s of field f (x, then y, then z).
template <typename T, int R, typename Src>
__device__ __forceinline__ void pair_sums(const Src &at, const Site &s, int ndim, T (&S)[R])
{
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        T acc = at(s.x + j, s.y, s.z) + at(s.x - j, s.y, s.z);
        if (ndim >= 2) acc = acc + (at(s.x, s.y + j, s.z) + at(s.x, s.y - j, s.z));
        if (ndim == 3) acc = acc + (at(s.x, s.y, s.z + j) + at(s.x, s.y, s.z - j));
        S[j - 1] = acc;
    }
}

template <typename T>
struct Field {
    const T *p;
    int64_t nx, ny, nz, pitch, plane;
    __device__ __forceinline__ T operator()(int64_t x, int64_t y, int64_t z) const
    {
        return p[wrap_any(z, nz) * plane + wrap_any(y, ny) * pitch + wrap_any(x, nx)];
    }
};

// Site s shifted by d along axis a.
__device__ __forceinline__ Site shifted(Site s, int a, int64_t d)
{
    if (a == 0) s.x += d; else if (a == 1) s.y += d; else s.z += d;
    return s;
}

// Direct-biharmonic chemical potential mu_a (g minus the second derivatives
// of c along the axes other than a) at site s.
template <typename T, int R, typename Src>
__device__ __forceinline__ T mu_axis(const StepArgs<T> &a, const Src &c, const Site &s, int ax,
                                     int ndim)
{
    T S[R];
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        T acc = T(0);
        for (int b = 0; b < ndim; ++b) {
            if (b == ax) continue;
            const Site p = shifted(s, b, j), m = shifted(s, b, -j);
            acc = acc + (c(p.x, p.y, p.z) + c(m.x, m.y, m.z));
        }
        S[j - 1] = acc;
    }
    const T c0 = c(s.x, s.y, s.z);
    return ch_mu<T, R>(a, c0, S, c0 * T(2 * (ndim - 1)));
}

// PASS 0: AC / GS / MC full step; PASS 1: CH chemical potential into
// scratch (direct biharmonic: mu_a of every axis a into scratch + a * fsize,
// fsize = the elements of one field buffer); PASS 2: CH update from scratch.
template <typename T, int KIND, int R, int PASS>
__global__ void __launch_bounds__(256) k_generic(StepArgs<T> a, T *scratch, int ndim)
{
    const int64_t N = a.nx * a.ny * a.nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const Site s = site_of(i, a.nx, a.ny);
    const int64_t off = s.z * a.plane + s.y * a.pitch + s.x;
    const int par = a.parity;
    const T ctrk = T(2 * ndim);
    Field<T> f0{a.buf[0][par], a.nx, a.ny, a.nz, a.pitch, a.plane};
    if constexpr (KIND == kAC) {
        T S[R];
        pair_sums<T, R>(f0, s, ndim, S);
        const T u0 = f0.p[off];
        a.buf[0][par ^ 1][off] = ac_update<T, R>(a, u0, S, u0 * ctrk);
    } else if constexpr (KIND == kGS) {
        Field<T> f1{a.buf[1][par], a.nx, a.ny, a.nz, a.pitch, a.plane};
        T Su[R], Sv[R];
        pair_sums<T, R>(f0, s, ndim, Su);
        pair_sums<T, R>(f1, s, ndim, Sv);
        const T u0 = f0.p[off], v0 = f1.p[off];
        T un, vn;
        gs_update<T, R>(a, u0, v0, Su, Sv, u0 * ctrk, v0 * ctrk, un, vn);
        a.buf[0][par ^ 1][off] = un;
        a.buf[1][par ^ 1][off] = vn;
    } else if constexpr (KIND == kMC) {
        Field<T> f1{a.buf[1][par], a.nx, a.ny, a.nz, a.pitch, a.plane};
        auto g = [&](int64_t x, int64_t y, int64_t z) { return mc_g(a, f0(x, y, z), f1(x, y, z)); };
        T Sp[R], Sg[R];
        pair_sums<T, R>(f0, s, ndim, Sp);
        pair_sums<T, R>(g, s, ndim, Sg);
        const T p0 = f0.p[off], r0 = f1.p[off];
        T pn, rn;
        mc_update<T, R>(a, p0, r0, Sp, Sg, p0 * ctrk, mc_g(a, p0, r0) * ctrk, pn, rn);
        a.buf[0][par ^ 1][off] = pn;
        a.buf[1][par ^ 1][off] = rn;
    } else if constexpr (KIND == kMH && PASS == 2) {
        // Model H (Eq. model-h, transverse projector one): k2 = dt c3, w1 =
        // w1_j/dx; m' = m + dt L mu - dt c3 div(m j), j_a' = j_a + dt L j_a +
        // dt c3 m grad_a mu, with mu from the first pass.
        Field<T> fm{scratch, a.nx, a.ny, a.nz, a.pitch, a.plane};
        const T m0 = f0.p[off], mu0 = scratch[off];
        T Sm[R];
        pair_sums<T, R>(fm, s, ndim, Sm);
        T div = T(0);
        for (int ax = 0; ax < ndim; ++ax) {
            Field<T> fj{a.buf[1 + ax][par], a.nx, a.ny, a.nz, a.pitch, a.plane};
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                const Site p = shifted(s, ax, k), q = shifted(s, ax, -k);
                div = fma(a.w1[k - 1], f0(p.x, p.y, p.z) * fj(p.x, p.y, p.z) - f0(q.x, q.y, q.z) * fj(q.x, q.y, q.z), div);
            }
        }
        a.buf[0][par ^ 1][off] = fma(-a.k2, div, ch_update<T, R>(a, m0, Sm, mu0 * ctrk));
        for (int ax = 0; ax < ndim; ++ax) {
            Field<T> fj{a.buf[1 + ax][par], a.nx, a.ny, a.nz, a.pitch, a.plane};
            T Sj[R];
            pair_sums<T, R>(fj, s, ndim, Sj);
            T grad = T(0);
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                const Site p = shifted(s, ax, k), q = shifted(s, ax, -k);
                grad = fma(a.w1[k - 1], fm(p.x, p.y, p.z) - fm(q.x, q.y, q.z), grad);
            }
            const T j0 = fj.p[off];
            a.buf[1 + ax][par ^ 1][off] = fma(a.k2 * m0, grad, ch_update<T, R>(a, j0, Sj, j0 * ctrk));
        }
    } else if constexpr (KIND == kCHD && PASS == 1) {
        const int64_t fsize = a.plane * a.nz;
        for (int ax = 0; ax < ndim; ++ax) scratch[ax * fsize + off] = mu_axis<T, R>(a, f0, s, ax, ndim);
    } else if constexpr (KIND == kCHD) {
        const int64_t fsize = a.plane * a.nz;
        T Sm[R], S4[R + 1];
        T ctrm = T(0);
        for (int j = 0; j < R; ++j) Sm[j] = T(0);
        for (int ax = 0; ax < ndim; ++ax) {
            Field<T> fm{scratch + ax * fsize, a.nx, a.ny, a.nz, a.pitch, a.plane};
            ctrm = ctrm + T(2) * fm.p[off];
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                const Site p = shifted(s, ax, j), m = shifted(s, ax, -j);
                Sm[j - 1] = Sm[j - 1] + (fm(p.x, p.y, p.z) + fm(m.x, m.y, m.z));
            }
        }
#pragma unroll
        for (int j = 1; j <= R + 1; ++j) {
            T acc = T(0);
            for (int ax = 0; ax < ndim; ++ax) {
                const Site p = shifted(s, ax, j), m = shifted(s, ax, -j);
                acc = acc + (f0(p.x, p.y, p.z) + f0(m.x, m.y, m.z));
            }
            S4[j - 1] = acc;
        }
        const T c0 = f0.p[off];
        a.buf[0][par ^ 1][off] = chd_update<T, R>(a, c0, Sm, ctrm, S4, c0 * ctrk);
    } else if constexpr (PASS == 1) {
        T S[R];
        pair_sums<T, R>(f0, s, ndim, S);
        const T c0 = f0.p[off];
        scratch[off] = ch_mu<T, R>(a, c0, S, c0 * ctrk);
    } else {
        Field<T> fm{scratch, a.nx, a.ny, a.nz, a.pitch, a.plane};
        T Sm[R];
        pair_sums<T, R>(fm, s, ndim, Sm);
        a.buf[0][par ^ 1][off] = ch_update<T, R>(a, f0.p[off], Sm, scratch[off] * ctrk);
    }
}

// Standalone reductions of the state buf[.][parity]: grid-stride over sites,
// one compensated partial per wave.
constexpr int kRedBlocks = 4096;

template <typename T, int KIND, int R>
__global__ void __launch_bounds__(256) k_reduce_state(StepArgs<T> a, int ndim)
{
    const int64_t N = a.nx * a.ny * a.nz;
    const int par = a.parity;
    Field<T> f0{a.buf[0][par], a.nx, a.ny, a.nz, a.pitch, a.plane};
    Field<T> f1{a.buf[nfields_kind(KIND) == 2 ? 1 : 0][par], a.nx, a.ny, a.nz, a.pitch, a.plane};
    RedState red;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Site s = site_of(i, a.nx, a.ny);
        const int64_t off = s.z * a.plane + s.y * a.pitch + s.x;
        const double x = (double)f0.p[off];
        acc_add(red.q0, x);
        red.bad += finite_val(x) ? 0u : 1u;
        if constexpr (nfields_kind(KIND) == 2) {
            const double y = (double)f1.p[off];
            acc_add(red.q1, y);
            red.bad += finite_val(y) ? 0u : 1u;
        } else {
            double S64[R];
            auto at = [&](int64_t xx, int64_t yy, int64_t zz) { return (double)f0(xx, yy, zz); };
            pair_sums<double, R>(at, s, ndim, S64);
            acc_add(red.q1, energy_density<R>(a.c1, a.c2, a.w64, x, S64, x * (2.0 * ndim)));
        }
    }
    const int64_t slot = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    red_flush(red, a.part, a.pstride, slot, threadIdx.x & 63);
}

// Fixed-order combination of the partials in two levels: block b of the
// first level takes a contiguous range of slots (thread t: slots t, t + 256,
// .. of the range, compensated), reduces it with a fixed binary tree in LDS
// and writes one pair per quantity; one block then combines those pairs the
// same way.  The result depends only on the slot count, never on timing.
constexpr int kFin = 256;

__device__ __forceinline__ Acc block_tree(Acc a, double *sh, double *sl)
{
    const int t = threadIdx.x;
    sh[t] = a.hi;
    sl[t] = a.lo;
    __syncthreads();
    for (int w = kFin / 2; w >= 1; w >>= 1) {
        if (t < w) {
            Acc x{sh[t], sl[t]};
            const Acc y{sh[t + w], sl[t + w]};
            acc_merge(x, y);
            sh[t] = x.hi;
            sl[t] = x.lo;
        }
        __syncthreads();
    }
    Acc r{sh[0], sl[0]};
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kFin) k_finalize1(const double2 *part, int64_t pstride,
                                                    int64_t slots, double2 *part2)
{
    __shared__ double sh[kFin], sl[kFin];
    const int64_t per = (slots + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = min(slots, lo + per);
    for (int q = 0; q < kNumQ; ++q) {
        Acc a{0.0, 0.0};
        for (int64_t i = lo + threadIdx.x; i < hi; i += kFin) {
            const double2 p = part[q * pstride + i];
            acc_add(a, p.x);
            a.lo += p.y;
        }
        const Acc r = block_tree(a, sh, sl);
        if (threadIdx.x == 0) part2[q * kFin + blockIdx.x] = make_double2(r.hi, r.lo);
    }
}

__global__ void __launch_bounds__(kFin) k_finalize2(const double2 *part2, int nb, double2 *out)
{
    __shared__ double sh[kFin], sl[kFin];
    for (int q = 0; q < kNumQ; ++q) {
        Acc a{0.0, 0.0};
        if ((int)threadIdx.x < nb) {
            const double2 p = part2[q * kFin + threadIdx.x];
            a.hi = p.x;
            a.lo = p.y;
        }
        const Acc r = block_tree(a, sh, sl);
        if (threadIdx.x == 0) {
            const double s = r.hi + r.lo;
            out[q] = make_double2(s, r.lo - (s - r.hi));
        }
    }
}

// SplitMix64 output finaliser (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double u01_of(uint64_t key, uint64_t idx)
{
    const uint64_t h = mix64(key + (idx + 1ull) * 0x9E3779B97F4A7C15ull);
    return (double)(h >> 11) * 0x1.0p-53;
}

__global__ void __launch_bounds__(256) k_init(InitArgs a)
{
    const int64_t N = a.nx * a.ny * a.nz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Site s = site_of(i, a.nx, a.ny);
        const int64_t off = s.z * a.plane + s.y * a.pitch + s.x;
        double val[2] = {0.0, 0.0};
        if (a.ic == 1) {
            val[0] = a.lo + a.span * u01_of(a.key0, (uint64_t)i);
            val[1] = a.lo + a.span * u01_of(a.key1, (uint64_t)i);
        } else if (a.ic == 2) {
            bool inside = false;
            for (int c = 0; c < a.ncubes; ++c) {
                const int64_t dx = wrap_any(s.x - a.cube[c][0], a.nx);
                const int64_t dy = wrap_any(s.y - a.cube[c][1], a.ny);
                const int64_t dz = wrap_any(s.z - a.cube[c][2], a.nz);
                const int64_t sx = a.side < a.nx ? a.side : a.nx;
                const int64_t sy = a.side < a.ny ? a.side : a.ny;
                const int64_t sz = a.side < a.nz ? a.side : a.nz;
                inside = inside || (dx < sx && dy < sy && dz < sz);
            }
            const double bu = inside ? a.in0 : a.v0;
            const double bv = inside ? a.in1 : a.v1;
            val[0] = bu + (a.lo + a.span * u01_of(a.key0, (uint64_t)i));
            val[1] = bv + (a.lo + a.span * u01_of(a.key1, (uint64_t)i));
        } else {
            val[0] = a.v0;
            val[1] = a.v1;
        }
        for (int f = 0; f < a.nfields && f < 2; ++f) {
            void *p = f == 0 ? a.f0 : a.f1;
            if (a.fp32)
                static_cast<float *>(p)[off] = (float)val[f];
            else
                static_cast<double *>(p)[off] = val[f];
        }
    }
}

__global__ void __launch_bounds__(256) k_copy(float4 *__restrict__ dst,
                                              const float4 *__restrict__ src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

hipError_t launch_generic(const Launch &L, const void *args, void *scratch, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        const int64_t N = a.nx * a.ny * a.nz;
        const dim3 grid((unsigned)cdiv(N, 256)), block(256);
        dispatch_kind_generic(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            dispatch_r(L.r, GenericRadii{}, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                T *sc = static_cast<T *>(scratch);
                if constexpr (KIND == kCH || KIND == kCHD || KIND == kMH) {
                    hipLaunchKernelGGL((k_generic<T, KIND, R, 1>), grid, block, 0, s, a, sc, L.ndim);
                    err = hipGetLastError();
                    if (err != hipSuccess) return;
                    hipLaunchKernelGGL((k_generic<T, KIND, R, 2>), grid, block, 0, s, a, sc, L.ndim);
                } else {
                    hipLaunchKernelGGL((k_generic<T, KIND, R, 0>), grid, block, 0, s, a, sc, L.ndim);
                }
                err = hipGetLastError();
            });
        });
    });
    return err;
}

int64_t reduce_partial_slots(int64_t nsites)
{
    return std::min<int64_t>(cdiv(nsites, 256), kRedBlocks) * 4;
}

hipError_t launch_reduce_state(const Launch &L, const void *args, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        const int64_t N = a.nx * a.ny * a.nz;
        const dim3 grid((unsigned)(reduce_partial_slots(N) / 4)), block(256);
        dispatch_kind_generic(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            dispatch_r(L.r, GenericRadii{}, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                hipLaunchKernelGGL((k_reduce_state<T, KIND, R>), grid, block, 0, s, a, L.ndim);
                err = hipGetLastError();
            });
        });
    });
    return err;
}

hipError_t launch_finalize(const double2 *part, int64_t pstride, int64_t slots, double2 *part2,
                           double2 *out, hipStream_t s)
{
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kFin, cdiv(slots, kFin)));
    hipLaunchKernelGGL(k_finalize1, dim3(nb), dim3(kFin), 0, s, part, pstride, slots, part2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize2, dim3(1), dim3(kFin), 0, s, part2, nb, out);
    return hipGetLastError();
}

hipError_t launch_init(const InitArgs &a, hipStream_t s)
{
    const int64_t N = a.nx * a.ny * a.nz;
    const int64_t blocks = std::min<int64_t>(cdiv(N, 256), 65536);
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t blocks = std::min<int64_t>(cdiv(n, 256), 1 << 20);
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<float4 *>(dst), static_cast<const float4 *>(src), n);
    return hipGetLastError();
}

}  // namespace pf
