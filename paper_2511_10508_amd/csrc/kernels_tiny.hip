// Serving class for tiny grids: the whole grid of a request in one
// workgroup's LDS.
//
// One workgroup of 1024 threads takes one request of the table at a time: it
// loads the request's fields into LDS (dense, x fastest), runs the request's
// steps of this tick there, ping-ponging between two copies of the fields,
// and writes the final state into the other buffer of each field.  HBM is
// touched once per tick instead of once per step, and a tick can run many
// steps of a tiny request without lengthening the tick.  Cahn-Hilliard keeps
// mu, Model C keeps g = rho + c3 phi^2 in a further LDS array.  Threads walk
// the grid row by row (thread t holds column t mod nx of every
// 1024 / nx-th row), so a site's coordinates cost no division.  Every site is
// evaluated with the fused kernels' functions and neighbour order (x pair,
// then y, then z), so the fields are bitwise those of the same request
// stepped alone.
#include "pf_device.h"
#include "pf_dispatch.h"

namespace pf {

namespace {

constexpr int kTinyThreads = 1024;

// Neighbour pair sums of the LDS array u at site (x, y, z): x pair, then y,
// then z, as the marching kernels form them.
template <typename T, int R, int NDIM>
__device__ __forceinline__ void tiny_pairs(const T *u, int32_t x, int32_t y, int32_t z, int32_t nx,
                                           int32_t ny, int32_t nz, T (&S)[R])
{
    const int32_t row = (z * ny + y) * nx;
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        T acc = u[row + wrap32(x + j, nx)] + u[row + wrap32(x - j, nx)];
        acc = acc + (u[(z * ny + wrap32(y + j, ny)) * nx + x] + u[(z * ny + wrap32(y - j, ny)) * nx + x]);
        if constexpr (NDIM == 3)
            acc = acc + (u[(wrap32(z + j, nz) * ny + y) * nx + x] + u[(wrap32(z - j, nz) * ny + y) * nx + x]);
        S[j - 1] = acc;
    }
}

// Calls f(i, x, y, z) for this thread's sites: column tid mod nx of rows
// tid / nx, tid / nx + rpp, .. (rpp = 1024 / nx rows per pass; threads past
// rpp nx idle).
template <typename F>
__device__ __forceinline__ void tiny_sweep(int32_t nx, int32_t ny, int32_t nz, F &&f)
{
    const int32_t rpp = kTinyThreads / nx;
    const int32_t tid = threadIdx.x;
    if (tid >= rpp * nx) return;
    const int32_t x = tid % nx, r0 = tid / nx, rows = ny * nz;
    int32_t y = r0 % ny, z = r0 / ny;
    for (int32_t row = r0; row < rows; row += rpp) {
        f(row * nx + x, x, y, z);
        y += rpp;
        while (y >= ny) {
            y -= ny;
            ++z;
        }
    }
}

template <typename T, int KIND, int R, int NDIM>
__global__ void __launch_bounds__(kTinyThreads) k_tiny(BatchTable<T> tb)
{
    constexpr int NF = nfields_kind(KIND);
    __shared__ T lds[kTinyLdsBytes / sizeof(T)];
    const int32_t n = *tb.count;
    for (int32_t e = blockIdx.x; e < n; e += gridDim.x) {
        const int32_t steps = tb.steps[e];  // uniform over the workgroup
        if (steps <= 0) continue;
        const StepArgs<T> &a = tb.args[e];
        const int32_t nx = (int32_t)a.nx, ny = (int32_t)a.ny, nz = (int32_t)a.nz;
        const int32_t N = nx * ny * nz;
        T *cur[NF], *nxt[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cur[f] = lds + f * N;
            nxt[f] = lds + (NF + f) * N;
        }
        T *aux = lds + 2 * NF * N;
        const int par = a.parity;
        const T ctr = T(2 * NDIM);
        tiny_sweep(nx, ny, nz, [&](int32_t i, int32_t x, int32_t y, int32_t z) {
            const int64_t off = (int64_t)z * a.plane + (int64_t)y * a.pitch + x;
#pragma unroll
            for (int f = 0; f < NF; ++f) cur[f][i] = a.buf[f][par][off];
        });
        __syncthreads();
        for (int32_t s = 0; s < steps; ++s) {
            if constexpr (KIND == kCH || KIND == kMC) {  // mu (CH) or g (MC) of every site
                tiny_sweep(nx, ny, nz, [&](int32_t i, int32_t x, int32_t y, int32_t z) {
                    if constexpr (KIND == kCH) {
                        T S[R];
                        tiny_pairs<T, R, NDIM>(cur[0], x, y, z, nx, ny, nz, S);
                        aux[i] = ch_mu<T, R>(a, cur[0][i], S, cur[0][i] * ctr);
                    } else {
                        aux[i] = mc_g(a, cur[0][i], cur[NF - 1][i]);
                    }
                });
                __syncthreads();
            }
            tiny_sweep(nx, ny, nz, [&](int32_t i, int32_t x, int32_t y, int32_t z) {
                const T u0 = cur[0][i];
                if constexpr (KIND == kAC) {
                    T S[R];
                    tiny_pairs<T, R, NDIM>(cur[0], x, y, z, nx, ny, nz, S);
                    nxt[0][i] = ac_update<T, R>(a, u0, S, u0 * ctr);
                } else if constexpr (KIND == kCH) {
                    T Sm[R];
                    tiny_pairs<T, R, NDIM>(aux, x, y, z, nx, ny, nz, Sm);
                    nxt[0][i] = ch_update<T, R>(a, u0, Sm, aux[i] * ctr);
                } else if constexpr (KIND == kGS) {
                    T Su[R], Sv[R];
                    tiny_pairs<T, R, NDIM>(cur[0], x, y, z, nx, ny, nz, Su);
                    tiny_pairs<T, R, NDIM>(cur[NF - 1], x, y, z, nx, ny, nz, Sv);
                    const T v0 = cur[NF - 1][i];
                    gs_update<T, R>(a, u0, v0, Su, Sv, u0 * ctr, v0 * ctr, nxt[0][i], nxt[NF - 1][i]);
                } else {
                    T Sp[R], Sg[R];
                    tiny_pairs<T, R, NDIM>(cur[0], x, y, z, nx, ny, nz, Sp);
                    tiny_pairs<T, R, NDIM>(aux, x, y, z, nx, ny, nz, Sg);
                    mc_update<T, R>(a, u0, cur[NF - 1][i], Sp, Sg, u0 * ctr, aux[i] * ctr, nxt[0][i],
                                    nxt[NF - 1][i]);
                }
            });
            __syncthreads();
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                T *t = cur[f];
                cur[f] = nxt[f];
                nxt[f] = t;
            }
        }
        tiny_sweep(nx, ny, nz, [&](int32_t i, int32_t x, int32_t y, int32_t z) {
            const int64_t off = (int64_t)z * a.plane + (int64_t)y * a.pitch + x;
#pragma unroll
            for (int f = 0; f < NF; ++f) a.buf[f][par ^ 1][off] = cur[f][i];
        });
        __syncthreads();  // the next request reuses the LDS
    }
}

// ---------------------------------------------------------------------------
// A single small 2D Allen-Cahn model stepped many times per launch: one copy
// of the grid in LDS (so FP64 grids up to 128^2 fit).  Thread t owns a
// segment of column t mod nx, rows [s L, (s + 1) L), s = t / nx, held in
// registers; per step it takes its sites' x-neighbours (and the r rows
// beyond its segment) from LDS and the rest from its registers, computes the
// segment's new values, and after a barrier writes them to LDS.  Same
// per-site functions and neighbour order as every other kernel, so the
// fields are bitwise those of steps taken one launch each.
constexpr int kLdsSegment = 16;  // rows per segment (128^2: 8 segments of 16 rows per column)

template <typename T, int R>
__global__ void __launch_bounds__(kTinyThreads) k_lds_steps(StepArgs<T> a, int32_t steps)
{
    constexpr int L = kLdsSegment;
    __shared__ T u[kTinyLdsBytes / sizeof(T)];
    const int32_t nx = (int32_t)a.nx, ny = (int32_t)a.ny;
    const int32_t tid = threadIdx.x;
    const int32_t x = tid % nx, y0 = (tid / nx) * L;
    const bool owner = y0 < ny;  // the host checks ny = L * segments with segments * nx <= 1024
    int32_t xm[R], xp[R], ym[R], yp[R];  // wrapped x-neighbours; LDS index of the rows beyond the segment
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        xp[j - 1] = wrap32(x + j, nx);
        xm[j - 1] = wrap32(x - j, nx);
        yp[j - 1] = wrap32(y0 + L - 1 + j, ny) * nx + x;
        ym[j - 1] = wrap32(y0 - j, ny) * nx + x;
    }
    const T ctr = T(4);
    const int par = a.parity;
    // c: the segment's values; the new value of row k replaces c[k - r] once
    // row k is computed (later rows need only rows from k + 1 - r on), so
    // r + 1 new values wait in nv
    T c[L], nv[R + 1];
    if (owner) {
#pragma unroll
        for (int k = 0; k < L; ++k) {
            c[k] = a.buf[0][par][(int64_t)(y0 + k) * a.pitch + x];
            u[(y0 + k) * nx + x] = c[k];
        }
    }
    __syncthreads();
    for (int32_t s = 0; s < steps; ++s) {
        if (owner) {
            static_for<0, L>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                const int32_t row = (y0 + k) * nx;
                T S[R];
                static_for<1, R + 1>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    T p, m;
                    if constexpr (k + j < L)
                        p = c[k + j];
                    else
                        p = u[yp[k + j - L]];
                    if constexpr (k - j >= 0)
                        m = c[k - j];
                    else
                        m = u[ym[j - k - 1]];
                    S[j - 1] = (u[row + xp[j - 1]] + u[row + xm[j - 1]]) + (p + m);
                });
                const T u0 = c[k];
                if constexpr (k >= R) c[k - R] = nv[(k - R) % (R + 1)];
                nv[k % (R + 1)] = ac_update<T, R>(a, u0, S, u0 * ctr);
            });
            static_for<L - R, L>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                c[k] = nv[k % (R + 1)];
            });
        }
        __syncthreads();
        if (owner) {
#pragma unroll
            for (int k = 0; k < L; ++k) u[(y0 + k) * nx + x] = c[k];
        }
        __syncthreads();
    }
    if (owner) {
        T *out = a.buf[0][par ^ (steps & 1)];
#pragma unroll
        for (int k = 0; k < L; ++k) out[(int64_t)(y0 + k) * a.pitch + x] = c[k];
    }
}

// Whole-wave lane rotations by DPP: lane i receives lane i + 1 (wave_rol:1)
// or lane i - 1 (wave_ror:1), lane 63 and lane 0 wrapping round.
__device__ __forceinline__ int rot_from_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x134, 0xF, 0xF, false); }
__device__ __forceinline__ int rot_from_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x13C, 0xF, 0xF, false); }
template <bool NEXT>
__device__ __forceinline__ float rot_lane(float x)
{
    const int v = __builtin_bit_cast(int, x);
    return __builtin_bit_cast(float, NEXT ? rot_from_next(v) : rot_from_prev(v));
}
template <bool NEXT>
__device__ __forceinline__ double rot_lane(double x)
{
    const long long b = __builtin_bit_cast(long long, x);
    int lo = (int)b, hi = (int)(b >> 32);
    lo = NEXT ? rot_from_next(lo) : rot_from_prev(lo);
    hi = NEXT ? rot_from_next(hi) : rot_from_prev(hi);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Whole-grid steps for 2D Allen-Cahn with r <= W on nx = 64 W columns and
// ny = 16 LR rows: wave w of the 16 holds rows [w LR, (w + 1) LR) in
// registers, lane l columns [l W, (l + 1) W), so that one wave spans a whole
// periodic row and x-neighbours across lanes are lane rotations (r <= W keeps
// them within the next lane).  Only the first and last r rows of each wave
// cross waves: they go through an LDS array of 16 x 2r rows, double-buffered
// by step parity, so one barrier per step.  The site arithmetic is that of
// every other kernel (same order).
constexpr int kRowWaves = 16;

template <typename T, int R, int W, int LR>
__global__ void __launch_bounds__(64 * kRowWaves) k_lds_rows(StepArgs<T> a, int32_t steps)
{
    static_assert(R <= W && R <= LR, "neighbours within the next lane and the next wave");
    constexpr int NX = 64 * W;
    // [step parity][wave][first r rows, then last r rows][x]
    __shared__ T bnd[2][kRowWaves][2 * R][NX];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    const int wu = (w + kRowWaves - 1) % kRowWaves, wd = (w + 1) % kRowWaves;
    const int32_t y0 = w * LR, x0 = l * W;
    const T ctr = T(4);
    const int par = a.parity;
    T c[2][W][LR];  // ping-pong: the state and the next state
#pragma unroll
    for (int k = 0; k < LR; ++k)
#pragma unroll
        for (int i = 0; i < W; ++i) c[0][i][k] = a.buf[0][par][(int64_t)(y0 + k) * a.pitch + x0 + i];
    auto put_edges = [&](auto sc, int b) {
        constexpr int S = decltype(sc)::value;
#pragma unroll
        for (int t = 0; t < R; ++t)
#pragma unroll
            for (int i = 0; i < W; ++i) {
                bnd[b][w][t][x0 + i] = c[S][i][t];
                bnd[b][w][R + t][x0 + i] = c[S][i][LR - R + t];
            }
    };
    put_edges(std::integral_constant<int, 0>{}, 0);
    __syncthreads();
    // one step from c[S] into c[S ^ 1], reading the edge rows of parity b
    auto step = [&](auto sc, int b) {
        constexpr int S = decltype(sc)::value;
        T up[R][W], dn[R][W];  // up[m]: row y0 - 1 - m; dn[m]: row y0 + LR + m
#pragma unroll
        for (int m = 0; m < R; ++m)
#pragma unroll
            for (int i = 0; i < W; ++i) {
                up[m][i] = bnd[b][wu][2 * R - 1 - m][x0 + i];
                dn[m][i] = bnd[b][wd][m][x0 + i];
            }
        static_for<0, LR>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            // columns x0 - W + q (q >= W - r) of lane l - 1, x0 + W + q (q < r) of lane l + 1
            T left[W], right[W];
            static_for<W - R, W>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                left[q] = rot_lane<false>(c[S][q][k]);
            });
            static_for<0, R>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                right[q] = rot_lane<true>(c[S][q][k]);
            });
            static_for<0, W>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                T Sx[R];
                static_for<1, R + 1>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    T xp, xm, p, m;
                    if constexpr (i + j < W)
                        xp = c[S][i + j][k];
                    else
                        xp = right[i + j - W];
                    if constexpr (i - j >= 0)
                        xm = c[S][i - j][k];
                    else
                        xm = left[i - j + W];
                    if constexpr (k + j < LR)
                        p = c[S][i][k + j];
                    else
                        p = dn[k + j - LR][i];
                    if constexpr (k - j >= 0)
                        m = c[S][i][k - j];
                    else
                        m = up[j - k - 1][i];
                    Sx[j - 1] = (xp + xm) + (p + m);
                });
                const T u0 = c[S][i][k];
                c[S ^ 1][i][k] = ac_update<T, R>(a, u0, Sx, u0 * ctr);
            });
        });
        put_edges(std::integral_constant<int, S ^ 1>{}, b ^ 1);
        __syncthreads();
    };
    // an odd step count takes its extra step first, so that the state ends in
    // c[0] (indices known at compile time keep c in registers)
    int b = 0;
    if (steps & 1) {
        step(std::integral_constant<int, 0>{}, b);
        b ^= 1;
#pragma unroll
        for (int k = 0; k < LR; ++k)
#pragma unroll
            for (int i = 0; i < W; ++i) c[0][i][k] = c[1][i][k];
    }
    for (int32_t s = steps & 1; s < steps; s += 2) {
        step(std::integral_constant<int, 0>{}, b);
        step(std::integral_constant<int, 1>{}, b ^ 1);
    }
    T *out = a.buf[0][par ^ (steps & 1)];
#pragma unroll
    for (int k = 0; k < LR; ++k)
#pragma unroll
        for (int i = 0; i < W; ++i) out[(int64_t)(y0 + k) * a.pitch + x0 + i] = c[0][i][k];
}

// (W, LR) of the row kernel for a grid, or W = 0
static void lds_rows_shape(const Launch &L, int64_t nx, int64_t ny, int64_t nz, int *W, int *LR)
{
    *W = 0;
    *LR = 0;
    if (L.kind != kAC || L.ndim != 2 || L.r < 1 || L.r > 2 || nz != 1) return;
    if ((nx != 64 && nx != 128) || (ny != 16 * 4 && ny != 16 * 8)) return;
    if (L.r > nx / 64) return;  // r <= W
    *W = (int)(nx / 64);
    *LR = (int)(ny / 16);
}

}  // namespace

bool lds_steps_available(const Launch &L, int64_t nx, int64_t ny, int64_t nz)
{
    // 2D, r <= 2, ny a multiple of the segment length with every segment of
    // every column a thread of one workgroup
    if (L.kind != kAC || L.ndim != 2 || L.r < 1 || L.r > 2 || nz != 1) return false;
    if (nx < 1 || ny < kLdsSegment || ny % kLdsSegment != 0) return false;
    if ((ny / kLdsSegment) * nx > kTinyThreads) return false;
    return nx * ny * (L.fp32 ? 4 : 8) <= kTinyLdsBytes;
}

hipError_t launch_lds_steps(const Launch &L, const void *args, int32_t steps, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (steps < 1) return err;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        if (!lds_steps_available(L, a.nx, a.ny, a.nz)) return;
        int W, LR;
        lds_rows_shape(L, a.nx, a.ny, a.nz, &W, &LR);
        if (W) {
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(1), dim3(64 * kRowWaves), 0, s, a, steps);
                err = hipGetLastError();
            };
            if (L.r == 1 && W == 1 && LR == 4) go(k_lds_rows<T, 1, 1, 4>);
            if (L.r == 1 && W == 1 && LR == 8) go(k_lds_rows<T, 1, 1, 8>);
            if (L.r == 1 && W == 2 && LR == 4) go(k_lds_rows<T, 1, 2, 4>);
            if (L.r == 1 && W == 2 && LR == 8) go(k_lds_rows<T, 1, 2, 8>);
            if (L.r == 2 && W == 2 && LR == 4) go(k_lds_rows<T, 2, 2, 4>);
            if (L.r == 2 && W == 2 && LR == 8) go(k_lds_rows<T, 2, 2, 8>);
            return;
        }
        dispatch_r(L.r, RList<1, 2>{}, [&](auto rc) {
            hipLaunchKernelGGL((k_lds_steps<T, decltype(rc)::value>), dim3(1), dim3(kTinyThreads), 0, s, a, steps);
            err = hipGetLastError();
        });
    });
    return err;
}

bool tiny_available(const Launch &L, int64_t nx, int64_t ny, int64_t nz)
{
    if (L.ndim < 2 || L.r < 1 || L.r > 4) return false;
    if (L.kind != kAC && L.kind != kCH && L.kind != kGS && L.kind != kMC) return false;
    if (nx > kTinyThreads || ny > 1 << 20 || nz > 1 << 20) return false;
    const int64_t N = nx * ny * nz;
    const int nf = nfields_kind(L.kind), arrays = 2 * nf + ((L.kind == kCH || L.kind == kMC) ? 1 : 0);
    return arrays * N * (L.fp32 ? 4 : 8) <= kTinyLdsBytes;
}

hipError_t launch_tiny(const Launch &L, const void *table, int32_t blocks, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const BatchTable<T> &t = *static_cast<const BatchTable<T> *>(table);
        dispatch_kind(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            dispatch_r(L.r, RList<1, 2, 3, 4>{}, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                if (L.ndim == 2)
                    hipLaunchKernelGGL((k_tiny<T, KIND, R, 2>), dim3(blocks), dim3(kTinyThreads), 0, s, t);
                else
                    hipLaunchKernelGGL((k_tiny<T, KIND, R, 3>), dim3(blocks), dim3(kTinyThreads), 0, s, t);
                err = hipGetLastError();
            });
        });
    });
    return err;
}

}  // namespace pf
