// Device code shared by all step kernels of libpfmi (gfx950, wave64).
//
// Per-site arithmetic lives in one set of inline functions so that every
// kernel family (fused marching, per-site generic, batched serving) produces
// bitwise identical fields: the neighbour sums are formed in the fixed order
// x, then y, then z, every multiply-add is an explicit fma(), and the code is
// built with -ffp-contract=off so nothing else is fused.
#pragma once

#include <type_traits>

#include "pf_internal.h"

namespace pf {

template <typename T> struct Vec;
template <> struct Vec<double> { static constexpr int V = 2; };
template <> struct Vec<float> { static constexpr int V = 4; };

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

__device__ __forceinline__ int64_t wrap_any(int64_t i, int64_t n)
{
    if (i >= 0 && i < n) return i;
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

// 16-byte vector access of V consecutive values.
__device__ __forceinline__ void vload(const double *p, double (&o)[2])
{
    const double2 q = *reinterpret_cast<const double2 *>(p);
    o[0] = q.x;
    o[1] = q.y;
}
__device__ __forceinline__ void vload(const float *p, float (&o)[4])
{
    const float4 q = *reinterpret_cast<const float4 *>(p);
    o[0] = q.x;
    o[1] = q.y;
    o[2] = q.z;
    o[3] = q.w;
}
__device__ __forceinline__ void vstore(double *p, const double (&o)[2])
{
    *reinterpret_cast<double2 *>(p) = make_double2(o[0], o[1]);
}
__device__ __forceinline__ void vstore(float *p, const float (&o)[4])
{
    *reinterpret_cast<float4 *>(p) = make_float4(o[0], o[1], o[2], o[3]);
}

// ---------------------------------------------------------------------------
// Compensated FP64 accumulation (TwoSum of Knuth; the low parts are summed
// plainly).  Used for every mass / energy reduction.
struct Acc {
    double hi, lo;
};
__device__ __forceinline__ void acc_add(Acc &a, double x)
{
    const double s = a.hi + x;
    const double bp = s - a.hi;
    const double e = (a.hi - (s - bp)) + (x - bp);
    a.hi = s;
    a.lo += e;
}
__device__ __forceinline__ void acc_merge(Acc &a, const Acc &b)
{
    acc_add(a, b.hi);
    a.lo += b.lo;
}
// Butterfly over the 64 lanes in a fixed order; lane 0 holds the result.
__device__ __forceinline__ Acc wave_reduce(Acc a)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Acc b;
        b.hi = __shfl_xor(a.hi, off);
        b.lo = __shfl_xor(a.lo, off);
        acc_merge(a, b);
    }
    return a;
}
__device__ __forceinline__ double wave_sum_exact(double c)
{
    // counts are small integers: any order is exact
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    return c;
}

struct RedState {
    Acc q0{0.0, 0.0}, q1{0.0, 0.0};
    double bad = 0.0;
};

__device__ __forceinline__ void red_flush(const RedState &r, double2 *part, int64_t pstride,
                                          int64_t slot, int lane)
{
    const Acc a = wave_reduce(r.q0);
    const Acc b = wave_reduce(r.q1);
    const double c = wave_sum_exact(r.bad);
    if (lane == 0) {
        part[slot] = make_double2(a.hi, a.lo);
        part[pstride + slot] = make_double2(b.hi, b.lo);
        part[2 * pstride + slot] = make_double2(c, 0.0);
    }
}

__device__ __forceinline__ bool finite_val(double x) { return isfinite(x); }

// ---------------------------------------------------------------------------
// Per-site model arithmetic.  S[j-1] is the sum of the 2*ndim neighbours at
// distance j (pairs added axis by axis: x, then y, then z); ctr = 2*ndim*u0.
// Each stencil term is fma(w_j, S_j - ctr, acc), the difference form that
// keeps a constant field an exact zero of the Laplacian.

// Allen-Cahn (Eq. model-a), forward Euler: k0 = dt c1, k1 = dt c2, wu = dt w_j/dx^2.
template <typename T, int R>
__device__ __forceinline__ T ac_update(const StepArgs<T> &a, T u0, const T (&S)[R], T ctr)
{
    const T g = fma(-(a.k1 * u0), u0, a.k0);  // dt (c1 - c2 u0^2)
    T acc = fma(g, u0, u0);
#pragma unroll
    for (int j = 0; j < R; ++j) acc = fma(a.wu[j], S[j] - ctr, acc);
    return acc;
}

// Cahn-Hilliard (Eq. model-b) chemical potential mu = c2 c^3 - c1 c - L c:
// k0 = c1, k1 = c2, wi = w_j/dx^2.  Also returns L c.
template <typename T, int R>
__device__ __forceinline__ T ch_mu(const StepArgs<T> &a, T c0, const T (&S)[R], T ctr)
{
    T lc = T(0);
#pragma unroll
    for (int j = 0; j < R; ++j) lc = fma(a.wi[j], S[j] - ctr, lc);
    return fma(a.k1 * c0, c0 * c0, -(a.k0 * c0)) - lc;
}
// Cahn-Hilliard update c' = c + dt L mu: wu = dt w_j/dx^2, S from mu.
template <typename T, int R>
__device__ __forceinline__ T ch_update(const StepArgs<T> &a, T c0, const T (&Sm)[R], T ctrm)
{
    T acc = c0;
#pragma unroll
    for (int j = 0; j < R; ++j) acc = fma(a.wu[j], Sm[j] - ctrm, acc);
    return acc;
}

// Gray-Scott: k0 = dt F, k1 = dt (F + k), k2 = dt, wu = dt Du w_j/dx^2,
// wv = dt Dv w_j/dx^2.
template <typename T, int R>
__device__ __forceinline__ void gs_update(const StepArgs<T> &a, T u0, T v0, const T (&Su)[R],
                                          const T (&Sv)[R], T ctru, T ctrv, T &un, T &vn)
{
    const T uvv = (u0 * v0) * v0;
    const T ru = fma(a.k0, T(1) - u0, -(a.k2 * uvv));
    const T rv = fma(a.k2, uvv, -(a.k1 * v0));
    T au = u0 + ru, av = v0 + rv;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        au = fma(a.wu[j], Su[j] - ctru, au);
        av = fma(a.wv[j], Sv[j] - ctrv, av);
    }
    un = au;
    vn = av;
}

// Landau free-energy density in FP64 at a site: -(1/2) x Lx + (c2/4) x^4 -
// (c1/2) x^2, with Lx from FP64 neighbour sums S64 (same pairing order).
template <int R>
__device__ __forceinline__ double energy_density(double c1, double c2, const double *w64,
                                                 double x, const double (&S64)[R],
                                                 double ctr64)
{
    double lx = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) lx = fma(w64[j], S64[j] - ctr64, lx);
    const double x2 = x * x;
    return fma(-0.5 * x, lx, x2 * fma(0.25 * c2, x2, -0.5 * c1));
}

// ---------------------------------------------------------------------------
// Work-item order: workgroups are dealt to the 8 XCDs round-robin
// (blockIdx % 8); remap so that each XCD runs one contiguous range of items,
// keeping neighbouring strips (which share halo columns) in one L2.
__device__ __forceinline__ int32_t xcd_item(int32_t b, int32_t nwg)
{
    const int32_t x = b & 7, q = b >> 3;
    const int32_t per = nwg >> 3, rem = nwg & 7;
    return x * per + (x < rem ? x : rem) + q;
}

// Gather the x-neighbourhood of a lane's V values: e[(d + D) V + v] holds
// element v of lane (lane + d), d = -D..D.  Edge lanes receive values from
// the other end of the wave; their results are masked as halo.
template <typename T, int V, int D>
__device__ __forceinline__ void gather_x(const T (&c)[V], T (&e)[(2 * D + 1) * V])
{
#pragma unroll
    for (int v = 0; v < V; ++v) e[D * V + v] = c[v];
#pragma unroll
    for (int d = 1; d <= D; ++d) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            e[(D + d) * V + v] = __shfl_down(c[v], d);
            e[(D - d) * V + v] = __shfl_up(c[v], d);
        }
    }
}

template <typename T, int KIND, int R>
struct Shape {
    static constexpr int V = Vec<T>::V;
    static constexpr int H = KIND == kCH ? 2 * R : R;  // halo of one step
    static constexpr int HV = (H + V - 1) / V * V;     // halo rounded to whole lanes
    static constexpr int SW = 64 * V;                  // strip width (loaded columns)
    static constexpr int OWMAX = SW - 2 * HV;          // most outputs per strip
    static constexpr int D = (R + V - 1) / V;          // neighbour lanes per side
    static constexpr int NE = (2 * D + 1) * V;
    static constexpr int K = 2 * R + 1;                // ring length (rows or planes)
    static constexpr int NF = KIND == kGS ? 2 : 1;
};

// Load the lane's V values of one row (x from xl, wrapped per element unless
// the whole strip lies inside the row).
template <typename T, int V>
__device__ __forceinline__ void load_row(const T *__restrict__ row, int64_t xl, int64_t nx,
                                         bool fast, T (&o)[V])
{
    if (fast) {
        vload(row + xl, o);
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = row[wrap_any(xl + v, nx)];
    }
}

template <typename T, int V>
__device__ __forceinline__ void store_row(T *__restrict__ row, int64_t xl, bool all,
                                          const bool (&ov)[V], const T (&o)[V])
{
    if (all) {
        vstore(row + xl, o);
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (ov[v]) row[xl + v] = o[v];
    }
}

// ===========================================================================
// 2D fused marching step.  One wave owns a strip of SW = 64 V columns (V
// values per lane, x-neighbours by lane shuffles) and marches along y over
// one chunk of output rows, keeping the last K = 2r+1 rows of every field
// (and for CH of mu) in registers.  Loads run K rows ahead (prefetch ring).
// CH computes mu = c2 c^3 - c1 c - L c for row t - r and the update for row
// t - 2r in the same sweep: the biharmonic never touches memory.
template <typename T, int KIND, int R, bool RED>
__device__ __forceinline__ void step2d_item(const StepArgs<T> &a, int par, int32_t item,
                                            int lane, int64_t pslot)
{
    using S = Shape<T, KIND, R>;
    constexpr int V = S::V, H = S::H, HV = S::HV, SW = S::SW, D = S::D, NE = S::NE, K = S::K,
                  NF = S::NF;
    const int32_t strip = item % a.strips;
    const int32_t chunk = item / a.strips;
    const int64_t nx = a.nx, ny = a.ny, pitch = a.pitch;
    const int64_t x0 = (int64_t)strip * a.ow;
    const int64_t xb = x0 - HV;
    const int64_t xl = xb + lane * V;
    const bool fast = (xb >= 0) && (xb + SW <= nx);
    const int64_t y0 = (int64_t)chunk * a.clen;
    const int64_t y1 = min(y0 + (int64_t)a.clen, ny);
    const int pl = lane * V;
    bool ov[V];
    bool allv = true;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        ov[v] = (pl + v >= HV) && (pl + v < HV + a.ow) && (xl + v < nx);
        allv = allv && ov[v];
    }
    const T *in[2] = {a.buf[0][par], a.buf[NF - 1][par]};
    T *out[2] = {a.buf[0][par ^ 1], a.buf[NF - 1][par ^ 1]};

    T ring[NF][K][V];
    T pre[NF][K][V];
    T mring[KIND == kCH ? K : 1][V];
    RedState red;

    const int64_t tb0 = y0 - H, tend = y1 + H;
    static_for<0, K>([&](auto phc) {
        constexpr int ph = decltype(phc)::value;
        const int64_t t = tb0 + ph;
        if (t < tend) {
            const int64_t off = wrap_any(t, ny) * pitch;
#pragma unroll
            for (int f = 0; f < NF; ++f) load_row<T, V>(in[f] + off, xl, nx, fast, pre[f][ph]);
        }
    });

    for (int64_t tb = tb0; tb < tend; tb += K) {
        static_for<0, K>([&](auto phc) {
            constexpr int ph = decltype(phc)::value;
            const int64_t t = tb + ph;
            if (t < tend) {
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int v = 0; v < V; ++v) ring[f][ph][v] = pre[f][ph][v];
                if (t + K < tend) {
                    const int64_t off = wrap_any(t + K, ny) * pitch;
#pragma unroll
                    for (int f = 0; f < NF; ++f)
                        load_row<T, V>(in[f] + off, xl, nx, fast, pre[f][ph]);
                }
                if constexpr (KIND != kCH) {
                    constexpr int co = (ph - R + K) % K;
                    const int64_t o = t - R;
                    if (o >= y0) {
                        T e[NF][NE];
#pragma unroll
                        for (int f = 0; f < NF; ++f) gather_x<T, V, D>(ring[f][co], e[f]);
                        T res[NF][V];
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            T Sf[NF][R];
                            static_for<1, R + 1>([&](auto jc) {
                                constexpr int j = decltype(jc)::value;
                                constexpr int sp = (co + j) % K, sm = (co - j + K) % K;
#pragma unroll
                                for (int f = 0; f < NF; ++f)
                                    Sf[f][j - 1] = (e[f][D * V + v + j] + e[f][D * V + v - j]) +
                                                   (ring[f][sp][v] + ring[f][sm][v]);
                            });
                            const T u0 = ring[0][co][v];
                            if constexpr (KIND == kAC) {
                                res[0][v] = ac_update<T, R>(a, u0, Sf[0], u0 * T(4));
                            } else {
                                const T v0 = ring[NF - 1][co][v];
                                gs_update<T, R>(a, u0, v0, Sf[0], Sf[NF - 1], u0 * T(4),
                                                v0 * T(4), res[0][v], res[NF - 1][v]);
                            }
                            if constexpr (RED) {
                                if (ov[v]) {
                                    const double x = (double)u0;
                                    acc_add(red.q0, x);
                                    red.bad += finite_val(x) ? 0.0 : 1.0;
                                    if constexpr (KIND == kAC) {
                                        double S64[R];
                                        static_for<1, R + 1>([&](auto jc) {
                                            constexpr int j = decltype(jc)::value;
                                            constexpr int sp = (co + j) % K, sm = (co - j + K) % K;
                                            S64[j - 1] = ((double)e[0][D * V + v + j] +
                                                          (double)e[0][D * V + v - j]) +
                                                         ((double)ring[0][sp][v] +
                                                          (double)ring[0][sm][v]);
                                        });
                                        acc_add(red.q1, energy_density<R>(a.c1, a.c2, a.w64, x,
                                                                          S64, x * 4.0));
                                    } else {
                                        const double y = (double)ring[NF - 1][co][v];
                                        acc_add(red.q1, y);
                                        red.bad += finite_val(y) ? 0.0 : 1.0;
                                    }
                                }
                            }
                        }
                        const int64_t ooff = wrap_any(o, ny) * pitch;
#pragma unroll
                        for (int f = 0; f < NF; ++f) store_row<T, V>(out[f] + ooff, xl, allv, ov, res[f]);
                    }
                } else {
                    // chemical potential of row m = t - r
                    constexpr int cm = (ph - R + K) % K;
                    const int64_t m = t - R;
                    if (m >= y0 - R) {
                        T e[NE];
                        gather_x<T, V, D>(ring[0][cm], e);
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            T Sc[R];
                            static_for<1, R + 1>([&](auto jc) {
                                constexpr int j = decltype(jc)::value;
                                constexpr int sp = (cm + j) % K, sm = (cm - j + K) % K;
                                Sc[j - 1] = (e[D * V + v + j] + e[D * V + v - j]) +
                                            (ring[0][sp][v] + ring[0][sm][v]);
                            });
                            const T c0 = ring[0][cm][v];
                            mring[cm][v] = ch_mu<T, R>(a, c0, Sc, c0 * T(4));
                            if constexpr (RED) {
                                if (ov[v] && m >= y0 && m < y1) {
                                    const double x = (double)c0;
                                    double S64[R];
                                    static_for<1, R + 1>([&](auto jc) {
                                        constexpr int j = decltype(jc)::value;
                                        constexpr int sp = (cm + j) % K, sm = (cm - j + K) % K;
                                        S64[j - 1] = ((double)e[D * V + v + j] +
                                                      (double)e[D * V + v - j]) +
                                                     ((double)ring[0][sp][v] +
                                                      (double)ring[0][sm][v]);
                                    });
                                    acc_add(red.q0, x);
                                    acc_add(red.q1,
                                            energy_density<R>(a.c1, a.c2, a.w64, x, S64, x * 4.0));
                                    red.bad += finite_val(x) ? 0.0 : 1.0;
                                }
                            }
                        }
                    }
                    // update of row o = t - 2r
                    constexpr int co = (ph - 2 * R + K) % K;
                    const int64_t o = t - 2 * R;
                    if (o >= y0) {
                        T em[NE];
                        gather_x<T, V, D>(mring[co], em);
                        T res[V];
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            T Sm[R];
                            static_for<1, R + 1>([&](auto jc) {
                                constexpr int j = decltype(jc)::value;
                                constexpr int sp = (co + j) % K, sm = (co - j + K) % K;
                                Sm[j - 1] = (em[D * V + v + j] + em[D * V + v - j]) +
                                            (mring[sp][v] + mring[sm][v]);
                            });
                            res[v] = ch_update<T, R>(a, ring[0][co][v], Sm, mring[co][v] * T(4));
                        }
                        store_row<T, V>(out[0] + wrap_any(o, ny) * pitch, xl, allv, ov, res);
                    }
                }
            }
        });
    }
    if constexpr (RED) red_flush(red, a.part, a.pstride, pslot, lane);
}

template <typename T, int KIND, int R, bool RED>
__global__ void __launch_bounds__(64 * kWaves2D) k_step2d(StepArgs<T> a)
{
    const int32_t nwg = gridDim.x;
    const int32_t wg = xcd_item(blockIdx.x, nwg);
    const int32_t item = wg * kWaves2D + (threadIdx.x >> 6);
    if (item >= a.items) return;
    step2d_item<T, KIND, R, RED>(a, a.parity, item, threadIdx.x & 63, item);
}

template <typename T, int KIND, int R>
__global__ void __launch_bounds__(64 * kWaves2D) k_step2d_batched(BatchTable<T> tb, int32_t k)
{
    const int32_t nwg = gridDim.x;
    const int32_t g = xcd_item(blockIdx.x, nwg) * kWaves2D + (threadIdx.x >> 6);
    if (g >= tb.item_start[tb.n]) return;
    int lo = 0, hi = tb.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tb.item_start[mid] <= g) lo = mid; else hi = mid - 1;
    }
    if (k >= tb.steps[lo]) return;
    const StepArgs<T> &a = tb.args[lo];
    step2d_item<T, KIND, R, false>(a, (a.parity + k) & 1, g - tb.item_start[lo],
                                   threadIdx.x & 63, 0);
}

// ===========================================================================
// 3D fused marching step.  A workgroup of NW = 16 waves owns a tile of 16
// rows (y) of one x-strip and marches along z.  Wave w holds tile row
// y0 - H + w; its z-window of K planes stays in registers, x-neighbours come
// from lane shuffles and y-neighbours from the other waves' rows through a
// double-buffered LDS plane (one barrier per plane).  Rows within H of the
// tile edge are halo: only rows [H, NW - H) are written.
template <typename T, int KIND, int R, bool RED>
__device__ __forceinline__ void step3d_item(const StepArgs<T> &a, int par, int32_t item,
                                            int64_t pslot_base)
{
    using S = Shape<T, KIND, R>;
    constexpr int V = S::V, H = S::H, HV = S::HV, SW = S::SW, D = S::D, NE = S::NE, K = S::K,
                  NF = S::NF;
    constexpr int NW = kWaves3D;
    constexpr int NL = KIND == kCH ? 2 : NF;  // LDS planes per buffer
    static_assert(2 * H < NW, "halo too wide for the 3D tile");
    __shared__ T lds[2][NL][NW][SW];

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int32_t strip = item % a.strips;
    const int32_t rest = item / a.strips;
    const int32_t ytile = rest % a.ytiles;
    const int32_t chunk = rest / a.ytiles;
    const int64_t nx = a.nx, ny = a.ny, nz = a.nz, pitch = a.pitch, plane = a.plane;
    const int64_t x0 = (int64_t)strip * a.ow;
    const int64_t xb = x0 - HV;
    const int64_t xl = xb + lane * V;
    const bool fast = (xb >= 0) && (xb + SW <= nx);
    const int64_t yo0 = (int64_t)ytile * (NW - 2 * H);      // first output row of the tile
    const int64_t yrow = yo0 - H + w;                        // this wave's row
    const bool out_row = (w >= H) && (w < NW - H) && (yrow < ny);
    const int64_t rowoff = wrap_any(yrow, ny) * pitch;
    const int64_t z0 = (int64_t)chunk * a.clen;
    const int64_t z1 = min(z0 + (int64_t)a.clen, nz);
    const int pl = lane * V;
    bool ov[V];
    bool allv = true;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        ov[v] = out_row && (pl + v >= HV) && (pl + v < HV + a.ow) && (xl + v < nx);
        allv = allv && ov[v];
    }
    const T *in[2] = {a.buf[0][par], a.buf[NF - 1][par]};
    T *out[2] = {a.buf[0][par ^ 1], a.buf[NF - 1][par ^ 1]};

    T ring[NF][K][V];
    T pre[NF][K][V];
    T mring[KIND == kCH ? K : 1][V];
    RedState red;

    const int64_t tb0 = z0 - H, tend = z1 + H;
    static_for<0, K>([&](auto phc) {
        constexpr int ph = decltype(phc)::value;
        const int64_t t = tb0 + ph;
        if (t < tend) {
            const int64_t off = wrap_any(t, nz) * plane + rowoff;
#pragma unroll
            for (int f = 0; f < NF; ++f) load_row<T, V>(in[f] + off, xl, nx, fast, pre[f][ph]);
        }
    });

    for (int64_t tb = tb0; tb < tend; tb += K) {
        static_for<0, K>([&](auto phc) {
            constexpr int ph = decltype(phc)::value;
            const int64_t t = tb + ph;
            if (t < tend) {
                const int buf = (int)(t & 1);
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int v = 0; v < V; ++v) ring[f][ph][v] = pre[f][ph][v];
                if (t + K < tend) {
                    const int64_t off = wrap_any(t + K, nz) * plane + rowoff;
#pragma unroll
                    for (int f = 0; f < NF; ++f)
                        load_row<T, V>(in[f] + off, xl, nx, fast, pre[f][ph]);
                }
                if constexpr (KIND != kCH) {
                    constexpr int co = (ph - R + K) % K;
                    const int64_t o = t - R;
#pragma unroll
                    for (int f = 0; f < NF; ++f)
#pragma unroll
                        for (int v = 0; v < V; ++v) lds[buf][f][w][pl + v] = ring[f][co][v];
                    __syncthreads();
                    if (o >= z0 && w >= R && w < NW - R) {
                        T e[NF][NE];
#pragma unroll
                        for (int f = 0; f < NF; ++f) gather_x<T, V, D>(ring[f][co], e[f]);
                        T res[NF][V];
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            T Sf[NF][R];
                            static_for<1, R + 1>([&](auto jc) {
                                constexpr int j = decltype(jc)::value;
                                constexpr int sp = (co + j) % K, sm = (co - j + K) % K;
#pragma unroll
                                for (int f = 0; f < NF; ++f)
                                    Sf[f][j - 1] =
                                        ((e[f][D * V + v + j] + e[f][D * V + v - j]) +
                                         (lds[buf][f][w + j][pl + v] + lds[buf][f][w - j][pl + v])) +
                                        (ring[f][sp][v] + ring[f][sm][v]);
                            });
                            const T u0 = ring[0][co][v];
                            if constexpr (KIND == kAC) {
                                res[0][v] = ac_update<T, R>(a, u0, Sf[0], u0 * T(6));
                            } else {
                                const T v0 = ring[NF - 1][co][v];
                                gs_update<T, R>(a, u0, v0, Sf[0], Sf[NF - 1], u0 * T(6),
                                                v0 * T(6), res[0][v], res[NF - 1][v]);
                            }
                            if constexpr (RED) {
                                if (ov[v]) {
                                    const double x = (double)u0;
                                    acc_add(red.q0, x);
                                    red.bad += finite_val(x) ? 0.0 : 1.0;
                                    if constexpr (KIND == kAC) {
                                        double S64[R];
                                        static_for<1, R + 1>([&](auto jc) {
                                            constexpr int j = decltype(jc)::value;
                                            constexpr int sp = (co + j) % K, sm = (co - j + K) % K;
                                            S64[j - 1] =
                                                (((double)e[0][D * V + v + j] +
                                                  (double)e[0][D * V + v - j]) +
                                                 ((double)lds[buf][0][w + j][pl + v] +
                                                  (double)lds[buf][0][w - j][pl + v])) +
                                                ((double)ring[0][sp][v] + (double)ring[0][sm][v]);
                                        });
                                        acc_add(red.q1, energy_density<R>(a.c1, a.c2, a.w64, x,
                                                                          S64, x * 6.0));
                                    } else {
                                        const double y = (double)ring[NF - 1][co][v];
                                        acc_add(red.q1, y);
                                        red.bad += finite_val(y) ? 0.0 : 1.0;
                                    }
                                }
                            }
                        }
                        if (o < z1) {
                            const int64_t ooff = wrap_any(o, nz) * plane + rowoff;
#pragma unroll
                            for (int f = 0; f < NF; ++f)
                                if (out_row) store_row<T, V>(out[f] + ooff, xl, allv, ov, res[f]);
                        }
                    }
                } else {
                    constexpr int cm = (ph - R + K) % K;
                    constexpr int co = (ph - 2 * R + K) % K;
                    const int64_t m = t - R;
                    const int64_t o = t - 2 * R;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        lds[buf][0][w][pl + v] = ring[0][cm][v];
                        lds[buf][1][w][pl + v] = mring[co][v];
                    }
                    __syncthreads();
                    if (m >= z0 - R && w >= R && w < NW - R) {
                        T e[NE];
                        gather_x<T, V, D>(ring[0][cm], e);
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            T Sc[R];
                            static_for<1, R + 1>([&](auto jc) {
                                constexpr int j = decltype(jc)::value;
                                constexpr int sp = (cm + j) % K, sm = (cm - j + K) % K;
                                Sc[j - 1] = ((e[D * V + v + j] + e[D * V + v - j]) +
                                             (lds[buf][0][w + j][pl + v] + lds[buf][0][w - j][pl + v])) +
                                            (ring[0][sp][v] + ring[0][sm][v]);
                            });
                            const T c0 = ring[0][cm][v];
                            mring[cm][v] = ch_mu<T, R>(a, c0, Sc, c0 * T(6));
                            if constexpr (RED) {
                                if (ov[v] && m >= z0 && m < z1) {
                                    const double x = (double)c0;
                                    double S64[R];
                                    static_for<1, R + 1>([&](auto jc) {
                                        constexpr int j = decltype(jc)::value;
                                        constexpr int sp = (cm + j) % K, sm = (cm - j + K) % K;
                                        S64[j - 1] =
                                            (((double)e[D * V + v + j] + (double)e[D * V + v - j]) +
                                             ((double)lds[buf][0][w + j][pl + v] +
                                              (double)lds[buf][0][w - j][pl + v])) +
                                            ((double)ring[0][sp][v] + (double)ring[0][sm][v]);
                                    });
                                    acc_add(red.q0, x);
                                    acc_add(red.q1,
                                            energy_density<R>(a.c1, a.c2, a.w64, x, S64, x * 6.0));
                                    red.bad += finite_val(x) ? 0.0 : 1.0;
                                }
                            }
                        }
                    }
                    if (o >= z0 && o < z1 && w >= 2 * R && w < NW - 2 * R) {
                        T em[NE];
                        gather_x<T, V, D>(mring[co], em);
                        T res[V];
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            T Sm[R];
                            static_for<1, R + 1>([&](auto jc) {
                                constexpr int j = decltype(jc)::value;
                                constexpr int sp = (co + j) % K, sm = (co - j + K) % K;
                                Sm[j - 1] = ((em[D * V + v + j] + em[D * V + v - j]) +
                                             (lds[buf][1][w + j][pl + v] + lds[buf][1][w - j][pl + v])) +
                                            (mring[sp][v] + mring[sm][v]);
                            });
                            res[v] = ch_update<T, R>(a, ring[0][co][v], Sm, mring[co][v] * T(6));
                        }
                        if (out_row)
                            store_row<T, V>(out[0] + wrap_any(o, nz) * plane + rowoff, xl, allv, ov,
                                            res);
                    }
                }
            }
        });
    }
    if constexpr (RED) red_flush(red, a.part, a.pstride, pslot_base + w, lane);
}

template <typename T, int KIND, int R, bool RED>
__global__ void __launch_bounds__(64 * kWaves3D) k_step3d(StepArgs<T> a)
{
    const int32_t item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= a.items) return;  // uniform over the workgroup
    step3d_item<T, KIND, R, RED>(a, a.parity, item, (int64_t)item * kWaves3D);
}

template <typename T, int KIND, int R>
__global__ void __launch_bounds__(64 * kWaves3D) k_step3d_batched(BatchTable<T> tb, int32_t k)
{
    const int32_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= tb.item_start[tb.n]) return;
    int lo = 0, hi = tb.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tb.item_start[mid] <= g) lo = mid; else hi = mid - 1;
    }
    if (k >= tb.steps[lo]) return;
    const StepArgs<T> &a = tb.args[lo];
    step3d_item<T, KIND, R, false>(a, (a.parity + k) & 1, g - tb.item_start[lo], 0);
}

}  // namespace pf
