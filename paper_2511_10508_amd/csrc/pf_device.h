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
// Field stores are streaming: nothing in the same step reads them back, so
// they are written non-temporally (they do not displace the input rows and
// halos that neighbouring strips still read from the caches).
typedef double pf_d2v __attribute__((ext_vector_type(2)));
typedef float pf_f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void vstore(double *p, const double (&o)[2])
{
    const pf_d2v v = {o[0], o[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<pf_d2v *>(p));
}
__device__ __forceinline__ void vstore(float *p, const float (&o)[4])
{
    const pf_f4v v = {o[0], o[1], o[2], o[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<pf_f4v *>(p));
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

// Landau free-energy density at a site from its chemical potential
// mu = c2 x^3 - c1 x - L x: the density -(1/2) x Lx + (c2/4) x^4 - (c1/2) x^2
// equals (1/2) x mu - (c2/4) x^4.  Used when mu is already FP64.
__device__ __forceinline__ double energy_from_mu(double c2, double x, double mu)
{
    const double x2 = x * x;
    return fma(0.5 * x, mu, -(0.25 * c2) * (x2 * x2));
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

// Whole-wave lane moves by DPP (a VALU move, no LDS round trip):
// wave_shl:1 gives lane i the value of lane i + 1, wave_shr:1 that of lane
// i - 1; lanes without a source receive 0 (they are halo lanes).
__device__ __forceinline__ int dpp_from_next(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_from_prev(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false);
}

// Value of lane (lane + D), D != 0, by |D| single-lane moves.
template <int D>
__device__ __forceinline__ float lane_shift(float x)
{
    int v = __builtin_bit_cast(int, x);
#pragma unroll
    for (int i = 0; i < (D > 0 ? D : -D); ++i) v = D > 0 ? dpp_from_next(v) : dpp_from_prev(v);
    return __builtin_bit_cast(float, v);
}
template <int D>
__device__ __forceinline__ double lane_shift(double x)
{
    const long long b = __builtin_bit_cast(long long, x);
    int lo = (int)b, hi = (int)(b >> 32);
#pragma unroll
    for (int i = 0; i < (D > 0 ? D : -D); ++i) {
        lo = D > 0 ? dpp_from_next(lo) : dpp_from_prev(lo);
        hi = D > 0 ? dpp_from_next(hi) : dpp_from_prev(hi);
    }
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Gather the x-neighbourhood a radius-R stencil needs around a lane's V
// values: e[k + R] is the value at column offset k (k = -R .. V-1+R) from the
// lane's first column, taken from lane floor(k / V) away.  Edge lanes receive
// zeros or values from beyond the strip; their results are masked as halo.
template <typename T, int V, int R>
__device__ __forceinline__ void gather_x(const T (&c)[V], T (&e)[V + 2 * R])
{
    static_for<0, V + 2 * R>([&](auto kc) {
        constexpr int k = decltype(kc)::value - R;
        constexpr int d = k >= 0 ? k / V : -((-k + V - 1) / V);
        constexpr int el = k - d * V;
        if constexpr (d == 0)
            e[k + R] = c[el];
        else
            e[k + R] = lane_shift<d>(c[el]);
    });
}

template <typename T, int KIND, int R, int TB = 1>
struct Shape {
    static constexpr int V = Vec<T>::V;
    static constexpr int H = (KIND == kCH ? 2 * R : R) * TB;  // halo of TB fused steps
    static constexpr int HV = (H + V - 1) / V * V;     // halo rounded to whole lanes
    static constexpr int SW = 64 * V;                  // strip width (loaded columns)
    static constexpr int OWMAX = SW - 2 * HV;          // most outputs per strip
    static constexpr int NE = V + 2 * R;               // gathered x-neighbourhood
    static constexpr int K = 2 * R + 1;                // ring length (rows or planes)
    static constexpr int NF = KIND == kGS ? 2 : 1;
};

// Row access of one lane.  FAST strips lie inside the row: the row pointer
// plus the strip start is wave-uniform and the lane adds a constant offset,
// so loads and stores are plain 16-byte vector accesses with no per-row
// vector address arithmetic.  Edge strips wrap each column once, up front.
template <typename T, int V, bool FAST>
struct RowIO;

template <typename T, int V>
struct RowIO<T, V, true> {
    int64_t xb;  // first column of the strip (uniform)
    int lo;      // lane * V
    __device__ __forceinline__ RowIO(int64_t xb_, int lane, int64_t) : xb(xb_), lo(lane * V) {}
    __device__ __forceinline__ void load(const T *__restrict__ row, T (&o)[V]) const
    {
        vload(row + xb + lo, o);
    }
};

template <typename T, int V>
struct RowIO<T, V, false> {
    int64_t col[V];
    __device__ __forceinline__ RowIO(int64_t xb, int lane, int64_t nx)
    {
#pragma unroll
        for (int v = 0; v < V; ++v) col[v] = wrap_any(xb + lane * V + v, nx);
    }
    __device__ __forceinline__ void load(const T *__restrict__ row, T (&o)[V]) const
    {
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = row[col[v]];
    }
};

// Output mask of a lane: which of its V columns are written, and whether all
// are (then one vector store).
template <int V>
struct OutMask {
    bool ov[V];
    bool all;
};

template <typename T, int V>
__device__ __forceinline__ void store_row(T *__restrict__ row, int64_t xl, const OutMask<V> &m,
                                          const T (&o)[V])
{
    if (m.all) {
        vstore(row + xl, o);
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (m.ov[v]) row[xl + v] = o[v];
    }
}

// ===========================================================================
// 2D fused marching step.  One wave owns a strip of SW = 64 V columns (V
// values per lane, x-neighbours by lane shuffles) and marches along y over
// one chunk of output rows.  Each radius-r stencil evaluation is a "stage"
// that consumes a ring of the last K = 2r+1 rows of its input stream (in
// registers) and produces one row of its output stream r rows behind:
//   AC, GS:  state n -> state n+1                       (1 stage per step)
//   CH:      state n -> mu -> state n+1                  (2 stages per step)
// With TB = 2 the stages of two time steps are chained, so one sweep over HBM
// advances the grid two steps; the intermediate state never leaves the
// registers.  Every stage uses the same per-site functions, so TB = 2 is
// bitwise equal to two TB = 1 steps.  Loads run K rows ahead (prefetch ring).

// Neighbour pair sums (x pair + y pair) at element v for j = 1..R around the
// centre row CS of a ring, with the centre row's x-neighbourhood in e.
template <typename T, int V, int R, int K, int CS>
__device__ __forceinline__ void pairs2d(const T (&rg)[K][V], const T (&e)[V + 2 * R], int v,
                                        T (&S)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int sp = (CS + j) % K, sm = (CS - j + K) % K;
        S[j - 1] = (e[R + v + j] + e[R + v - j]) + (rg[sp][v] + rg[sm][v]);
    });
}

template <typename T, int V, int R, int K, int CS>
__device__ __forceinline__ void pairs2d64(const T (&rg)[K][V], const T (&e)[V + 2 * R], int v,
                                          double (&S)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int sp = (CS + j) % K, sm = (CS - j + K) % K;
        S[j - 1] = ((double)e[R + v + j] + (double)e[R + v - j]) +
                   ((double)rg[sp][v] + (double)rg[sm][v]);
    });
}

// AC / GS step of the centre row CS of the state rings rg (NF fields); with
// RED the state at that row is reduced (masked by om and red_row).
template <typename T, int KIND, int R, int K, int CS, bool RED>
__device__ __forceinline__ void stage_acgs(const StepArgs<T> &a,
                                           const T (&rg)[KIND == kGS ? 2 : 1][K][Vec<T>::V],
                                           T (&res)[KIND == kGS ? 2 : 1][Vec<T>::V],
                                           const OutMask<Vec<T>::V> &om, bool red_row,
                                           RedState &red)
{
    constexpr int V = Vec<T>::V, NF = KIND == kGS ? 2 : 1;
    T e[NF][V + 2 * R];
#pragma unroll
    for (int f = 0; f < NF; ++f) gather_x<T, V, R>(rg[f][CS], e[f]);
    double rs0 = 0.0, rs1 = 0.0, rbad = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sf[NF][R];
#pragma unroll
        for (int f = 0; f < NF; ++f) pairs2d<T, V, R, K, CS>(rg[f], e[f], v, Sf[f]);
        const T u0 = rg[0][CS][v];
        if constexpr (KIND == kAC) {
            res[0][v] = ac_update<T, R>(a, u0, Sf[0], u0 * T(4));
        } else {
            const T v0 = rg[NF - 1][CS][v];
            gs_update<T, R>(a, u0, v0, Sf[0], Sf[NF - 1], u0 * T(4), v0 * T(4), res[0][v],
                            res[NF - 1][v]);
        }
        if constexpr (RED) {
            if (red_row && om.ov[v]) {
                const double x = (double)u0;
                rs0 += x;
                rbad += finite_val(x) ? 0.0 : 1.0;
                if constexpr (KIND == kAC) {
                    if constexpr (std::is_same<T, double>::value) {
                        rs1 += energy_density<R>(a.c1, a.c2, a.w64, x, Sf[0], x * 4.0);
                    } else {
                        double S64[R];
                        pairs2d64<T, V, R, K, CS>(rg[0], e[0], v, S64);
                        rs1 += energy_density<R>(a.c1, a.c2, a.w64, x, S64, x * 4.0);
                    }
                } else {
                    const double y = (double)rg[NF - 1][CS][v];
                    rs1 += y;
                    rbad += finite_val(y) ? 0.0 : 1.0;
                }
            }
        }
    }
    if constexpr (RED) {
        if (red_row) {
            acc_add(red.q0, rs0);
            acc_add(red.q1, rs1);
            red.bad += rbad;
        }
    }
}

// CH chemical potential of the centre row CS of the concentration ring c.
template <typename T, int R, int K, int CS, bool RED>
__device__ __forceinline__ void stage_mu(const StepArgs<T> &a, const T (&c)[K][Vec<T>::V],
                                         T (&mu)[Vec<T>::V], const OutMask<Vec<T>::V> &om,
                                         bool red_row, RedState &red)
{
    constexpr int V = Vec<T>::V;
    T e[V + 2 * R];
    gather_x<T, V, R>(c[CS], e);
    double rs0 = 0.0, rs1 = 0.0, rbad = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sc[R];
        pairs2d<T, V, R, K, CS>(c, e, v, Sc);
        const T c0 = c[CS][v];
        mu[v] = ch_mu<T, R>(a, c0, Sc, c0 * T(4));
        if constexpr (RED) {
            if (red_row && om.ov[v]) {
                const double x = (double)c0;
                rs0 += x;
                if constexpr (std::is_same<T, double>::value) {
                    rs1 += energy_from_mu(a.c2, x, mu[v]);
                } else {
                    double S64[R];
                    pairs2d64<T, V, R, K, CS>(c, e, v, S64);
                    rs1 += energy_density<R>(a.c1, a.c2, a.w64, x, S64, x * 4.0);
                }
                rbad += finite_val(x) ? 0.0 : 1.0;
            }
        }
    }
    if constexpr (RED) {
        if (red_row) {
            acc_add(red.q0, rs0);
            acc_add(red.q1, rs1);
            red.bad += rbad;
        }
    }
}

// CH update of the centre row CS: c' = c + dt L mu.
template <typename T, int R, int K, int CS>
__device__ __forceinline__ void stage_chupd(const StepArgs<T> &a, const T (&m)[K][Vec<T>::V],
                                            const T (&c0)[Vec<T>::V], T (&res)[Vec<T>::V])
{
    constexpr int V = Vec<T>::V;
    T em[V + 2 * R];
    gather_x<T, V, R>(m[CS], em);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sm[R];
        pairs2d<T, V, R, K, CS>(m, em, v, Sm);
        res[v] = ch_update<T, R>(a, c0[v], Sm, m[CS][v] * T(4));
    }
}

template <int K, int D>
struct Slot {
    template <int PH>
    static constexpr int at = ((PH - D) % K + 2 * K) % K;
};

template <typename T, int KIND, int R, bool RED, bool FAST, int TB>
__device__ __forceinline__ void march2d(const StepArgs<T> &a, int par, int64_t xb, int64_t y0,
                                        int64_t y1, int lane, int64_t pslot)
{
    using S = Shape<T, KIND, R, TB>;
    constexpr int V = S::V, H = S::H, HV = S::HV, K = S::K, NF = S::NF;
    const int64_t nx = a.nx, ny = a.ny, pitch = a.pitch;
    const int64_t xl = xb + lane * V;
    const int pl = lane * V;
    OutMask<V> om;
    om.all = true;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        om.ov[v] = (pl + v >= HV) && (pl + v < HV + a.ow) && (xl + v < nx);
        om.all = om.all && om.ov[v];
    }
    const RowIO<T, V, FAST> io(xb, lane, nx);
    const T *in[2] = {a.buf[0][par], a.buf[NF - 1][par]};
    T *out[2] = {a.buf[0][par ^ 1], a.buf[NF - 1][par ^ 1]};

    T ring[NF][K][V];                                    // state n (loaded)
    T pre[NF][K][V];                                     // prefetched rows
    T r1[TB == 2 ? NF : 1][K][V];                        // state n+1 (TB = 2)
    T m0[KIND == kCH ? K : 1][V];                        // mu of state n
    T m1[(KIND == kCH && TB == 2) ? K : 1][V];           // mu of state n+1
    RedState red[TB];

    const int64_t tb0 = y0 - H, tend = y1 + H;
    static_for<0, K>([&](auto phc) {
        constexpr int ph = decltype(phc)::value;
        const int64_t t = tb0 + ph;
        if (t < tend) {
            const int64_t off = wrap_any(t, ny) * pitch;
#pragma unroll
            for (int f = 0; f < NF; ++f) io.load(in[f] + off, pre[f][ph]);
        }
    });

    for (int64_t tb = tb0; tb < tend; tb += K) {
        static_for<0, K>([&](auto phc) {
            constexpr int ph = decltype(phc)::value;
            const int64_t t = tb + ph;
            if (t < tend) {
                const int64_t age = t - tb0;  // a stage of depth k is valid once age >= 2 k r
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int v = 0; v < V; ++v) ring[f][ph][v] = pre[f][ph][v];
                if (t + K < tend) {
                    const int64_t off = wrap_any(t + K, ny) * pitch;
#pragma unroll
                    for (int f = 0; f < NF; ++f) io.load(in[f] + off, pre[f][ph]);
                }
                if constexpr (KIND != kCH) {
                    constexpr int s1 = Slot<K, R>::template at<ph>;
                    if (age >= 2 * R) {
                        const int64_t row = t - R;
                        T res[NF][V];
                        stage_acgs<T, KIND, R, K, s1, RED>(a, ring, res, om, row >= y0 && row < y1,
                                                           red[0]);
                        if constexpr (TB == 1) {
                            const int64_t ooff = wrap_any(row, ny) * pitch;
#pragma unroll
                            for (int f = 0; f < NF; ++f) store_row<T, V>(out[f] + ooff, xl, om, res[f]);
                        } else {
#pragma unroll
                            for (int f = 0; f < NF; ++f)
#pragma unroll
                                for (int v = 0; v < V; ++v) r1[f][s1][v] = res[f][v];
                        }
                    }
                    if constexpr (TB == 2) {
                        constexpr int s2 = Slot<K, 2 * R>::template at<ph>;
                        if (age >= 4 * R) {
                            const int64_t row = t - 2 * R;
                            T res[NF][V];
                            stage_acgs<T, KIND, R, K, s2, RED>(a, r1, res, om, row >= y0 && row < y1,
                                                               red[TB - 1]);
                            const int64_t ooff = wrap_any(row, ny) * pitch;
#pragma unroll
                            for (int f = 0; f < NF; ++f) store_row<T, V>(out[f] + ooff, xl, om, res[f]);
                        }
                    }
                } else {
                    constexpr int s1 = Slot<K, R>::template at<ph>;
                    constexpr int s2 = Slot<K, 2 * R>::template at<ph>;
                    if (age >= 2 * R) {
                        const int64_t row = t - R;
                        stage_mu<T, R, K, s1, RED>(a, ring[0], m0[s1], om, row >= y0 && row < y1,
                                                   red[0]);
                    }
                    if (age >= 4 * R) {
                        T res[V];
                        stage_chupd<T, R, K, s2>(a, m0, ring[0][s2], res);
                        if constexpr (TB == 1) {
                            store_row<T, V>(out[0] + wrap_any(t - 2 * R, ny) * pitch, xl, om, res);
                        } else {
#pragma unroll
                            for (int v = 0; v < V; ++v) r1[0][s2][v] = res[v];
                        }
                    }
                    if constexpr (TB == 2) {
                        constexpr int s3 = Slot<K, 3 * R>::template at<ph>;
                        constexpr int s4 = Slot<K, 4 * R>::template at<ph>;
                        if (age >= 6 * R) {
                            const int64_t row = t - 3 * R;
                            stage_mu<T, R, K, s3, RED>(a, r1[0], m1[s3], om, row >= y0 && row < y1,
                                                       red[TB - 1]);
                        }
                        if (age >= 8 * R) {
                            T res[V];
                            stage_chupd<T, R, K, s4>(a, m1, r1[0][s4], res);
                            store_row<T, V>(out[0] + wrap_any(t - 4 * R, ny) * pitch, xl, om, res);
                        }
                    }
                }
            }
        });
    }
    if constexpr (RED) {
        red_flush(red[0], a.part, a.pstride, pslot, lane);
        if constexpr (TB == 2) red_flush(red[TB - 1], a.part, a.pstride, pslot + a.items, lane);
    }
}

template <typename T, int KIND, int R, bool RED, int TB>
__device__ __forceinline__ void step2d_item(const StepArgs<T> &a, int par, int32_t item,
                                            int lane, int64_t pslot)
{
    using S = Shape<T, KIND, R, TB>;
    const int32_t strip = item % a.strips;
    const int32_t chunk = item / a.strips;
    const int64_t xb = (int64_t)strip * a.ow - S::HV;
    const int64_t y0 = (int64_t)chunk * a.clen;
    const int64_t y1 = min(y0 + (int64_t)a.clen, a.ny);
    if (xb >= 0 && xb + S::SW <= a.nx)
        march2d<T, KIND, R, RED, true, TB>(a, par, xb, y0, y1, lane, pslot);
    else
        march2d<T, KIND, R, RED, false, TB>(a, par, xb, y0, y1, lane, pslot);
}

// Single-model 2D launch of TB fused steps: reads buf[parity], writes
// buf[parity ^ 1].
template <typename T, int KIND, int R, bool RED, int TB>
__global__ void __launch_bounds__(64 * kWaves2D) k_step2d(StepArgs<T> a)
{
    const int32_t nwg = gridDim.x;
    const int32_t wg = xcd_item(blockIdx.x, nwg);
    const int32_t item = wg * kWaves2D + (threadIdx.x >> 6);
    if (item >= a.items) return;
    step2d_item<T, KIND, R, RED, TB>(a, a.parity, item, threadIdx.x & 63, item);
}

// Request of global work item g in a batch table (binary search over the
// item prefix sums).
template <typename T>
__device__ __forceinline__ int batch_request(const BatchTable<T> &tb, int32_t n, int32_t g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tb.item_start[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Persistent batched 2D step: a fixed grid strides over the work items of
// every request in the table (step k of the tick; requests with fewer steps
// this tick skip).  Each request is stepped exactly as by k_step2d.
template <typename T, int KIND, int R>
__global__ void __launch_bounds__(64 * kWaves2D) k_step2d_batched(BatchTable<T> tb, int32_t k)
{
    const int32_t n = *tb.count;
    const int32_t total = tb.item_start[n];
    const int32_t stride = gridDim.x * kWaves2D;
    for (int32_t g = blockIdx.x * kWaves2D + (threadIdx.x >> 6); g < total; g += stride) {
        const int i = batch_request(tb, n, g);
        if (k >= tb.steps[i]) continue;
        const StepArgs<T> &a = tb.args[i];
        step2d_item<T, KIND, R, false, 1>(a, (a.parity + k) & 1, g - tb.item_start[i],
                                          threadIdx.x & 63, 0);
    }
}

// ===========================================================================
// 3D fused marching step.  A workgroup of NW = 16 waves owns a tile of 16
// rows (y) of one x-strip and marches along z.  Wave w holds tile row
// y0 - H + w.  As in 2D the step is a chain of radius-r stages (two per CH
// step, one per AC/GS step; TB steps per sweep); each stage keeps a z-window
// of K = 2r+1 planes of its input stream in registers, takes x-neighbours by
// lane shuffles and y-neighbours from the other waves' rows of its centre
// plane in LDS.  Stage k's centre plane was produced r iterations earlier,
// so every stage's LDS row is written before one barrier per plane; a stage
// at depth k is valid for rows [k r, NW - k r) of the tile, and only rows
// [H, NW - H) are written.

template <typename T, int KIND, int R, int TB>
struct Lds3D {
    using S = Shape<T, KIND, R, TB>;
    static constexpr int NST = (KIND == kCH ? 2 : 1) * TB;  // stages
    static constexpr int NFS = KIND == kCH ? 1 : S::NF;      // fields per stage input
    static constexpr int NB = NST * NFS <= 2 ? 2 : 1;        // buffers (double when it fits)
    using type = T[NB][NST][NFS][kWaves3D][S::SW];
};

// Pair sums at element v around centre plane slot CS of a ring, with the
// centre row's x-neighbourhood e and the centre plane's rows in LDS L.
template <typename T, int V, int R, int K, int CS, int SW>
__device__ __forceinline__ void pairs3d(const T (&rg)[K][V], const T (&e)[V + 2 * R],
                                        const T (&L)[kWaves3D][SW], int w, int pl, int v,
                                        T (&S)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int sp = (CS + j) % K, sm = (CS - j + K) % K;
        S[j - 1] = ((e[R + v + j] + e[R + v - j]) + (L[w + j][pl + v] + L[w - j][pl + v])) +
                   (rg[sp][v] + rg[sm][v]);
    });
}

template <typename T, int V, int R, int K, int CS, int SW>
__device__ __forceinline__ void pairs3d64(const T (&rg)[K][V], const T (&e)[V + 2 * R],
                                          const T (&L)[kWaves3D][SW], int w, int pl, int v,
                                          double (&S)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int sp = (CS + j) % K, sm = (CS - j + K) % K;
        S[j - 1] = (((double)e[R + v + j] + (double)e[R + v - j]) +
                    ((double)L[w + j][pl + v] + (double)L[w - j][pl + v])) +
                   ((double)rg[sp][v] + (double)rg[sm][v]);
    });
}

template <typename T, int KIND, int R, int K, int CS, int SW, bool RED>
__device__ __forceinline__ void stage3_acgs(const StepArgs<T> &a,
                                            const T (&rg)[KIND == kGS ? 2 : 1][K][Vec<T>::V],
                                            const T (&L)[KIND == kGS ? 2 : 1][kWaves3D][SW], int w,
                                            T (&res)[KIND == kGS ? 2 : 1][Vec<T>::V],
                                            const OutMask<Vec<T>::V> &om, bool red_row, RedState &red)
{
    constexpr int V = Vec<T>::V, NF = KIND == kGS ? 2 : 1;
    const int pl = (threadIdx.x & 63) * V;
    T e[NF][V + 2 * R];
#pragma unroll
    for (int f = 0; f < NF; ++f) gather_x<T, V, R>(rg[f][CS], e[f]);
    double rs0 = 0.0, rs1 = 0.0, rbad = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sf[NF][R];
#pragma unroll
        for (int f = 0; f < NF; ++f) pairs3d<T, V, R, K, CS, SW>(rg[f], e[f], L[f], w, pl, v, Sf[f]);
        const T u0 = rg[0][CS][v];
        if constexpr (KIND == kAC) {
            res[0][v] = ac_update<T, R>(a, u0, Sf[0], u0 * T(6));
        } else {
            const T v0 = rg[NF - 1][CS][v];
            gs_update<T, R>(a, u0, v0, Sf[0], Sf[NF - 1], u0 * T(6), v0 * T(6), res[0][v],
                            res[NF - 1][v]);
        }
        if constexpr (RED) {
            if (red_row && om.ov[v]) {
                const double x = (double)u0;
                rs0 += x;
                rbad += finite_val(x) ? 0.0 : 1.0;
                if constexpr (KIND == kAC) {
                    if constexpr (std::is_same<T, double>::value) {
                        rs1 += energy_density<R>(a.c1, a.c2, a.w64, x, Sf[0], x * 6.0);
                    } else {
                        double S64[R];
                        pairs3d64<T, V, R, K, CS, SW>(rg[0], e[0], L[0], w, pl, v, S64);
                        rs1 += energy_density<R>(a.c1, a.c2, a.w64, x, S64, x * 6.0);
                    }
                } else {
                    const double y = (double)rg[NF - 1][CS][v];
                    rs1 += y;
                    rbad += finite_val(y) ? 0.0 : 1.0;
                }
            }
        }
    }
    if constexpr (RED) {
        if (red_row) {
            acc_add(red.q0, rs0);
            acc_add(red.q1, rs1);
            red.bad += rbad;
        }
    }
}

template <typename T, int R, int K, int CS, int SW, bool RED>
__device__ __forceinline__ void stage3_mu(const StepArgs<T> &a, const T (&c)[K][Vec<T>::V],
                                          const T (&L)[kWaves3D][SW], int w, T (&mu)[Vec<T>::V],
                                          const OutMask<Vec<T>::V> &om, bool red_row, RedState &red)
{
    constexpr int V = Vec<T>::V;
    const int pl = (threadIdx.x & 63) * V;
    T e[V + 2 * R];
    gather_x<T, V, R>(c[CS], e);
    double rs0 = 0.0, rs1 = 0.0, rbad = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sc[R];
        pairs3d<T, V, R, K, CS, SW>(c, e, L, w, pl, v, Sc);
        const T c0 = c[CS][v];
        mu[v] = ch_mu<T, R>(a, c0, Sc, c0 * T(6));
        if constexpr (RED) {
            if (red_row && om.ov[v]) {
                const double x = (double)c0;
                rs0 += x;
                if constexpr (std::is_same<T, double>::value) {
                    rs1 += energy_from_mu(a.c2, x, mu[v]);
                } else {
                    double S64[R];
                    pairs3d64<T, V, R, K, CS, SW>(c, e, L, w, pl, v, S64);
                    rs1 += energy_density<R>(a.c1, a.c2, a.w64, x, S64, x * 6.0);
                }
                rbad += finite_val(x) ? 0.0 : 1.0;
            }
        }
    }
    if constexpr (RED) {
        if (red_row) {
            acc_add(red.q0, rs0);
            acc_add(red.q1, rs1);
            red.bad += rbad;
        }
    }
}

template <typename T, int R, int K, int CS, int SW>
__device__ __forceinline__ void stage3_chupd(const StepArgs<T> &a, const T (&m)[K][Vec<T>::V],
                                             const T (&L)[kWaves3D][SW], int w,
                                             const T (&c0)[Vec<T>::V], T (&res)[Vec<T>::V])
{
    constexpr int V = Vec<T>::V;
    const int pl = (threadIdx.x & 63) * V;
    T em[V + 2 * R];
    gather_x<T, V, R>(m[CS], em);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sm[R];
        pairs3d<T, V, R, K, CS, SW>(m, em, L, w, pl, v, Sm);
        res[v] = ch_update<T, R>(a, c0[v], Sm, m[CS][v] * T(6));
    }
}

template <typename T, int KIND, int R, bool RED, bool FAST, int TB>
__device__ __forceinline__ void march3d(const StepArgs<T> &a, int par, int64_t xb, int64_t yrow,
                                        bool out_row, int64_t z0, int64_t z1, int64_t pslot,
                                        typename Lds3D<T, KIND, R, TB>::type &lds)
{
    using S = Shape<T, KIND, R, TB>;
    using LD = Lds3D<T, KIND, R, TB>;
    constexpr int V = S::V, H = S::H, HV = S::HV, K = S::K, NF = S::NF, SW = S::SW;
    constexpr int NW = kWaves3D;
    static_assert(2 * H < NW, "halo too wide for the 3D tile");

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t nx = a.nx, ny = a.ny, nz = a.nz, pitch = a.pitch, plane = a.plane;
    const int64_t xl = xb + lane * V;
    const int64_t rowoff = wrap_any(yrow, ny) * pitch;
    const int pl = lane * V;
    OutMask<V> om;
    om.all = true;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        om.ov[v] = out_row && (pl + v >= HV) && (pl + v < HV + a.ow) && (xl + v < nx);
        om.all = om.all && om.ov[v];
    }
    const RowIO<T, V, FAST> io(xb, lane, nx);
    const T *in[2] = {a.buf[0][par], a.buf[NF - 1][par]};
    T *out[2] = {a.buf[0][par ^ 1], a.buf[NF - 1][par ^ 1]};

    T ring[NF][K][V];
    T pre[NF][K][V];
    T r1[TB == 2 ? NF : 1][K][V];
    T m0[KIND == kCH ? K : 1][V];
    T m1[(KIND == kCH && TB == 2) ? K : 1][V];
    // rings that feed LDS rows before first being computed hold zeros
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if constexpr (KIND == kCH) {
                m0[i][v] = T(0);
                if constexpr (TB == 2) m1[i][v] = T(0);
            }
            if constexpr (TB == 2)
#pragma unroll
                for (int f = 0; f < NF; ++f) r1[f][i][v] = T(0);
        }
    RedState red[TB];
    // a stage at depth k computes rows [k r, NW - k r) of the tile
    auto rows_ok = [&](int k) { return w >= k * R && w < NW - k * R; };

    const int64_t tb0 = z0 - H, tend = z1 + H;
    static_for<0, K>([&](auto phc) {
        constexpr int ph = decltype(phc)::value;
        const int64_t t = tb0 + ph;
        if (t < tend) {
            const int64_t off = wrap_any(t, nz) * plane + rowoff;
#pragma unroll
            for (int f = 0; f < NF; ++f) io.load(in[f] + off, pre[f][ph]);
        }
    });

    for (int64_t tb = tb0; tb < tend; tb += K) {
        static_for<0, K>([&](auto phc) {
            constexpr int ph = decltype(phc)::value;
            const int64_t t = tb + ph;
            if (t < tend) {
                const int64_t age = t - tb0;
                const int buf = LD::NB == 2 ? (int)(t & 1) : 0;
                auto &L = lds[buf];
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int v = 0; v < V; ++v) ring[f][ph][v] = pre[f][ph][v];
                if (t + K < tend) {
                    const int64_t off = wrap_any(t + K, nz) * plane + rowoff;
#pragma unroll
                    for (int f = 0; f < NF; ++f) io.load(in[f] + off, pre[f][ph]);
                }
                constexpr int s1 = Slot<K, R>::template at<ph>;
                constexpr int s2 = Slot<K, 2 * R>::template at<ph>;
                constexpr int s3 = Slot<K, 3 * R>::template at<ph>;
                constexpr int s4 = Slot<K, 4 * R>::template at<ph>;
                if constexpr (LD::NB == 1) __syncthreads();  // previous plane's readers are done
                // centre rows of every stage's input stream
                if constexpr (KIND != kCH) {
#pragma unroll
                    for (int f = 0; f < NF; ++f)
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            L[0][f][w][pl + v] = ring[f][s1][v];
                            if constexpr (TB == 2) L[TB - 1][f][w][pl + v] = r1[f][s2][v];
                        }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        L[0][0][w][pl + v] = ring[0][s1][v];
                        L[1][0][w][pl + v] = m0[s2][v];
                        if constexpr (TB == 2) {
                            L[TB][0][w][pl + v] = r1[0][s3][v];
                            L[TB + 1][0][w][pl + v] = m1[s4][v];
                        }
                    }
                }
                __syncthreads();
                if constexpr (KIND != kCH) {
                    if (age >= 2 * R && rows_ok(1)) {
                        const int64_t pz = t - R;
                        T res[NF][V];
                        stage3_acgs<T, KIND, R, K, s1, SW, RED>(a, ring, L[0], w, res, om,
                                                                pz >= z0 && pz < z1, red[0]);
                        if constexpr (TB == 1) {
                            if (out_row) {
                                const int64_t ooff = wrap_any(pz, nz) * plane + rowoff;
#pragma unroll
                                for (int f = 0; f < NF; ++f)
                                    store_row<T, V>(out[f] + ooff, xl, om, res[f]);
                            }
                        } else {
#pragma unroll
                            for (int f = 0; f < NF; ++f)
#pragma unroll
                                for (int v = 0; v < V; ++v) r1[f][s1][v] = res[f][v];
                        }
                    }
                    if constexpr (TB == 2) {
                        if (age >= 4 * R && rows_ok(2)) {
                            const int64_t pz = t - 2 * R;
                            T res[NF][V];
                            stage3_acgs<T, KIND, R, K, s2, SW, RED>(a, r1, L[TB - 1], w, res, om,
                                                                    pz >= z0 && pz < z1, red[TB - 1]);
                            if (out_row) {
                                const int64_t ooff = wrap_any(pz, nz) * plane + rowoff;
#pragma unroll
                                for (int f = 0; f < NF; ++f)
                                    store_row<T, V>(out[f] + ooff, xl, om, res[f]);
                            }
                        }
                    }
                } else {
                    if (age >= 2 * R && rows_ok(1)) {
                        const int64_t pz = t - R;
                        stage3_mu<T, R, K, s1, SW, RED>(a, ring[0], L[0][0], w, m0[s1], om,
                                                        pz >= z0 && pz < z1, red[0]);
                    }
                    if (age >= 4 * R && rows_ok(2)) {
                        T res[V];
                        stage3_chupd<T, R, K, s2, SW>(a, m0, L[1][0], w, ring[0][s2], res);
                        if constexpr (TB == 1) {
                            if (out_row)
                                store_row<T, V>(out[0] + wrap_any(t - 2 * R, nz) * plane + rowoff, xl,
                                                om, res);
                        } else {
#pragma unroll
                            for (int v = 0; v < V; ++v) r1[0][s2][v] = res[v];
                        }
                    }
                    if constexpr (TB == 2) {
                        if (age >= 6 * R && rows_ok(3)) {
                            const int64_t pz = t - 3 * R;
                            stage3_mu<T, R, K, s3, SW, RED>(a, r1[0], L[TB][0], w, m1[s3], om,
                                                            pz >= z0 && pz < z1, red[TB - 1]);
                        }
                        if (age >= 8 * R && rows_ok(4)) {
                            T res[V];
                            stage3_chupd<T, R, K, s4, SW>(a, m1, L[TB + 1][0], w, r1[0][s4], res);
                            if (out_row)
                                store_row<T, V>(out[0] + wrap_any(t - 4 * R, nz) * plane + rowoff,
                                                xl, om, res);
                        }
                    }
                }
            }
        });
    }
    if constexpr (RED) {
        red_flush(red[0], a.part, a.pstride, pslot, lane);
        if constexpr (TB == 2)
            red_flush(red[TB - 1], a.part, a.pstride, pslot + (int64_t)a.items * kWaves3D, lane);
    }
}

template <typename T, int KIND, int R, bool RED, int TB>
__device__ __forceinline__ void step3d_item(const StepArgs<T> &a, int par, int32_t item,
                                            int64_t pslot_base)
{
    using S = Shape<T, KIND, R, TB>;
    constexpr int NW = kWaves3D;
    const int w = threadIdx.x >> 6;
    const int32_t strip = item % a.strips;
    const int32_t rest = item / a.strips;
    const int32_t ytile = rest % a.ytiles;
    const int32_t chunk = rest / a.ytiles;
    const int64_t xb = (int64_t)strip * a.ow - S::HV;
    const int64_t yrow = (int64_t)ytile * (NW - 2 * S::H) - S::H + w;
    const bool out_row = (w >= S::H) && (w < NW - S::H) && (yrow < a.ny);
    const int64_t z0 = (int64_t)chunk * a.clen;
    const int64_t z1 = min(z0 + (int64_t)a.clen, a.nz);
    __shared__ typename Lds3D<T, KIND, R, TB>::type lds;
    // the FAST choice is uniform over the workgroup (it depends on the strip only)
    if (xb >= 0 && xb + S::SW <= a.nx)
        march3d<T, KIND, R, RED, true, TB>(a, par, xb, yrow, out_row, z0, z1, pslot_base + w, lds);
    else
        march3d<T, KIND, R, RED, false, TB>(a, par, xb, yrow, out_row, z0, z1, pslot_base + w, lds);
}

template <typename T, int KIND, int R, bool RED, int TB>
__global__ void __launch_bounds__(64 * kWaves3D) k_step3d(StepArgs<T> a)
{
    const int32_t item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= a.items) return;  // uniform over the workgroup
    step3d_item<T, KIND, R, RED, TB>(a, a.parity, item, (int64_t)item * kWaves3D);
}

// Persistent batched 3D step (see k_step2d_batched); the item loop is uniform
// over the workgroup, so every wave reaches the same barriers.
template <typename T, int KIND, int R>
__global__ void __launch_bounds__(64 * kWaves3D) k_step3d_batched(BatchTable<T> tb, int32_t k)
{
    const int32_t n = *tb.count;
    const int32_t total = tb.item_start[n];
    for (int32_t g = blockIdx.x; g < total; g += gridDim.x) {
        const int i = batch_request(tb, n, g);
        if (k >= tb.steps[i]) continue;
        const StepArgs<T> &a = tb.args[i];
        step3d_item<T, KIND, R, false, 1>(a, (a.parity + k) & 1, g - tb.item_start[i], 0);
    }
}

}  // namespace pf
