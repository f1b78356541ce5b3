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
__device__ __forceinline__ int32_t wrap32(int32_t i, int32_t n)
{
    if (i >= 0 && i < n) return i;
    int32_t m = i % n;
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
    uint32_t bad = 0;  // non-finite sites this lane reduced
};

__device__ __forceinline__ void red_flush(const RedState &r, double2 *part, int64_t pstride,
                                          int64_t slot, int lane)
{
    const Acc a = wave_reduce(r.q0);
    const Acc b = wave_reduce(r.q1);
    const double c = wave_sum_exact((double)r.bad);
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

// Cahn-Hilliard (Eq. model-b) chemical potential mu = c2 c^3 - c1 c - L c =
// c (c2 c^2 - c1) - L c: k0 = c1, k1 = c2, wi = w_j/dx^2.
template <typename T, int R>
__device__ __forceinline__ T ch_mu(const StepArgs<T> &a, T c0, const T (&S)[R], T ctr)
{
    T lc = T(0);
#pragma unroll
    for (int j = 0; j < R; ++j) lc = fma(a.wi[j], S[j] - ctr, lc);
    return fma(c0, fma(a.k1 * c0, c0, -a.k0), -lc);
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

// Cahn-Hilliard with the direct biharmonic stencil: c' = c + dt (L g - B c),
// g = c2 c^3 - c1 c, B = sum_a D4_a + 2 sum_{a<b} D2_a D2_b.  Split by axis,
// L g - B c = sum_a D2_a mu_a - sum_a D4_a c with mu_a = g - sum_{b != a} D2_b c,
// the chemical potential without the a-axis term; mu_a is ch_mu over the
// pairs of the other axes.  chd_g: g alone (k0 = c1, k1 = c2).
template <typename T>
__device__ __forceinline__ T chd_g(const StepArgs<T> &a, T c0)
{
    return c0 * fma(a.k1 * c0, c0, -a.k0);
}
// Update from Sm (pairs of mu_a along axis a, summed over axes; ctrm = the
// matching centre terms 2 sum_a mu_a) and S4 (fourth-derivative pairs of c,
// ctr4 = 2 ndim c): wu = dt w_j/dx^2, w4 = -dt w4_j/dx^4, j = 1..R+1.
template <typename T, int R>
__device__ __forceinline__ T chd_update(const StepArgs<T> &a, T c0, const T (&Sm)[R], T ctrm,
                                        const T (&S4)[R + 1], T ctr4)
{
    T acc = c0;
#pragma unroll
    for (int j = 0; j < R; ++j) acc = fma(a.wu[j], Sm[j] - ctrm, acc);
#pragma unroll
    for (int j = 0; j <= R; ++j) acc = fma(a.w4[j], S4[j] - ctr4, acc);
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

// Model C (Eq. model-c): k0 = dt c1, k1 = dt c2, k2 = 2 dt, k3 = c3, wu = wv =
// dt w_j/dx^2.  The rho equation diffuses g = rho + c3 phi^2 (mc_g); Sp are
// the neighbour sums of phi, Sg those of g, ctrp / ctrg the centre terms.
template <typename T>
__device__ __forceinline__ T mc_g(const StepArgs<T> &a, T p, T r)
{
    return fma(a.k3, p * p, r);
}
template <typename T, int R>
__device__ __forceinline__ void mc_update(const StepArgs<T> &a, T p0, T r0, const T (&Sp)[R],
                                          const T (&Sg)[R], T ctrp, T ctrg, T &pn, T &rn)
{
    const T g = fma(-(a.k1 * p0), p0, a.k0) - a.k2 * r0;  // dt (c1 - c2 phi^2 - 2 rho)
    T acc = fma(g, p0, p0);
    T accr = r0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        acc = fma(a.wu[j], Sp[j] - ctrp, acc);
        accr = fma(a.wv[j], Sg[j] - ctrg, accr);
    }
    pn = acc;
    rn = accr;
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

// The same energy summed by parts, for FP32 storage (the state widened to
// FP64): over the periodic grid, -(1/2) sum_i x_i (L x)_i equals
// sum_i x_i sum_j w_j sum_axes (x_i - x_{i + j e_axis}) = sum_i x_i (wd x_i -
// sum_j w_j P_j), where P[j-1] is the sum over the axes of the forward
// neighbours at distance j and wd = ndim sum_j w_j; so each site takes only
// its forward neighbours, and a multiply-add per distance.  With the local
// terms the density is x^2 ((c2/4) x^2 + wd - c1/2) - x sum_j w_j P_j.  The
// per-site values differ from energy_density, the sum over the grid (every
// reduction reports only sums) is the same up to rounding.
template <int R>
__device__ __forceinline__ double energy_by_parts(double c1, double c2, const double *w64, double wd,
                                                  double x, const double (&P)[R])
{
    double s = w64[0] * P[0];
#pragma unroll
    for (int j = 1; j < R; ++j) s = fma(w64[j], P[j], s);
    const double x2 = x * x;
    return fma(x2, fma(0.25 * c2, x2, wd - 0.5 * c1), -(x * s));
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
// i - 1; lanes without a source receive 0 (bound control: they are halo
// lanes), so the move needs no initialised destination.
__device__ __forceinline__ int dpp_from_next(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_from_prev(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);
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
    // halo of TB fused steps: CH composes two radius-r stages, the direct
    // biharmonic reaches r + 1
    static constexpr int H = (KIND == kCH ? 2 * R : KIND == kCHD ? R + 1 : R) * TB;
    static constexpr int HV = (H + V - 1) / V * V;     // halo rounded to whole lanes
    static constexpr int SW = 64 * V;                  // strip width (loaded columns)
    static constexpr int OWMAX = SW - 2 * HV;          // most outputs per strip
    static constexpr int NE = V + 2 * R;               // gathered x-neighbourhood
    static constexpr int K = KIND == kCHD ? 2 * R + 3 : 2 * R + 1;  // ring length (rows or planes)
    static constexpr int NF = nfields_kind(KIND);
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

// ---------------------------------------------------------------------------
// Row end of a lane's reductions: s0, s1 are the row's masked sums (mass and
// energy density, or the two fields' sums when TWO); value(f, v) returns the
// reduced value of field f at element v.  Non-finite values are counted only
// when a row sum is not finite, which is exact: a NaN or infinity among the
// addends always makes the sum non-finite, and a sum of finite values that
// overflows is recounted to zero.
template <int V, bool TWO, typename F>
__device__ __forceinline__ void red_row_end(RedState &red, const OutMask<V> &om, double s0,
                                            double s1, F &&value)
{
    if (!(finite_val(s0) && finite_val(s1))) {
        uint32_t bad = 0;
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (om.ov[v]) {
                bad += finite_val(value(0, v)) ? 0u : 1u;
                if constexpr (TWO) bad += finite_val(value(1, v)) ? 0u : 1u;
            }
        red.bad += bad;
    }
    acc_add(red.q0, s0);
    acc_add(red.q1, s1);
}

// ---------------------------------------------------------------------------
// Ring slot holding the row (plane) D iterations behind phase PH of a K-long
// ring that is written at slot PH on phase PH.
template <int K, int D>
struct Slot {
    template <int PH>
    static constexpr int at = ((PH - D) % K + 2 * K) % K;
};

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

}  // namespace pf
