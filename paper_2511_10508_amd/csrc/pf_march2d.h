// 2D fused marching kernels of libpfmi (gfx950, wave64): see the section
// comment below for the work decomposition.
#pragma once

#include "pf_device.h"

namespace pf {

// ===========================================================================
// 2D fused marching step.  One wave owns a strip of SW = 64 V columns (V
// values per lane, x-neighbours by DPP lane shifts) and marches along y over
// one chunk of output rows.  Each radius-r stencil evaluation is a "stage"
// that consumes a ring of the last K = 2r+1 rows of its input stream (in
// registers) and produces one row of its output stream r rows behind:
//   AC, GS:  state n -> state n+1                       (1 stage per step)
//   CH:      state n -> mu -> state n+1                  (2 stages per step)
// With TB = 2 the stages of two time steps are chained, so one sweep over HBM
// advances the grid two steps; the intermediate state never leaves the
// registers.  Every stage uses the same per-site functions, so TB = 2 is
// bitwise equal to two TB = 1 steps.  Loads run PD rows ahead (a prefetch
// ring; PD = K except where the registers are short).

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

// Forward-neighbour sums over the axes at distances 1..R of element v, in
// FP64 from the widened values (x forward along +x, y along the ring).
template <typename T, int V, int R, int K, int CS>
__device__ __forceinline__ void fwd2d64(const T (&rg)[K][V], const T (&e)[V + 2 * R], int v,
                                        double (&P)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int sp = (CS + j) % K;
        P[j - 1] = (double)e[R + v + j] + (double)rg[sp][v];
    });
}

// Neighbour pair sums of g = rho + c3 phi^2 (Model C) at element v: the
// x-neighbours come gathered in eg, the y-neighbours' g from the rings.
template <typename T, int V, int R, int K, int CS>
__device__ __forceinline__ void pairs2d_g(const StepArgs<T> &a, const T (&rp)[K][V],
                                          const T (&rr)[K][V], const T (&eg)[V + 2 * R], int v,
                                          T (&S)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int sp = (CS + j) % K, sm = (CS - j + K) % K;
        S[j - 1] = (eg[R + v + j] + eg[R + v - j]) +
                   (mc_g(a, rp[sp][v], rr[sp][v]) + mc_g(a, rp[sm][v], rr[sm][v]));
    });
}

// AC / GS / Model C step of the centre row CS of the state rings rg (NF
// fields); with RED the state at that row is reduced (masked by om and
// red_row).
template <typename T, int KIND, int R, int K, int CS, bool RED>
__device__ __forceinline__ void stage_acgs(const StepArgs<T> &a,
                                           const T (&rg)[nfields_kind(KIND)][K][Vec<T>::V],
                                           T (&res)[nfields_kind(KIND)][Vec<T>::V],
                                           const OutMask<Vec<T>::V> &om, bool red_row,
                                           RedState &red)
{
    constexpr int V = Vec<T>::V, NF = nfields_kind(KIND);
    T e[NF][V + 2 * R];
    T gc[V];  // Model C: g of the centre row
    gather_x<T, V, R>(rg[0][CS], e[0]);
    if constexpr (KIND == kMC) {
#pragma unroll
        for (int v = 0; v < V; ++v) gc[v] = mc_g(a, rg[0][CS][v], rg[1][CS][v]);
        gather_x<T, V, R>(gc, e[1]);
    } else if constexpr (NF == 2) {
        gather_x<T, V, R>(rg[1][CS], e[1]);
    }
    double s0 = 0.0, s1 = 0.0;  // the row's masked reduction sums
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sf[NF][R];
        pairs2d<T, V, R, K, CS>(rg[0], e[0], v, Sf[0]);
        if constexpr (KIND == kMC)
            pairs2d_g<T, V, R, K, CS>(a, rg[0], rg[1], e[1], v, Sf[1]);
        else if constexpr (NF == 2)
            pairs2d<T, V, R, K, CS>(rg[1], e[1], v, Sf[1]);
        const T u0 = rg[0][CS][v];
        if constexpr (KIND == kAC) {
            res[0][v] = ac_update<T, R>(a, u0, Sf[0], u0 * T(4));
        } else if constexpr (KIND == kMC) {
            mc_update<T, R>(a, u0, rg[1][CS][v], Sf[0], Sf[1], u0 * T(4), gc[v] * T(4), res[0][v],
                            res[1][v]);
        } else {
            const T v0 = rg[NF - 1][CS][v];
            gs_update<T, R>(a, u0, v0, Sf[0], Sf[NF - 1], u0 * T(4), v0 * T(4), res[0][v],
                            res[NF - 1][v]);
        }
        if constexpr (RED) {
            if (om.ov[v]) {
                const double x = (double)u0;
                s0 += x;
                if constexpr (KIND == kAC) {
                    if constexpr (std::is_same<T, double>::value) {
                        s1 += energy_density<R>(a.c1, a.c2, a.w64, x, Sf[0], x * 4.0);
                    } else {
                        double Pn[R];
                        fwd2d64<T, V, R, K, CS>(rg[0], e[0], v, Pn);
                        s1 += energy_by_parts<R>(a.c1, a.c2, a.w64, 2.0 * a.w64sum, x, Pn);
                    }
                } else {
                    s1 += (double)rg[NF - 1][CS][v];
                }
            }
        }
    }
    if constexpr (RED)
        if (red_row)
            red_row_end<V, NF == 2>(red, om, s0, s1, [&](int f, int v) {
                return (double)rg[f == 0 ? 0 : NF - 1][CS][v];
            });
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
    double s0 = 0.0, s1 = 0.0;  // the row's masked reduction sums
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sc[R];
        pairs2d<T, V, R, K, CS>(c, e, v, Sc);
        const T c0 = c[CS][v];
        mu[v] = ch_mu<T, R>(a, c0, Sc, c0 * T(4));
        if constexpr (RED) {
            if (om.ov[v]) {
                const double x = (double)c0;
                s0 += x;
                if constexpr (std::is_same<T, double>::value) {
                    s1 += energy_from_mu(a.c2, x, mu[v]);
                } else {
                    double Pn[R];
                    fwd2d64<T, V, R, K, CS>(c, e, v, Pn);
                    s1 += energy_by_parts<R>(a.c1, a.c2, a.w64, 2.0 * a.w64sum, x, Pn);
                }
            }
        }
    }
    if constexpr (RED)
        if (red_row)
            red_row_end<V, false>(red, om, s0, s1, [&](int, int v) { return (double)c[CS][v]; });
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

// Direct-biharmonic Cahn-Hilliard, first half: on its arrival, row PH of the
// concentration ring c gets mu_y = g - D2_x c (the chemical potential without
// the y term) into the ring my.
template <typename T, int R, int K, int PH>
__device__ __forceinline__ void chd_row_mu_y(const StepArgs<T> &a, const T (&c)[K][Vec<T>::V],
                                             T (&my)[K][Vec<T>::V])
{
    constexpr int V = Vec<T>::V;
    T e[V + 2 * R];
    gather_x<T, V, R>(c[PH], e);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T S[R];
#pragma unroll
        for (int j = 1; j <= R; ++j) S[j - 1] = e[R + v + j] + e[R + v - j];
        const T c0 = c[PH][v];
        my[PH][v] = ch_mu<T, R>(a, c0, S, c0 * T(2));
    }
}

// Direct-biharmonic Cahn-Hilliard, second half: the update of the centre row
// CS of the K = 2R+3 ring (R+1 rows behind the newest) from mu_x = g - D2_y c
// of that row (x-pairs), the mu_y ring (y-pairs) and the fourth-derivative
// pairs of c along x and y.  With RED the state at that row is reduced.
template <typename T, int R, int K, int CS, bool RED>
__device__ __forceinline__ void stage_chd(const StepArgs<T> &a, const T (&c)[K][Vec<T>::V],
                                          const T (&my)[K][Vec<T>::V], T (&res)[Vec<T>::V],
                                          const OutMask<Vec<T>::V> &om, bool red_row,
                                          RedState &red)
{
    constexpr int V = Vec<T>::V, R4 = R + 1;
    T mx[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T S[R];
        static_for<1, R + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            S[j - 1] = c[(CS + j) % K][v] + c[(CS - j + K) % K][v];
        });
        mx[v] = ch_mu<T, R>(a, c[CS][v], S, c[CS][v] * T(2));
    }
    T em[V + 2 * R], ec[V + 2 * R4];
    gather_x<T, V, R>(mx, em);
    gather_x<T, V, R4>(c[CS], ec);
    double s0 = 0.0, s1 = 0.0;  // the row's masked reduction sums
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sm[R], S4[R4];
        static_for<1, R + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            Sm[j - 1] = (em[R + v + j] + em[R + v - j]) + (my[(CS + j) % K][v] + my[(CS - j + K) % K][v]);
        });
        static_for<1, R4 + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            S4[j - 1] = (ec[R4 + v + j] + ec[R4 + v - j]) + (c[(CS + j) % K][v] + c[(CS - j + K) % K][v]);
        });
        const T c0 = c[CS][v];
        res[v] = chd_update<T, R>(a, c0, Sm, (mx[v] + my[CS][v]) * T(2), S4, c0 * T(4));
        if constexpr (RED) {
            if (om.ov[v]) {
                const double x = (double)c0;
                s0 += x;
                if constexpr (std::is_same<T, double>::value) {
                    // the full chemical potential: mu_x + mu_y - g
                    s1 += energy_from_mu(a.c2, x, (mx[v] + my[CS][v]) - chd_g(a, c0));
                } else {
                    double Pn[R];
                    static_for<1, R + 1>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        Pn[j - 1] = (double)ec[R4 + v + j] + (double)c[(CS + j) % K][v];
                    });
                    s1 += energy_by_parts<R>(a.c1, a.c2, a.w64, 2.0 * a.w64sum, x, Pn);
                }
            }
        }
    }
    if constexpr (RED)
        if (red_row)
            red_row_end<V, false>(red, om, s0, s1, [&](int, int v) { return (double)c[CS][v]; });
}

// Prefetch depth PD of the input rows: the loads for row t + PD are issued
// while row t is processed (PD divides the ring length K).  K rows ahead,
// except for the FP64 two-step Cahn-Hilliard kernel with fused reductions,
// where one row ahead frees the registers for a third wave per SIMD and
// measures faster.
template <typename T, int KIND, int R, int TB, bool RED>
constexpr int prefetch_depth2d()
{
    return (std::is_same<T, double>::value && KIND == kCH && TB == 2 && RED) ? 1
                                                                            : Shape<T, KIND, R, TB>::K;
}

template <typename T, int KIND, int R, bool RED, bool FAST, int TB>
__device__ __forceinline__ void march2d(const StepArgs<T> &a, int par, int64_t xb, int32_t y0,
                                        int32_t y1, int lane, int64_t pslot)
{
    using S = Shape<T, KIND, R, TB>;
    constexpr int V = S::V, H = S::H, HV = S::HV, K = S::K, NF = S::NF;
    const int64_t nx = a.nx, pitch = a.pitch;
    const int32_t ny = (int32_t)a.ny;  // rows are 32-bit: scalar compares and modulo
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
    constexpr int PD = prefetch_depth2d<T, KIND, R, TB, RED>();
    static_assert(K % PD == 0, "row t is prefetched into slot t mod PD of a K-phase loop");
    T pre[NF][PD][V];                                    // rows t+1 .. t+PD
    T r1[TB == 2 ? NF : 1][K][V];                        // state n+1 (TB = 2)
    T m0[KIND == kCH ? K : 1][V];                        // mu of state n
    T m1[(KIND == kCH && TB == 2) ? K : 1][V];           // mu of state n+1
    T my[KIND == kCHD ? K : 1][V];                       // direct biharmonic: mu_y rows
    RedState red[TB];

    const int32_t tb0 = y0 - H, tend = y1 + H;
    // The first PD rows are loaded unconditionally (a row past the march is a
    // valid wrapped row, read and not used), so that every load of the
    // unguarded main loop below has a fixed number of loads issued after it
    // and the compiler can wait for it alone instead of draining all of them.
    static_for<0, PD>([&](auto phc) {
        constexpr int ph = decltype(phc)::value;
        const int64_t off = (int64_t)wrap32(tb0 + ph, ny) * pitch;
#pragma unroll
        for (int f = 0; f < NF; ++f) io.load(in[f] + off, pre[f][ph]);
    });

    // One row t of the march at ring phase ph; G guards the rows and the
    // prefetch against the end of the march (the tail only).
    auto phase = [&](auto phc, auto gc, int32_t tb) {
        constexpr int ph = decltype(phc)::value;
        constexpr bool G = decltype(gc)::value;
        const int32_t t = tb + ph;
        if (!G || t < tend) {
            const int32_t age = t - tb0;  // a stage of depth k is valid once age >= 2 k r
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int v = 0; v < V; ++v) ring[f][ph][v] = pre[f][ph % PD][v];
            if (!G || t + PD < tend) {
                const int64_t off = (int64_t)wrap32(t + PD, ny) * pitch;
#pragma unroll
                for (int f = 0; f < NF; ++f) io.load(in[f] + off, pre[f][ph % PD]);
            }
            if constexpr (KIND == kCHD) {
                chd_row_mu_y<T, R, K, ph>(a, ring[0], my);
                constexpr int s1 = Slot<K, R + 1>::template at<ph>;
                if (age >= 2 * (R + 1)) {
                    const int32_t row = t - (R + 1);
                    T res[V];
                    stage_chd<T, R, K, s1, RED>(a, ring[0], my, res, om, row >= y0 && row < y1,
                                                red[0]);
                    store_row<T, V>(out[0] + (int64_t)wrap32(row, ny) * pitch, xl, om, res);
                }
            } else if constexpr (KIND != kCH) {
                constexpr int s1 = Slot<K, R>::template at<ph>;
                if (age >= 2 * R) {
                    const int32_t row = t - R;
                    T res[NF][V];
                    stage_acgs<T, KIND, R, K, s1, RED>(a, ring, res, om, row >= y0 && row < y1,
                                                       red[0]);
                    if constexpr (TB == 1) {
                        const int64_t ooff = (int64_t)wrap32(row, ny) * pitch;
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
                        const int32_t row = t - 2 * R;
                        T res[NF][V];
                        stage_acgs<T, KIND, R, K, s2, RED>(a, r1, res, om, row >= y0 && row < y1,
                                                           red[TB - 1]);
                        const int64_t ooff = (int64_t)wrap32(row, ny) * pitch;
#pragma unroll
                        for (int f = 0; f < NF; ++f) store_row<T, V>(out[f] + ooff, xl, om, res[f]);
                    }
                }
            } else {
                constexpr int s1 = Slot<K, R>::template at<ph>;
                constexpr int s2 = Slot<K, 2 * R>::template at<ph>;
                if (age >= 2 * R) {
                    const int32_t row = t - R;
                    stage_mu<T, R, K, s1, RED>(a, ring[0], m0[s1], om, row >= y0 && row < y1,
                                               red[0]);
                }
                if (age >= 4 * R) {
                    T res[V];
                    stage_chupd<T, R, K, s2>(a, m0, ring[0][s2], res);
                    if constexpr (TB == 1) {
                        store_row<T, V>(out[0] + (int64_t)wrap32(t - 2 * R, ny) * pitch, xl, om, res);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) r1[0][s2][v] = res[v];
                    }
                }
                if constexpr (TB == 2) {
                    constexpr int s3 = Slot<K, 3 * R>::template at<ph>;
                    constexpr int s4 = Slot<K, 4 * R>::template at<ph>;
                    if (age >= 6 * R) {
                        const int32_t row = t - 3 * R;
                        stage_mu<T, R, K, s3, RED>(a, r1[0], m1[s3], om, row >= y0 && row < y1,
                                                   red[TB - 1]);
                    }
                    if (age >= 8 * R) {
                        T res[V];
                        stage_chupd<T, R, K, s4>(a, m1, r1[0][s4], res);
                        store_row<T, V>(out[0] + (int64_t)wrap32(t - 4 * R, ny) * pitch, xl, om, res);
                    }
                }
            }
        }
    };
    int32_t tb = tb0;
    for (; tb + K + PD <= tend; tb += K)
        static_for<0, K>([&](auto phc) { phase(phc, std::false_type{}, tb); });
    for (; tb < tend; tb += K)
        static_for<0, K>([&](auto phc) { phase(phc, std::true_type{}, tb); });
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
    const int32_t y0 = chunk * a.clen;
    const int32_t y1 = min(y0 + a.clen, (int32_t)a.ny);
    if (xb >= 0 && xb + S::SW <= a.nx)
        march2d<T, KIND, R, RED, true, TB>(a, par, xb, y0, y1, lane, pslot);
    else
        march2d<T, KIND, R, RED, false, TB>(a, par, xb, y0, y1, lane, pslot);
}

// Single-model 2D launch of TB fused steps: reads buf[parity], writes
// buf[parity ^ 1].
// Waves per SIMD the register allocation must allow (1: no constraint).  The
// FP64 two-step Cahn-Hilliard kernel with reductions lands a few registers
// above 128; held to 128 (four waves per SIMD instead of three) it spills one
// register pair and runs 6 % faster.  The same hint measured slower on the
// two-step Gray-Scott kernels, so it is not applied generally.
template <typename T, int KIND, int R, bool RED, int TB>
constexpr int min_waves2d()
{
    return (std::is_same<T, double>::value && KIND == kCH && R == 2 && RED && TB == 2) ? 4 : 1;
}

template <typename T, int KIND, int R, bool RED, int TB>
__global__ void __launch_bounds__(64 * kWaves2D)
    __attribute__((amdgpu_waves_per_eu(min_waves2d<T, KIND, R, RED, TB>())))
    k_step2d(StepArgs<T> a)
{
    const int32_t nwg = gridDim.x;
    const int32_t wg = xcd_item(blockIdx.x, nwg);
    // a wave's item is uniform over its lanes: say so, so that the strip and
    // row arithmetic of the march runs on the scalar unit
    const int32_t item = __builtin_amdgcn_readfirstlane(wg * kWaves2D + (int)(threadIdx.x >> 6));
    if (item >= a.items) return;
    step2d_item<T, KIND, R, RED, TB>(a, a.parity, item, threadIdx.x & 63, item);
}

// Persistent batched 2D step: a fixed grid strides over the work items of
// every request in the table (step k of the tick; requests with fewer steps
// this tick skip).  Each request is stepped exactly as by k_step2d.  With
// TB = 2, k is even and a request with two or more steps left in the tick
// takes a two-step sweep, one with a single step left a single step; both
// read buffer parity + k / 2 and write the other.
template <typename T, int KIND, int R, int TB>
__global__ void __launch_bounds__(64 * kWaves2D) k_step2d_batched(BatchTable<T> tb, int32_t k)
{
    const int32_t n = *tb.count;
    const int32_t total = tb.item_start[n];
    const int32_t stride = gridDim.x * kWaves2D;
    for (int32_t g = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves2D + (int)(threadIdx.x >> 6));
         g < total; g += stride) {
        const int i = batch_request(tb, n, g);
        const int32_t left = tb.steps[i] - k;  // uniform over the wave
        if (left <= 0) continue;
        const StepArgs<T> &a = tb.args[i];
        const int par = (a.parity + k / TB) & 1;
        if constexpr (TB == 2) {
            if (left >= 2) {
                step2d_item<T, KIND, R, false, 2>(a, par, g - tb.item_start[i], threadIdx.x & 63, 0);
                continue;
            }
        }
        step2d_item<T, KIND, R, false, 1>(a, par, g - tb.item_start[i], threadIdx.x & 63, 0);
    }
}

}  // namespace pf
