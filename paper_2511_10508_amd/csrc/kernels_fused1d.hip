// 1D fused step kernels of libpfmi (gfx950, wave64).
//
// A 1D grid is one periodic row of nx sites.  It is cut into strips of
// OW <= 64 V - 2 HV outputs; a strip loads SW = 64 V sites (V per lane,
// 16-byte vectors) starting HV sites before its first output, so the HV
// halo lanes on either side carry the neighbours that the stages need (every
// stage takes its x-neighbours by DPP lane shifts).  One wave owns a segment
// of consecutive strips and walks it with PD strips of loads in flight.  Each
// strip is read once from HBM; the halo columns that neighbouring strips
// share come from L2.  Every stage uses the per-site functions of the 2D and
// 3D kernels with the centre term 2 u0 of one axis; Model H (m, j) runs here
// fused as well.
#include "pf_device.h"
#include "pf_dispatch.h"

namespace pf {

using Fused1DRadii = RList<1, 2, 3, 4>;

namespace {

constexpr int kWaves1D = 4;  // waves per workgroup
constexpr int kPrefetch1D = 2;  // strips of loads in flight per wave

// Strip geometry of the 1D kernels: the common Shape, except Model H, which
// steps two fields (m, j) with two radius-r stages per step (mu, then the
// coupled update), like Cahn-Hilliard.
template <typename T, int KIND, int R, int TB>
struct Shape1D {
    using S = Shape<T, KIND, R, TB>;
    static constexpr int V = S::V, SW = S::SW;
    static constexpr int NF = KIND == kMH ? 2 : S::NF;
    static constexpr int H = KIND == kMH ? 2 * R * TB : S::H;
    static constexpr int HV = (H + V - 1) / V * V;
    static constexpr int OWMAX = SW - 2 * HV;
};

// Neighbour pair sums S[j-1] = e[v+j] + e[v-j] of a gathered neighbourhood
// e of radius RE (>= R) at element v.
template <typename T, int R, int RE, int NE>
__device__ __forceinline__ void pairs1d(const T (&e)[NE], int v, T (&S)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        S[j - 1] = e[RE + v + j] + e[RE + v - j];
    });
}

// Forward neighbours x_{+j} in FP64 (energy by parts, FP32 storage).
template <typename T, int R, int RE, int NE>
__device__ __forceinline__ void fwd1d64(const T (&e)[NE], int v, double (&P)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        P[j - 1] = (double)e[RE + v + j];
    });
}

// One time step of a strip held in registers: in -> out (NF fields, V
// values per lane).  With RED the state `in` is reduced over the lanes'
// output elements (om).
template <typename T, int KIND, int R, bool RED>
__device__ __forceinline__ void stage1d(const StepArgs<T> &a,
                                        const T (&in)[Shape1D<T, KIND, R, 1>::NF][Vec<T>::V],
                                        T (&out)[Shape1D<T, KIND, R, 1>::NF][Vec<T>::V],
                                        const OutMask<Vec<T>::V> &om, RedState &red)
{
    constexpr int V = Vec<T>::V, NF = Shape1D<T, KIND, R, 1>::NF;
    constexpr bool F64 = std::is_same<T, double>::value;
    double s0 = 0.0, s1 = 0.0;  // the strip's masked reduction sums
    if constexpr (KIND == kAC || KIND == kGS) {
        T e[NF][V + 2 * R];
#pragma unroll
        for (int f = 0; f < NF; ++f) gather_x<T, V, R>(in[f], e[f]);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T S[NF][R];
#pragma unroll
            for (int f = 0; f < NF; ++f) pairs1d<T, R, R>(e[f], v, S[f]);
            const T u0 = in[0][v];
            if constexpr (KIND == kAC) {
                out[0][v] = ac_update<T, R>(a, u0, S[0], u0 * T(2));
            } else {
                const T v0 = in[1][v];
                gs_update<T, R>(a, u0, v0, S[0], S[1], u0 * T(2), v0 * T(2), out[0][v], out[1][v]);
            }
            if constexpr (RED) {
                if (om.ov[v]) {
                    const double x = (double)u0;
                    s0 += x;
                    if constexpr (KIND == kGS) {
                        s1 += (double)in[1][v];
                    } else if constexpr (F64) {
                        double S64[R];
#pragma unroll
                        for (int j = 0; j < R; ++j) S64[j] = S[0][j];
                        s1 += energy_density<R>(a.c1, a.c2, a.w64, x, S64, 2.0 * x);
                    } else {
                        double Pn[R];
                        fwd1d64<T, R, R>(e[0], v, Pn);
                        s1 += energy_by_parts<R>(a.c1, a.c2, a.w64, a.w64sum, x, Pn);
                    }
                }
            }
        }
    } else if constexpr (KIND == kMC) {
        T g[V], ep[V + 2 * R], eg[V + 2 * R];
#pragma unroll
        for (int v = 0; v < V; ++v) g[v] = mc_g(a, in[0][v], in[1][v]);
        gather_x<T, V, R>(in[0], ep);
        gather_x<T, V, R>(g, eg);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T Sp[R], Sg[R];
            pairs1d<T, R, R>(ep, v, Sp);
            pairs1d<T, R, R>(eg, v, Sg);
            const T p0 = in[0][v];
            mc_update<T, R>(a, p0, in[1][v], Sp, Sg, p0 * T(2), g[v] * T(2), out[0][v], out[1][v]);
            if constexpr (RED) {
                if (om.ov[v]) {
                    s0 += (double)p0;
                    s1 += (double)in[1][v];
                }
            }
        }
    } else if constexpr (KIND == kCH) {
        T e[V + 2 * R], mu[V], em[V + 2 * R];
        gather_x<T, V, R>(in[0], e);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T S[R];
            pairs1d<T, R, R>(e, v, S);
            mu[v] = ch_mu<T, R>(a, in[0][v], S, in[0][v] * T(2));
        }
        gather_x<T, V, R>(mu, em);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T Sm[R];
            pairs1d<T, R, R>(em, v, Sm);
            const T c0 = in[0][v];
            out[0][v] = ch_update<T, R>(a, c0, Sm, mu[v] * T(2));
            if constexpr (RED) {
                if (om.ov[v]) {
                    const double x = (double)c0;
                    s0 += x;
                    if constexpr (F64) {
                        s1 += energy_from_mu(a.c2, x, mu[v]);
                    } else {
                        double Pn[R];
                        fwd1d64<T, R, R>(e, v, Pn);
                        s1 += energy_by_parts<R>(a.c1, a.c2, a.w64, a.w64sum, x, Pn);
                    }
                }
            }
        }
    } else if constexpr (KIND == kMH) {
        // Model H in 1D (fields m, j): mu as Cahn-Hilliard; m' = m + dt L mu
        // - dt c3 D1(m j), j' = j + dt L j + dt c3 m D1 mu (k2 = dt c3, w1 =
        // w1_k/dx), each sum in the per-site kernel's order
        T e[V + 2 * R], mu[V], em[V + 2 * R], mj[V], ep[V + 2 * R], ej[V + 2 * R];
        gather_x<T, V, R>(in[0], e);
        gather_x<T, V, R>(in[1], ej);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T S[R];
            pairs1d<T, R, R>(e, v, S);
            mu[v] = ch_mu<T, R>(a, in[0][v], S, in[0][v] * T(2));
            mj[v] = in[0][v] * in[1][v];
        }
        gather_x<T, V, R>(mu, em);
        gather_x<T, V, R>(mj, ep);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T Sm[R], Sj[R];
            pairs1d<T, R, R>(em, v, Sm);
            pairs1d<T, R, R>(ej, v, Sj);
            T div = T(0), grad = T(0);
            static_for<1, R + 1>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                div = fma(a.w1[k - 1], ep[R + v + k] - ep[R + v - k], div);
            });
            static_for<1, R + 1>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                grad = fma(a.w1[k - 1], em[R + v + k] - em[R + v - k], grad);
            });
            const T m0 = in[0][v], j0 = in[1][v];
            out[0][v] = fma(-a.k2, div, ch_update<T, R>(a, m0, Sm, mu[v] * T(2)));
            out[1][v] = fma(a.k2 * m0, grad, ch_update<T, R>(a, j0, Sj, j0 * T(2)));
            if constexpr (RED)
                if (om.ov[v]) s0 += (double)m0;
        }
    } else {  // kCHD: in 1D mu_x = g, so c' = c + dt (D2 g - D4 c)
        constexpr int R4 = R + 1;
        T g[V], eg[V + 2 * R], ec[V + 2 * R4];
#pragma unroll
        for (int v = 0; v < V; ++v) g[v] = chd_g(a, in[0][v]);
        gather_x<T, V, R>(g, eg);
        gather_x<T, V, R4>(in[0], ec);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T Sg[R], S4[R4];
            pairs1d<T, R, R>(eg, v, Sg);
            pairs1d<T, R4, R4>(ec, v, S4);
            const T c0 = in[0][v];
            out[0][v] = chd_update<T, R>(a, c0, Sg, g[v] * T(2), S4, c0 * T(2));
            if constexpr (RED) {
                if (om.ov[v]) {
                    const double x = (double)c0;
                    s0 += x;
                    if constexpr (F64) {
                        double S64[R];
                        static_for<1, R + 1>([&](auto jc) {
                            constexpr int j = decltype(jc)::value;
                            S64[j - 1] = ec[R4 + v + j] + ec[R4 + v - j];
                        });
                        s1 += energy_density<R>(a.c1, a.c2, a.w64, x, S64, 2.0 * x);
                    } else {
                        double Pn[R];
                        fwd1d64<T, R, R4>(ec, v, Pn);
                        s1 += energy_by_parts<R>(a.c1, a.c2, a.w64, a.w64sum, x, Pn);
                    }
                }
            }
        }
    }
    // Model H reduces m only (mass, non-finite count)
    constexpr bool TWO = NF == 2 && KIND != kMH;
    if constexpr (RED)
        red_row_end<V, TWO>(red, om, s0, s1, [&](int f, int v) { return (double)in[f][v]; });
}

// Strip loads of one lane.  FAST: every strip of the segment lies inside
// [0, nx), one 16-byte vector per field; otherwise each element wraps.
template <typename T, int NF, int V, bool FAST>
__device__ __forceinline__ void load_strip(const T *const (&in)[2], int64_t x0, int pl, int64_t nx,
                                           T (&o)[NF][V])
{
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if constexpr (FAST) {
            vload(in[f] + x0 + pl, o[f]);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) o[f][v] = in[f][wrap_any(x0 + pl + v, nx)];
        }
    }
}

// March of one wave over strips [s0, s1) of the row, TB fused steps.
template <typename T, int KIND, int R, bool RED, int TB, bool FAST>
__device__ __forceinline__ void march1d(const StepArgs<T> &a, int32_t s0, int32_t s1, int lane,
                                        int64_t pslot)
{
    using S = Shape1D<T, KIND, R, TB>;
    constexpr int V = S::V, HV = S::HV, NF = S::NF, PD = kPrefetch1D;
    const int64_t nx = a.nx, ow = a.ow;
    const int pl = lane * V;
    const int par = a.parity;
    const T *const in[2] = {a.buf[0][par], a.buf[NF - 1][par]};
    T *const out[2] = {a.buf[0][par ^ 1], a.buf[NF - 1][par ^ 1]};
    RedState red[TB];
    T pre[PD][NF][V];
    // strips past the segment are clamped to its last strip: loaded, not used
    auto x0_of = [&](int32_t s) { return (int64_t)min(s, s1 - 1) * ow - HV; };
    static_for<0, PD>([&](auto phc) {
        constexpr int ph = decltype(phc)::value;
        load_strip<T, NF, V, FAST>(in, x0_of(s0 + ph), pl, nx, pre[ph]);
    });
    auto strip = [&](auto phc, int32_t s) {
        constexpr int ph = decltype(phc)::value;
        T cur[NF][V];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int v = 0; v < V; ++v) cur[f][v] = pre[ph][f][v];
        load_strip<T, NF, V, FAST>(in, x0_of(s + PD), pl, nx, pre[ph]);
        const int64_t x0 = (int64_t)s * ow - HV;
        OutMask<V> om;
        om.all = true;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            om.ov[v] = (pl + v >= HV) && (pl + v < HV + ow) && (x0 + pl + v < nx);
            om.all = om.all && om.ov[v];
        }
        T res[NF][V];
        stage1d<T, KIND, R, RED>(a, cur, res, om, red[0]);
        if constexpr (TB == 2) {
            T res2[NF][V];
            stage1d<T, KIND, R, RED>(a, res, res2, om, red[TB - 1]);
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int v = 0; v < V; ++v) res[f][v] = res2[f][v];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) store_row<T, V>(out[f], x0 + pl, om, res[f]);
    };
    int32_t sb = s0;
    for (; sb + PD <= s1; sb += PD)
        static_for<0, PD>([&](auto phc) { strip(phc, sb + decltype(phc)::value); });
    static_for<0, PD>([&](auto phc) {
        if (sb + decltype(phc)::value < s1) strip(phc, sb + decltype(phc)::value);
    });
    if constexpr (RED) {
        red_flush(red[0], a.part, a.pstride, pslot, lane);
        if constexpr (TB == 2) red_flush(red[TB - 1], a.part, a.pstride, pslot + a.items, lane);
    }
}

// Single-model 1D launch of TB fused steps: wave `item` owns strips
// [item clen, min((item + 1) clen, strips)).
template <typename T, int KIND, int R, bool RED, int TB>
__global__ void __launch_bounds__(64 * kWaves1D) k_step1d(StepArgs<T> a)
{
    using S = Shape1D<T, KIND, R, TB>;
    const int32_t nwg = gridDim.x;
    const int32_t wg = xcd_item(blockIdx.x, nwg);
    const int32_t item = __builtin_amdgcn_readfirstlane(wg * kWaves1D + (int)(threadIdx.x >> 6));
    if (item >= a.items) return;
    const int32_t s0 = item * a.clen;
    const int32_t s1 = min(s0 + a.clen, a.strips);
    const int lane = threadIdx.x & 63;
    const bool fast = (int64_t)s0 * a.ow - S::HV >= 0 &&
                      (int64_t)(s1 - 1) * a.ow - S::HV + S::SW <= a.nx;
    if (fast)
        march1d<T, KIND, R, RED, TB, true>(a, s0, s1, lane, item);
    else
        march1d<T, KIND, R, RED, TB, false>(a, s0, s1, lane, item);
}

}  // namespace

bool plan_fused1d(const Launch &L, int64_t nx, int32_t clen, int tb, int32_t *strips, int32_t *ow,
                  int32_t *chunks, int32_t *items, int32_t *blocks, int32_t *threads)
{
    bool ok = false;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        dispatch_kind_generic(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            ok = dispatch_r(L.r, Fused1DRadii{}, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                const int owmax = tb == 2 ? Shape1D<T, KIND, R, 2>::OWMAX : Shape1D<T, KIND, R, 1>::OWMAX;
                constexpr int V = Shape1D<T, KIND, R, 1>::V;
                const int64_t st = cdiv(nx, owmax);
                *strips = (int32_t)st;
                *ow = (int32_t)(cdiv(cdiv(nx, st), V) * V);
                *chunks = (int32_t)cdiv(st, clen);
                *items = *chunks;
                *blocks = (int32_t)cdiv(*items, kWaves1D);
                *threads = 64 * kWaves1D;
            });
        });
    });
    return ok;
}

hipError_t launch_fused1d(const Launch &L, const void *args, int32_t blocks, int32_t threads,
                          int red, int tb, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        dispatch_kind_generic(L.kind, [&](auto kc) {
            constexpr int KIND = decltype(kc)::value;
            dispatch_r(L.r, Fused1DRadii{}, [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                if (tb == 2) {
                    if (red)
                        hipLaunchKernelGGL((k_step1d<T, KIND, R, true, 2>), dim3(blocks), dim3(threads), 0, s, a);
                    else
                        hipLaunchKernelGGL((k_step1d<T, KIND, R, false, 2>), dim3(blocks), dim3(threads), 0, s, a);
                } else {
                    if (red)
                        hipLaunchKernelGGL((k_step1d<T, KIND, R, true, 1>), dim3(blocks), dim3(threads), 0, s, a);
                    else
                        hipLaunchKernelGGL((k_step1d<T, KIND, R, false, 1>), dim3(blocks), dim3(threads), 0, s, a);
                }
                err = hipGetLastError();
            });
        });
    });
    return err;
}

}  // namespace pf
