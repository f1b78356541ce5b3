// 3D fused marching kernels of libpfmi (gfx950, wave64): see the section
// comment below for the work decomposition.
#pragma once

#include "pf_device.h"

namespace pf {

// ===========================================================================
// 3D fused marching step.  A workgroup of 16 waves owns a tile of NR rows
// (y) of one x-strip and marches along z.  Each wave holds RPW tile rows:
// with RPW = 1 the wave's 64 lanes hold row w (RW = 64 V columns); with
// RPW = 2 lanes 0-31 hold row 2w and lanes 32-63 row 2w+1 (RW = 32 V
// columns, 512 contiguous bytes each).  Two rows per wave double the tile
// height for the same registers per lane, which halves the share of the tile
// lost to the y-halo (2H of NR rows) at the price of a wider share lost to
// the x-halo (2HV of RW columns); the layout is chosen per kernel.  With
// RPW = 4 rows of 16 lanes make the same 32-row tile with 8 waves, so two
// workgroups share a CU and one's barrier wait is covered by the other's
// work, for a still wider x-halo share (Cahn-Hilliard with r = 3: a 48-row
// tile of 12 waves, see Tile3D).
// As in 2D the step is a chain of radius-r stages (two per CH step, one per
// AC/GS step; TB steps per sweep); each stage keeps a z-window of K = 2r+1
// planes of its input stream in registers, takes x-neighbours by lane
// shifts and y-neighbours from the other rows of its centre plane in LDS.
// With two or four rows per wave a shift across a row boundary brings the
// other row's edge value into a halo column, on which no valid output
// depends.  Stage k's centre plane was produced r iterations earlier, so
// every stage's LDS row is written before one barrier per plane; a stage at
// depth k is valid for rows [k r, NR - k r) of the tile, and only rows
// [H, NR - H) are written.

template <typename T, int KIND, int R, int TB, int RPW_ = 2>
struct Tile3D {
    using S = Shape<T, KIND, R, TB>;
    static constexpr int V = S::V, H = S::H, HV = S::HV;
    static constexpr int RPW = RPW_;                         // rows per wave (1, 2 or 4)
    static constexpr int LPR = 64 / RPW;                     // lanes per row
    // waves per workgroup: 16; with four rows per wave 8 (the same 32-row
    // tile in half the lanes, so that two workgroups share a CU at up to 128
    // registers a lane), or 12 for Cahn-Hilliard with r = 3 and the direct
    // biharmonic with r = 1, whose kernels need 129-168 registers: one
    // workgroup per CU either way, and twelve waves make three per SIMD and a
    // 48-row tile (CH r = 3: 36 rows written of 48 instead of 20 of 32).  The
    // direct biharmonic with r >= 2 needs up to 256 registers and stays at 8.
    static constexpr int NW = RPW == 4 ? (((KIND == kCH && R == 3) || (KIND == kCHD && R == 1)) ? 12 : 8)
                                       : kWaves3D;
    static constexpr int NR = RPW * NW;                      // tile rows
    static constexpr int RW = LPR * V;                       // loaded columns per row
    static constexpr int OWMAX = RW - 2 * HV;                // most outputs per row
    // LDS planes: the centre plane of every stage's input stream
    // (the direct biharmonic: c at the arriving plane, c and mu_y at the
    // centre plane)
    static constexpr int NST = (KIND == kCH ? 2 : KIND == kCHD ? 3 : 1) * TB;
    // fields per plane (the passes of a two-pass CH step stage one stream)
    static constexpr int NFS = (KIND == kCH || KIND == kCHMU || KIND == kCHUP) ? 1 : S::NF;
    static constexpr int NB = (NST * NFS <= 2 || KIND == kCHD) ? 2 : 1;  // LDS buffers (double when it fits)
    using lds_type = T[NB][NST][NFS][NR][RW];
    static_assert(RPW == 1 || RPW == 2 || RPW == 4, "one, two or four rows per wave");
    static_assert(2 * H < NR && OWMAX > 0, "halo too wide for the 3D tile");
};

// Tile row of this lane: the wave index with one row per wave (uniform over
// the wave, which lets its row arithmetic run on the scalar unit), else
// RPW rows per wave of LPR lanes each.
template <int RPW, int LPR>
__device__ __forceinline__ int tile_row()
{
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if constexpr (RPW == 1)
        return w;
    else
        return RPW * w + (int)(threadIdx.x & 63) / LPR;
}

// Pair sums at element v around centre plane slot CS of a ring, with the
// centre row's x-neighbourhood e and the centre plane's rows in LDS L (this
// lane's row rw, first column pl).
template <typename T, int V, int R, int K, int CS, int NR, int RW>
__device__ __forceinline__ void pairs3d(const T (&rg)[K][V], const T (&e)[V + 2 * R],
                                        const T (&L)[NR][RW], int rw, int pl, int v, T (&S)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int sp = (CS + j) % K, sm = (CS - j + K) % K;
        S[j - 1] = ((e[R + v + j] + e[R + v - j]) + (L[rw + j][pl + v] + L[rw - j][pl + v])) +
                   (rg[sp][v] + rg[sm][v]);
    });
}

// Forward-neighbour sums over the axes at distances 1..R of element v, in
// FP64 from the widened values (+x from e, +y from the LDS rows, +z along
// the ring).
template <typename T, int V, int R, int K, int CS, int NR, int RW>
__device__ __forceinline__ void fwd3d64(const T (&rg)[K][V], const T (&e)[V + 2 * R],
                                        const T (&L)[NR][RW], int rw, int pl, int v,
                                        double (&P)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int sp = (CS + j) % K;
        P[j - 1] = ((double)e[R + v + j] + (double)L[rw + j][pl + v]) + (double)rg[sp][v];
    });
}

// Neighbour pair sums of g = rho + c3 phi^2 (Model C) at element v: x from
// the gathered eg, y from the centre plane's g rows in LDS, z from the rings.
template <typename T, int V, int R, int K, int CS, int NR, int RW>
__device__ __forceinline__ void pairs3d_g(const StepArgs<T> &a, const T (&rp)[K][V],
                                          const T (&rr)[K][V], const T (&eg)[V + 2 * R],
                                          const T (&Lg)[NR][RW], int rw, int pl, int v, T (&S)[R])
{
    static_for<1, R + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int sp = (CS + j) % K, sm = (CS - j + K) % K;
        S[j - 1] = ((eg[R + v + j] + eg[R + v - j]) + (Lg[rw + j][pl + v] + Lg[rw - j][pl + v])) +
                   (mc_g(a, rp[sp][v], rr[sp][v]) + mc_g(a, rp[sm][v], rr[sm][v]));
    });
}

// AC / GS / Model C step of the centre plane CS of the rings rg; the centre
// plane's rows of every field (Model C: phi and g) are in L.
template <typename T, int KIND, int R, int K, int CS, int NR, int RW, bool RED>
__device__ __forceinline__ void stage3_acgs(const StepArgs<T> &a,
                                            const T (&rg)[nfields_kind(KIND)][K][Vec<T>::V],
                                            const T (&L)[nfields_kind(KIND)][NR][RW], int rw,
                                            int pl, T (&res)[nfields_kind(KIND)][Vec<T>::V],
                                            const OutMask<Vec<T>::V> &om, bool red_row, RedState &red)
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
        pairs3d<T, V, R, K, CS, NR, RW>(rg[0], e[0], L[0], rw, pl, v, Sf[0]);
        if constexpr (KIND == kMC)
            pairs3d_g<T, V, R, K, CS, NR, RW>(a, rg[0], rg[1], e[1], L[1], rw, pl, v, Sf[1]);
        else if constexpr (NF == 2)
            pairs3d<T, V, R, K, CS, NR, RW>(rg[1], e[1], L[1], rw, pl, v, Sf[1]);
        const T u0 = rg[0][CS][v];
        if constexpr (KIND == kAC) {
            res[0][v] = ac_update<T, R>(a, u0, Sf[0], u0 * T(6));
        } else if constexpr (KIND == kMC) {
            mc_update<T, R>(a, u0, rg[1][CS][v], Sf[0], Sf[1], u0 * T(6), gc[v] * T(6), res[0][v],
                            res[1][v]);
        } else {
            const T v0 = rg[NF - 1][CS][v];
            gs_update<T, R>(a, u0, v0, Sf[0], Sf[NF - 1], u0 * T(6), v0 * T(6), res[0][v],
                            res[NF - 1][v]);
        }
        if constexpr (RED) {
            if (om.ov[v]) {
                const double x = (double)u0;
                s0 += x;
                if constexpr (KIND == kAC) {
                    if constexpr (std::is_same<T, double>::value) {
                        s1 += energy_density<R>(a.c1, a.c2, a.w64, x, Sf[0], x * 6.0);
                    } else {
                        double Pn[R];
                        fwd3d64<T, V, R, K, CS, NR, RW>(rg[0], e[0], L[0], rw, pl, v, Pn);
                        s1 += energy_by_parts<R>(a.c1, a.c2, a.w64, 3.0 * a.w64sum, x, Pn);
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

template <typename T, int R, int K, int CS, int NR, int RW, bool RED>
__device__ __forceinline__ void stage3_mu(const StepArgs<T> &a, const T (&c)[K][Vec<T>::V],
                                          const T (&L)[NR][RW], int rw, int pl, T (&mu)[Vec<T>::V],
                                          const OutMask<Vec<T>::V> &om, bool red_row, RedState &red)
{
    constexpr int V = Vec<T>::V;
    T e[V + 2 * R];
    gather_x<T, V, R>(c[CS], e);
    double s0 = 0.0, s1 = 0.0;  // the row's masked reduction sums
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sc[R];
        pairs3d<T, V, R, K, CS, NR, RW>(c, e, L, rw, pl, v, Sc);
        const T c0 = c[CS][v];
        mu[v] = ch_mu<T, R>(a, c0, Sc, c0 * T(6));
        if constexpr (RED) {
            if (om.ov[v]) {
                const double x = (double)c0;
                s0 += x;
                if constexpr (std::is_same<T, double>::value) {
                    s1 += energy_from_mu(a.c2, x, mu[v]);
                } else {
                    double Pn[R];
                    fwd3d64<T, V, R, K, CS, NR, RW>(c, e, L, rw, pl, v, Pn);
                    s1 += energy_by_parts<R>(a.c1, a.c2, a.w64, 3.0 * a.w64sum, x, Pn);
                }
            }
        }
    }
    if constexpr (RED)
        if (red_row)
            red_row_end<V, false>(red, om, s0, s1, [&](int, int v) { return (double)c[CS][v]; });
}

template <typename T, int R, int K, int CS, int NR, int RW>
__device__ __forceinline__ void stage3_chupd(const StepArgs<T> &a, const T (&m)[K][Vec<T>::V],
                                             const T (&L)[NR][RW], int rw, int pl,
                                             const T (&c0)[Vec<T>::V], T (&res)[Vec<T>::V])
{
    constexpr int V = Vec<T>::V;
    T em[V + 2 * R];
    gather_x<T, V, R>(m[CS], em);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T Sm[R];
        pairs3d<T, V, R, K, CS, NR, RW>(m, em, L, rw, pl, v, Sm);
        res[v] = ch_update<T, R>(a, c0[v], Sm, m[CS][v] * T(6));
    }
}

// Direct-biharmonic Cahn-Hilliard in 3D: c' = c + dt (sum_a D2_a mu_a -
// sum_a D4_a c), mu_a = g - sum_{b != a} D2_b c (the chemical potential
// without the a-axis term).  The ring holds K = 2r + 3 planes of c; the
// update runs on the centre plane CS, r + 1 planes behind the newest, so the
// halo is r + 1 instead of the composed form's 2r.  Every sum is formed in
// the per-site kernel's order (pairs x, then y, then z), so the fields are
// bitwise those of the per-site kernels.
//
// mu_y of the centre plane from its x-neighbourhood (lane shifts) and the
// z-ring (no y term: computed before the plane's barrier).
template <typename T, int R, int K, int CS>
__device__ __forceinline__ void stage3_chd_mu_y(const StepArgs<T> &a, const T (&c)[K][Vec<T>::V],
                                                T (&my)[Vec<T>::V])
{
    constexpr int V = Vec<T>::V;
    T e[V + 2 * R];
    gather_x<T, V, R>(c[CS], e);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T S[R];
        static_for<1, R + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            S[j - 1] = (e[R + v + j] + e[R + v - j]) + (c[(CS + j) % K][v] + c[(CS - j + K) % K][v]);
        });
        const T c0 = c[CS][v];
        my[v] = ch_mu<T, R>(a, c0, S, c0 * T(4));
    }
}

// mu_z of the arriving plane SA (x by lane shifts, y from its plane in LDS)
// into slot SA of the mu_z ring.
template <typename T, int R, int K, int SA, int NR, int RW>
__device__ __forceinline__ void stage3_chd_mu_z(const StepArgs<T> &a, const T (&c)[K][Vec<T>::V],
                                                const T (&L)[NR][RW], int rw, int pl,
                                                T (&mz)[K][Vec<T>::V])
{
    constexpr int V = Vec<T>::V;
    T e[V + 2 * R];
    gather_x<T, V, R>(c[SA], e);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T S[R];
        static_for<1, R + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            S[j - 1] = (e[R + v + j] + e[R + v - j]) + (L[rw + j][pl + v] + L[rw - j][pl + v]);
        });
        const T c0 = c[SA][v];
        mz[SA][v] = ch_mu<T, R>(a, c0, S, c0 * T(4));
    }
}

// The update of the centre plane CS: mu_x (y-pairs from the centre plane of
// c in LDS Lc, z-pairs from the ring), then the D2 pairs of mu_x (x, lane
// shifts), mu_y (y, its plane in LDS Lm) and mu_z (z, its ring) and the D4
// pairs of c (lane shifts, Lc, ring); with RED the state at CS is reduced.
template <typename T, int R, int K, int CS, int NR, int RW, bool RED>
__device__ __forceinline__ void stage3_chd_update(const StepArgs<T> &a, const T (&c)[K][Vec<T>::V],
                                                  const T (&my)[Vec<T>::V], const T (&mz)[K][Vec<T>::V],
                                                  const T (&Lc)[NR][RW], const T (&Lm)[NR][RW], int rw,
                                                  int pl, T (&res)[Vec<T>::V], const OutMask<Vec<T>::V> &om,
                                                  bool red_row, RedState &red)
{
    constexpr int V = Vec<T>::V, R4 = R + 1;
    T mx[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T S[R];
        static_for<1, R + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            S[j - 1] = (Lc[rw + j][pl + v] + Lc[rw - j][pl + v]) + (c[(CS + j) % K][v] + c[(CS - j + K) % K][v]);
        });
        const T c0 = c[CS][v];
        mx[v] = ch_mu<T, R>(a, c0, S, c0 * T(4));
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
            Sm[j - 1] = ((em[R + v + j] + em[R + v - j]) + (Lm[rw + j][pl + v] + Lm[rw - j][pl + v])) +
                        (mz[(CS + j) % K][v] + mz[(CS - j + K) % K][v]);
        });
        static_for<1, R4 + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            S4[j - 1] = ((ec[R4 + v + j] + ec[R4 + v - j]) + (Lc[rw + j][pl + v] + Lc[rw - j][pl + v])) +
                        (c[(CS + j) % K][v] + c[(CS - j + K) % K][v]);
        });
        const T c0 = c[CS][v];
        const T musum = (mx[v] + my[v]) + mz[CS][v];
        res[v] = chd_update<T, R>(a, c0, Sm, musum * T(2), S4, c0 * T(6));
        if constexpr (RED) {
            if (om.ov[v]) {
                const double x = (double)c0;
                s0 += x;
                if constexpr (std::is_same<T, double>::value) {
                    // the full chemical potential: (mu_x + mu_y + mu_z - g) / 2
                    s1 += energy_from_mu(a.c2, x, 0.5 * (musum - chd_g(a, c0)));
                } else {
                    double Pn[R];
                    static_for<1, R + 1>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        Pn[j - 1] = ((double)ec[R4 + v + j] + (double)Lc[rw + j][pl + v]) +
                                    (double)c[(CS + j) % K][v];
                    });
                    s1 += energy_by_parts<R>(a.c1, a.c2, a.w64, 3.0 * a.w64sum, x, Pn);
                }
            }
        }
    }
    if constexpr (RED)
        if (red_row)
            red_row_end<V, false>(red, om, s0, s1, [&](int, int v) { return (double)c[CS][v]; });
}

// Prefetch depth of the two passes of a two-pass Cahn-Hilliard step: each
// holds one ring of K planes (the mu pass) or one ring plus c's centre planes
// (the update pass), which leaves room for K planes in flight up to r = 2;
// at r = 3 the update pass (two fields in flight) and the FP32 mu pass with
// reductions (the FP64 energy) prefetch one plane.
template <typename T, int KIND, int R, bool RED>
constexpr int kTwoPassPD =
    (R == 3 && (KIND == kCHUP || (RED && std::is_same<T, float>::value))) ? 1 : 2 * R + 1;

// Prefetch depth PD of the input planes: K planes ahead, or one plane where
// the K-deep prefetch ring would not fit the 128 registers a lane of a
// 16-wave workgroup can hold (wider stencils, and two-step sweeps with fused
// reductions), where a plane's work is also long enough to hide one plane's
// load latency.  FP64 Cahn-Hilliard with r = 2 has room for the K = 5 ring
// (about 120 registers with reductions).
template <typename T, int KIND, int R, int TB, bool RED, int RPW>
constexpr int prefetch_depth()
{
    if (std::is_same<T, double>::value && KIND == kCH && R == 2 && TB == 1) return 2 * R + 1;
    if (KIND == kCH && R == 3 && TB == 1 && RPW == 4) return 2;
    // FP64 two-step Cahn-Hilliard with r = 1 on four rows: K planes fit at
    // 118 registers, two 8-wave workgroups per CU (1-2 % faster than one)
    if (std::is_same<T, double>::value && KIND == kCH && R == 1 && TB == 2 && RPW == 4) return 2 * R + 1;
    if (KIND == kCHD) return 1;
    if (KIND == kCHMU || KIND == kCHUP) return kTwoPassPD<T, KIND, R, RED>;
    return (R >= 2 || (TB == 2 && RED)) ? 1 : 2 * R + 1;
}

template <typename T, int KIND, int R, bool RED, bool FAST, int TB, int RPW>
__device__ __forceinline__ void march3d(const StepArgs<T> &a, int par, int64_t xb, int64_t yrow,
                                        bool out_row, int32_t z0, int32_t z1, int64_t pslot,
                                        typename Tile3D<T, KIND, R, TB, RPW>::lds_type &lds)
{
    using S = Shape<T, KIND, R, TB>;
    using TL = Tile3D<T, KIND, R, TB, RPW>;
    constexpr int V = S::V, H = S::H, HV = S::HV, K = S::K, NF = S::NF;
    constexpr int NR = TL::NR, RW = TL::RW;

    const int lane = threadIdx.x & 63;
    const int lx = lane % TL::LPR;                           // lane within the row segment
    const int rw = tile_row<TL::RPW, TL::LPR>();             // tile row
    const int64_t nx = a.nx, ny = a.ny, pitch = a.pitch, plane = a.plane;
    const int32_t nz = (int32_t)a.nz;  // planes are 32-bit: scalar compares and modulo
    const int64_t xl = xb + lx * V;
    const int64_t rowoff = wrap_any(yrow, ny) * pitch;
    const int pl = lx * V;
    OutMask<V> om;
    om.all = true;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        om.ov[v] = out_row && (pl + v >= HV) && (pl + v < HV + a.ow) && (xl + v < nx);
        om.all = om.all && om.ov[v];
    }
    const RowIO<T, V, FAST> io(xb, lx, nx);
    const T *in[2] = {a.buf[0][par], a.buf[NF - 1][par]};
    T *out[2] = {a.buf[0][par ^ 1], a.buf[NF - 1][par ^ 1]};

    T ring[NF][K][V];
    constexpr int PD = prefetch_depth<T, KIND, R, TB, RED, RPW>();
    T pre[NF][PD][V];                                // planes t+1 .. t+PD
    T r1[TB == 2 ? NF : 1][K][V];
    T m0[KIND == kCH ? K : 1][V];
    T m1[(KIND == kCH && TB == 2) ? K : 1][V];
    T mz[KIND == kCHD ? K : 1][V];                   // direct biharmonic: mu_z ring
    // phases per loop iteration: a multiple of the ring depth and of the
    // prefetch depth, so that plane t sits in ring slot t mod K and prefetch
    // slot t mod PD at compile time
    constexpr int NP = K % PD == 0 ? K : K * PD;
    // rings that feed LDS rows or later stages before first being computed hold zeros
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if constexpr (KIND == kCH) {
                m0[i][v] = T(0);
                if constexpr (TB == 2) m1[i][v] = T(0);
            }
            if constexpr (KIND == kCHD) mz[i][v] = T(0);
            if constexpr (TB == 2)
#pragma unroll
                for (int f = 0; f < NF; ++f) r1[f][i][v] = T(0);
        }
    RedState red[TB];
    // a stage at depth k computes rows [k r, NR - k r) of the tile
    auto rows_ok = [&](int k) { return rw >= k * R && rw < NR - k * R; };

    const int32_t tb0 = z0 - H, tend = z1 + H;
    // The first PD planes are loaded unconditionally (a plane past the march
    // is a valid wrapped plane, read and not used), so that every load of the
    // unguarded main loop below has a fixed number of loads issued after it
    // and the compiler can wait for it alone instead of draining all of them.
    static_for<0, PD>([&](auto phc) {
        constexpr int ph = decltype(phc)::value;
        const int64_t off = (int64_t)wrap32(tb0 + ph, nz) * plane + rowoff;
#pragma unroll
        for (int f = 0; f < NF; ++f) io.load(in[f] + off, pre[f][ph]);
    });

    // One plane t of the march at ring phase ph; G guards the planes and the
    // prefetch against the end of the march (the tail only).  The guards are
    // uniform over the workgroup, so every wave reaches the same barriers.
    auto phase = [&](auto phc, auto gc, int32_t tb) {
        constexpr int ph = decltype(phc)::value;
        constexpr bool G = decltype(gc)::value;
        const int32_t t = tb + ph;
        if (!G || t < tend) {
            const int32_t age = t - tb0;
            const int buf = TL::NB == 2 ? (int)(t & 1) : 0;
            auto &L = lds[buf];
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int v = 0; v < V; ++v) ring[f][ph % K][v] = pre[f][ph % PD][v];
            if (!G || t + PD < tend) {
                const int64_t off = (int64_t)wrap32(t + PD, nz) * plane + rowoff;
#pragma unroll
                for (int f = 0; f < NF; ++f) io.load(in[f] + off, pre[f][ph % PD]);
            }
            if constexpr (KIND == kCHD) {
                // the direct biharmonic: mu_z of the arriving plane t, and the
                // update of the centre plane t - (r + 1)
                constexpr int sa = ph % K, sc = Slot<K, R + 1>::template at<ph>;
                T my[V];
                stage3_chd_mu_y<T, R, K, sc>(a, ring[0], my);
                if constexpr (TL::NB == 1) __syncthreads();
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    L[0][0][rw][pl + v] = ring[0][sa][v];
                    L[1][0][rw][pl + v] = ring[0][sc][v];
                    L[2][0][rw][pl + v] = my[v];
                }
                __syncthreads();
                if (rows_ok(1)) stage3_chd_mu_z<T, R, K, sa, NR, RW>(a, ring[0], L[0][0], rw, pl, mz);
                if (age >= 2 * H && rw >= H && rw < NR - H) {
                    const int32_t pz = t - H;
                    T res[V];
                    stage3_chd_update<T, R, K, sc, NR, RW, RED>(a, ring[0], my, mz, L[1][0], L[2][0], rw, pl,
                                                                res, om, pz >= z0 && pz < z1, red[0]);
                    if (out_row)
                        store_row<T, V>(out[0] + (int64_t)wrap32(pz, nz) * plane + rowoff, xl, om, res);
                }
            } else if constexpr (KIND == kCHMU || KIND == kCHUP) {
                // one radius-r stage: mu of c (with the reductions of c), or
                // the update of c from the mu stream and c's centre plane
                constexpr int s1 = Slot<K, R>::template at<ph>;
                if constexpr (TL::NB == 1) __syncthreads();
#pragma unroll
                for (int v = 0; v < V; ++v) L[0][0][rw][pl + v] = ring[0][s1][v];
                __syncthreads();
                if (age >= 2 * R && rows_ok(1)) {
                    const int32_t pz = t - R;
                    T res[V];
                    if constexpr (KIND == kCHMU)
                        stage3_mu<T, R, K, s1, NR, RW, RED>(a, ring[0], L[0][0], rw, pl, res, om,
                                                            pz >= z0 && pz < z1, red[0]);
                    else
                        stage3_chupd<T, R, K, s1, NR, RW>(a, ring[0], L[0][0], rw, pl, ring[NF - 1][s1], res);
                    if (out_row)
                        store_row<T, V>(out[0] + (int64_t)wrap32(pz, nz) * plane + rowoff, xl, om, res);
                }
            } else {
                constexpr int s1 = Slot<K, R>::template at<ph>;
                constexpr int s2 = Slot<K, 2 * R>::template at<ph>;
                constexpr int s3 = Slot<K, 3 * R>::template at<ph>;
                constexpr int s4 = Slot<K, 4 * R>::template at<ph>;
                if constexpr (TL::NB == 1) __syncthreads();  // previous plane's readers are done
                // centre rows of every stage's input stream
                if constexpr (KIND != kCH) {
#pragma unroll
                    for (int f = 0; f < NF; ++f)
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            // Model C keeps phi and g = rho + c3 phi^2 (the diffused field) in LDS
                            // (the g branch is live only for Model C, NF = 2)
                            L[0][f][rw][pl + v] = (KIND == kMC && f == 1)
                                                      ? mc_g(a, ring[0][s1][v], ring[NF - 1][s1][v])
                                                      : ring[f][s1][v];
                            if constexpr (TB == 2)
                                L[TB - 1][f][rw][pl + v] = (KIND == kMC && f == 1)
                                                               ? mc_g(a, r1[0][s2][v], r1[NF - 1][s2][v])
                                                               : r1[f][s2][v];
                        }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        L[0][0][rw][pl + v] = ring[0][s1][v];
                        L[1][0][rw][pl + v] = m0[s2][v];
                        if constexpr (TB == 2) {
                            L[TB][0][rw][pl + v] = r1[0][s3][v];
                            L[TB + 1][0][rw][pl + v] = m1[s4][v];
                        }
                    }
                }
                __syncthreads();
                if constexpr (KIND != kCH) {
                    if (age >= 2 * R && rows_ok(1)) {
                        const int32_t pz = t - R;
                        T res[NF][V];
                        stage3_acgs<T, KIND, R, K, s1, NR, RW, RED>(a, ring, L[0], rw, pl, res, om,
                                                                    pz >= z0 && pz < z1, red[0]);
                        if constexpr (TB == 1) {
                            if (out_row) {
                                const int64_t ooff = (int64_t)wrap32(pz, nz) * plane + rowoff;
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
                            const int32_t pz = t - 2 * R;
                            T res[NF][V];
                            stage3_acgs<T, KIND, R, K, s2, NR, RW, RED>(
                                a, r1, L[TB - 1], rw, pl, res, om, pz >= z0 && pz < z1, red[TB - 1]);
                            if (out_row) {
                                const int64_t ooff = (int64_t)wrap32(pz, nz) * plane + rowoff;
#pragma unroll
                                for (int f = 0; f < NF; ++f)
                                    store_row<T, V>(out[f] + ooff, xl, om, res[f]);
                            }
                        }
                    }
                } else {
                    if (age >= 2 * R && rows_ok(1)) {
                        const int32_t pz = t - R;
                        stage3_mu<T, R, K, s1, NR, RW, RED>(a, ring[0], L[0][0], rw, pl, m0[s1], om,
                                                            pz >= z0 && pz < z1, red[0]);
                    }
                    if (age >= 4 * R && rows_ok(2)) {
                        T res[V];
                        stage3_chupd<T, R, K, s2, NR, RW>(a, m0, L[1][0], rw, pl, ring[0][s2], res);
                        if constexpr (TB == 1) {
                            if (out_row)
                                store_row<T, V>(out[0] + (int64_t)wrap32(t - 2 * R, nz) * plane + rowoff, xl,
                                                om, res);
                        } else {
#pragma unroll
                            for (int v = 0; v < V; ++v) r1[0][s2][v] = res[v];
                        }
                    }
                    if constexpr (TB == 2) {
                        if (age >= 6 * R && rows_ok(3)) {
                            const int32_t pz = t - 3 * R;
                            stage3_mu<T, R, K, s3, NR, RW, RED>(a, r1[0], L[TB][0], rw, pl, m1[s3],
                                                                om, pz >= z0 && pz < z1, red[TB - 1]);
                        }
                        if (age >= 8 * R && rows_ok(4)) {
                            T res[V];
                            stage3_chupd<T, R, K, s4, NR, RW>(a, m1, L[TB + 1][0], rw, pl, r1[0][s4],
                                                              res);
                            if (out_row)
                                store_row<T, V>(out[0] + (int64_t)wrap32(t - 4 * R, nz) * plane + rowoff,
                                                xl, om, res);
                        }
                    }
                }
            }
        }
    };
    int32_t tb = tb0;
    for (; tb + NP + PD <= tend; tb += NP)
        static_for<0, NP>([&](auto phc) { phase(phc, std::false_type{}, tb); });
    for (; tb < tend; tb += NP)
        static_for<0, NP>([&](auto phc) { phase(phc, std::true_type{}, tb); });
    if constexpr (RED) {
        red_flush(red[0], a.part, a.pstride, pslot, lane);
        if constexpr (TB == 2)
            red_flush(red[TB - 1], a.part, a.pstride, pslot + (int64_t)a.items * kWaves3D, lane);
        if constexpr (TL::NW < kWaves3D) {
            // an 8- or 12-wave workgroup clears the partial slots of the waves
            // it does not have (each item owns kWaves3D slots per time step)
            constexpr int M = kWaves3D - TL::NW;
            const int tid = threadIdx.x;
            const int64_t base = pslot - __builtin_amdgcn_readfirstlane(tid >> 6) + TL::NW;
            if (tid < kNumQ * M * TB) {
                const int q = tid / (M * TB), rest = tid % (M * TB), s = rest % M, step = rest / M;
                a.part[(int64_t)q * a.pstride + base + s + step * (int64_t)a.items * kWaves3D] =
                    make_double2(0.0, 0.0);
            }
        }
    }
}

template <typename T, int KIND, int R, bool RED, int TB, int RPW>
__device__ __forceinline__ void step3d_item(const StepArgs<T> &a, int par, int32_t item,
                                            int64_t pslot_base)
{
    using TL = Tile3D<T, KIND, R, TB, RPW>;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rw = tile_row<TL::RPW, TL::LPR>();
    const int32_t strip = item % a.strips;
    const int32_t rest = item / a.strips;
    const int32_t ytile = rest % a.ytiles;
    const int32_t chunk = rest / a.ytiles;
    const int64_t xb = (int64_t)strip * a.ow - TL::HV;
    const int64_t yrow = (int64_t)ytile * (TL::NR - 2 * TL::H) - TL::H + rw;
    const bool out_row = (rw >= TL::H) && (rw < TL::NR - TL::H) && (yrow < a.ny);
    const int32_t z0 = chunk * a.clen;
    const int32_t z1 = min(z0 + a.clen, (int32_t)a.nz);
    __shared__ typename TL::lds_type lds;
    // the FAST choice is uniform over the workgroup (it depends on the strip only)
    if (xb >= 0 && xb + TL::RW <= a.nx)
        march3d<T, KIND, R, RED, true, TB, RPW>(a, par, xb, yrow, out_row, z0, z1, pslot_base + w, lds);
    else
        march3d<T, KIND, R, RED, false, TB, RPW>(a, par, xb, yrow, out_row, z0, z1, pslot_base + w, lds);
}

template <typename T, int KIND, int R, bool RED, int TB, int RPW>
__global__ void __launch_bounds__((64 * Tile3D<T, KIND, R, TB, RPW>::NW)) k_step3d(StepArgs<T> a)
{
    const int32_t item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= a.items) return;  // uniform over the workgroup
    step3d_item<T, KIND, R, RED, TB, RPW>(a, a.parity, item, (int64_t)item * kWaves3D);
}

// Rows per wave of the batched (serving) 3D kernels: two, or four (8-wave
// workgroups, up to 256 registers a lane) for the classes whose two-row
// kernel would spill (Model C, Gray-Scott with r >= 3).
template <int KIND, int R>
constexpr int batched_rpw()
{
    return (KIND == kMC || (KIND == kGS && R >= 3)) ? 4 : 2;
}

// Persistent batched 3D step (see k_step2d_batched); the item loop and the
// choice of a two-step sweep are uniform over the workgroup, so every wave
// reaches the same barriers.
template <typename T, int KIND, int R, int TB>
__global__ void __launch_bounds__((64 * Tile3D<T, KIND, R, 1, batched_rpw<KIND, R>()>::NW))
    k_step3d_batched(BatchTable<T> tb, int32_t k)
{
    constexpr int RPW = batched_rpw<KIND, R>();
    const int32_t n = *tb.count;
    const int32_t total = tb.item_start[n];
    for (int32_t g = blockIdx.x; g < total; g += gridDim.x) {
        const int i = batch_request(tb, n, g);
        const int32_t left = tb.steps[i] - k;
        if (left <= 0) continue;
        const StepArgs<T> &a = tb.args[i];
        const int par = (a.parity + k / TB) & 1;
        if constexpr (TB == 2) {
            if (left >= 2) {
                step3d_item<T, KIND, R, false, 2, RPW>(a, par, g - tb.item_start[i], 0);
                continue;
            }
        }
        step3d_item<T, KIND, R, false, 1, RPW>(a, par, g - tb.item_start[i], 0);
    }
}

}  // namespace pf
