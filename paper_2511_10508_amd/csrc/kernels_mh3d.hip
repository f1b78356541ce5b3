// Model H (Eq. model-h, transverse projector one) on 3D grids in one pass,
// over column tiles (r = 1, this comment) or on the 3D march (r = 2, below).
//
// A workgroup owns an x-y tile of output columns and marches along z
// over a chunk of planes.  Each thread holds one column of the tile plus a
// halo of 2r on each side (the columns of mu's own neighbours): for every
// plane it keeps z-windows of m, j_x, j_y, j_z (3r + 1 planes) and of mu
// (2r + 1 planes) in registers, and the centre planes the x-y neighbours
// come from in LDS (double-buffered, one barrier per plane).  When plane t
// arrives:
//   mu at plane t - r   = c2 m^3 - c1 m - L m            (tile + r halo)
//   the update at q = t - 2r:
//     m'   = m + dt L mu - dt c3 div(m j)
//     j_a' = j_a + dt L j_a + dt c3 m D1_a mu
// so mu never reaches HBM, each field is read once and written once per
// step (up to the re-read tile halos), and the loads of plane t + 2 are in
// flight while plane t is computed.  Every value is formed with the
// per-site kernel's functions in its order (pairs x, then y, then z;
// divergence x, then y, then z), so the fields are bitwise those of the
// two-pass per-site kernel.
#include "pf_dispatch.h"
#include "pf_march3d.h"

namespace pf {

namespace {

constexpr int kMH3Items = 2048;  // work items a launch aims for (z chunks)

// Output columns of a tile: 32 x 16.
template <typename T, int R>
struct MH3Tile {
    static constexpr int TX = 32, TY = 16;
    static constexpr int G = 2 * R;                      // staged halo
    static constexpr int LX = TX + 2 * G, LY = TY + 2 * G;
    static constexpr int NT = LX * LY;                   // columns (threads that load)
    static constexpr int THREADS = (NT + 63) / 64 * 64;
    static constexpr int ZW = 3 * R + 1;                 // z-window of the fields
    static constexpr int MW = 2 * R + 1;                 // z-window of mu
};

// Planes in LDS per buffer: m at the mu plane, then m, j_x, j_y, j_z and mu
// at the update plane.
enum { kLm = 0, kLmq = 1, kLjx = 2, kLjy = 3, kLjz = 4, kLmu = 5, kLPlanes = 6 };

template <typename T, int R>
__global__ void __launch_bounds__((MH3Tile<T, R>::THREADS)) k_mh3d(StepArgs<T> a, int32_t tiles_x,
                                                             int32_t tiles_y, int32_t clen)
{
    using TL = MH3Tile<T, R>;
    constexpr int G = TL::G, LX = TL::LX, LY = TL::LY, ZW = TL::ZW, MW = TL::MW;
    __shared__ T L[2][kLPlanes][LY][LX];

    const int32_t item = xcd_item(blockIdx.x, gridDim.x);
    const int32_t tx = item % tiles_x, rest = item / tiles_x;
    const int32_t ty = rest % tiles_y, chunk = rest / tiles_y;
    const int32_t nz = (int32_t)a.nz;
    const int32_t z0 = chunk * clen, z1 = min(z0 + clen, nz);
    const int tid = threadIdx.x;
    const bool col = tid < TL::NT;  // threads past the tile's columns only take part in barriers
    const int lx = col ? tid % LX : 0, ly = col ? tid / LX : 0;
    const int64_t x0 = (int64_t)tx * TL::TX, y0 = (int64_t)ty * TL::TY;
    const int64_t coff = wrap_any(y0 - G + ly, a.ny) * a.pitch + wrap_any(x0 - G + lx, a.nx);
    const bool mu_col = col && lx >= R && lx < LX - R && ly >= R && ly < LY - R;
    const bool out_col = col && lx >= G && lx < LX - G && ly >= G && ly < LY - G &&
                         x0 + lx - G < a.nx && y0 + ly - G < a.ny;
    const int par = a.parity;
    const T *__restrict__ in[4] = {a.buf[0][par], a.buf[1][par], a.buf[2][par], a.buf[3][par]};
    T *__restrict__ out[4] = {a.buf[0][par ^ 1], a.buf[1][par ^ 1], a.buf[2][par ^ 1], a.buf[3][par ^ 1]};
    const T ctr = T(6);

    // z-windows: fm[i] holds m at plane t - 3r + i (i <= 3r), fj[c][i] j_c at
    // plane t - 3r + i (i <= 2r; j is first needed r planes after m), mu[i]
    // mu at plane t - 3r + i (before this plane's mu is shifted in).  Loads
    // run two planes ahead into pm / pj, alternating between two register
    // sets so that a value is first touched two planes after its load.
    T fm[ZW], fj[3][MW], mu[MW], pm[2], pj[2][3];
#pragma unroll
    for (int i = 0; i < ZW; ++i) fm[i] = T(0);
#pragma unroll
    for (int i = 0; i < MW; ++i) {
        mu[i] = T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) fj[c][i] = T(0);
    }
    const int32_t t0 = z0 - G, tend = z1 + G;
    auto off_of = [&](int32_t t) { return (int64_t)wrap32(t, nz) * a.plane + coff; };
    auto load_m = [&](int32_t t, T &v) { v = col ? in[0][off_of(t)] : T(0); };
    auto load_j = [&](int32_t t, T (&v)[3]) {
        const int64_t off = off_of(t);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = col ? in[1 + c][off] : T(0);
    };
    load_m(t0, pm[0]);
    load_j(t0 - R, pj[0]);
    load_m(t0 + 1, pm[1]);
    load_j(t0 + 1 - R, pj[1]);

    auto phase = [&](int32_t t, auto parc) {
        constexpr int PH = decltype(parc)::value;
        const int32_t age = t - t0;
        // shift the windows by one plane: m of plane t and j of plane t - r
        // enter; m of t + 2 and j of t + 2 - r are requested
#pragma unroll
        for (int i = 0; i < ZW - 1; ++i) fm[i] = fm[i + 1];
        fm[ZW - 1] = pm[PH];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int i = 0; i < MW - 1; ++i) fj[c][i] = fj[c][i + 1];
            fj[c][MW - 1] = pj[PH][c];
        }
        load_m(t + 2, pm[PH]);
        load_j(t + 2 - R, pj[PH]);
        // centre planes: m at t - r (index 2r), m / j / mu at q = t - 2r (index r;
        // mu(q) is mu[r + 1] until this plane's mu is shifted in)
        auto &B = L[t & 1];
        if (col) {
            B[kLm][ly][lx] = fm[2 * R];
            B[kLmq][ly][lx] = fm[R];
            B[kLjx][ly][lx] = fj[0][R];
            B[kLjy][ly][lx] = fj[1][R];
            B[kLjz][ly][lx] = fj[2][R];
            B[kLmu][ly][lx] = mu[R + 1];
        }
        __syncthreads();
        // mu of plane t - r
        T mnew = T(0);
        if (age >= 2 * R && mu_col) {
            T S[R];
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                T acc = B[kLm][ly][lx + j] + B[kLm][ly][lx - j];
                acc = acc + (B[kLm][ly + j][lx] + B[kLm][ly - j][lx]);
                acc = acc + (fm[2 * R + j] + fm[2 * R - j]);
                S[j - 1] = acc;
            }
            const T c0 = fm[2 * R];
            mnew = ch_mu<T, R>(a, c0, S, c0 * ctr);
        }
#pragma unroll
        for (int i = 0; i < MW - 1; ++i) mu[i] = mu[i + 1];
        mu[MW - 1] = mnew;  // now mu[i] holds plane t - 3r + i: mu(q) = mu[r]
        // the update of plane q = t - 2r
        if (age >= 4 * R && out_col) {
            const int32_t q = t - 2 * R;
            const T m0 = fm[R], mu0 = B[kLmu][ly][lx];
            T Sm[R];
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                T acc = B[kLmu][ly][lx + j] + B[kLmu][ly][lx - j];
                acc = acc + (B[kLmu][ly + j][lx] + B[kLmu][ly - j][lx]);
                acc = acc + (mu[R + j] + mu[R - j]);
                Sm[j - 1] = acc;
            }
            T div = T(0);
#pragma unroll
            for (int k = 1; k <= R; ++k)
                div = fma(a.w1[k - 1], B[kLmq][ly][lx + k] * B[kLjx][ly][lx + k] -
                                           B[kLmq][ly][lx - k] * B[kLjx][ly][lx - k], div);
#pragma unroll
            for (int k = 1; k <= R; ++k)
                div = fma(a.w1[k - 1], B[kLmq][ly + k][lx] * B[kLjy][ly + k][lx] -
                                           B[kLmq][ly - k][lx] * B[kLjy][ly - k][lx], div);
#pragma unroll
            for (int k = 1; k <= R; ++k)
                div = fma(a.w1[k - 1], fm[R + k] * fj[2][R + k] - fm[R - k] * fj[2][R - k], div);
            const int64_t off = off_of(q);
            out[0][off] = fma(-a.k2, div, ch_update<T, R>(a, m0, Sm, mu0 * ctr));
            const T km = a.k2 * m0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int pl = kLjx + ax;
                T Sj[R];
                T grad = T(0);
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    T acc = B[pl][ly][lx + j] + B[pl][ly][lx - j];
                    acc = acc + (B[pl][ly + j][lx] + B[pl][ly - j][lx]);
                    acc = acc + (fj[ax][R + j] + fj[ax][R - j]);
                    Sj[j - 1] = acc;
                }
#pragma unroll
                for (int k = 1; k <= R; ++k) {
                    T d;
                    if (ax == 0)
                        d = B[kLmu][ly][lx + k] - B[kLmu][ly][lx - k];
                    else if (ax == 1)
                        d = B[kLmu][ly + k][lx] - B[kLmu][ly - k][lx];
                    else
                        d = mu[R + k] - mu[R - k];
                    grad = fma(a.w1[k - 1], d, grad);
                }
                const T j0 = fj[ax][R];
                out[1 + ax][off] = fma(km, grad, ch_update<T, R>(a, j0, Sj, j0 * ctr));
            }
        }
    };
    // two planes per iteration: the register sets alternate at compile time
    // (the trip count is uniform over the workgroup, so every thread reaches
    // the same barriers)
    int32_t t = t0;
    for (; t + 1 < tend; t += 2) {
        phase(t, std::integral_constant<int, 0>{});
        phase(t + 1, std::integral_constant<int, 1>{});
    }
    if (t < tend) phase(t, std::integral_constant<int, 0>{});
}

// ---------------------------------------------------------------------------
// The same step on the 3D march of the other models (used for r = 2, see
// mh3d_marches): a workgroup of 8 waves
// owns a tile of 32 rows (four 16-lane rows per wave, V values per lane) of
// one x-strip and marches along z.  x-neighbours come by lane shifts, y-
// neighbours from the six centre planes in LDS (double-buffered, one barrier
// per plane), z-neighbours from rings in registers: m (planes t - 3r .. t),
// j (loaded r planes later, t - 3r .. t - r) and mu (t - 3r .. t - r).  The
// halo is 2r in x and y; values are formed in the order above, so the fields
// are bitwise those of the column kernel and of the per-site kernels.
template <typename T, int R>
struct MH3March {
    static constexpr int V = Vec<T>::V, H = 2 * R, HV = (H + V - 1) / V * V;
    static constexpr int RPW = 4, LPR = 64 / RPW, NW = 8, NR = RPW * NW, RW = LPR * V;
    static constexpr int OWMAX = RW - 2 * HV;
    static constexpr int PD = 1;         // planes in flight (the rings take up to 250 registers)
    static constexpr int K = 3 * R + 1;  // ring slots
};

// LDS planes per buffer: m at the mu plane, then m, j_x, j_y, j_z and mu at
// the update plane (as in the column kernel).
enum { kXm = 0, kXmq = 1, kXjx = 2, kXmu = 5, kXPlanes = 6 };

template <typename T, int R, bool FAST>
__device__ __forceinline__ void mh3d_march(const StepArgs<T> &a, int64_t xb, int lx, int rw, int64_t rowoff,
                                           bool out_row, int32_t z0, int32_t z1,
                                           T (&lds)[2][kXPlanes][MH3March<T, R>::NR][MH3March<T, R>::RW])
{
    using TL = MH3March<T, R>;
    constexpr int V = TL::V, H = TL::H, HV = TL::HV, NR = TL::NR, K = TL::K, PD = TL::PD;
    const int32_t nz = (int32_t)a.nz;
    const int64_t plane = a.plane;
    const int64_t xl = xb + lx * V;
    const int pl = lx * V;
    OutMask<V> om;
    om.all = true;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        om.ov[v] = out_row && (pl + v >= HV) && (pl + v < HV + a.ow) && (xl + v < a.nx);
        om.all = om.all && om.ov[v];
    }
    const RowIO<T, V, FAST> io(xb, lx, a.nx);
    const int par = a.parity;
    const T *in[4] = {a.buf[0][par], a.buf[1][par], a.buf[2][par], a.buf[3][par]};
    T *out[4] = {a.buf[0][par ^ 1], a.buf[1][par ^ 1], a.buf[2][par ^ 1], a.buf[3][par ^ 1]};
    const T ctr = T(6);

    // ring slot of a value that entered D planes ago: Slot<K, D>; m of plane
    // p enters at plane p, j and mu of plane p at plane p + r
    T m[K][V], j[3][K][V], mu[K][V], pm[PD][V], pj[PD][3][V];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            m[i][v] = mu[i][v] = T(0);
            j[0][i][v] = j[1][i][v] = j[2][i][v] = T(0);
        }
    const int32_t tb0 = z0 - H, tend = z1 + H;
    auto load = [&](int32_t t, T (&vm)[V], T (&vj)[3][V]) {
        const int64_t offm = (int64_t)wrap32(t, nz) * plane + rowoff;
        const int64_t oj = (int64_t)wrap32(t - R, nz) * plane + rowoff;
        io.load(in[0] + offm, vm);
#pragma unroll
        for (int c = 0; c < 3; ++c) io.load(in[1 + c] + oj, vj[c]);
    };
    // the first PD planes load unconditionally (a plane past the march is a
    // valid wrapped plane, read and not used)
    static_for<0, PD>([&](auto phc) {
        constexpr int ph = decltype(phc)::value;
        load(tb0 + ph, pm[ph], pj[ph]);
    });
    auto rows_ok = [&](int k) { return rw >= k * R && rw < NR - k * R; };

    // plane t at ring phase ph; G guards the tail (uniform over the workgroup)
    auto phase = [&](auto phc, auto gc, int32_t tb) {
        constexpr int ph = decltype(phc)::value;
        constexpr bool G = decltype(gc)::value;
        const int32_t t = tb + ph;
        if (!G || t < tend) {
            const int32_t age = t - tb0;
            constexpr int s0 = ph % K;                            // entered at this plane
            constexpr int sr = Slot<K, R>::template at<ph>;       // m(t - r), j(q), mu(q)
            constexpr int sq = Slot<K, 2 * R>::template at<ph>;   // m(q)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                m[s0][v] = pm[ph % PD][v];
#pragma unroll
                for (int c = 0; c < 3; ++c) j[c][s0][v] = pj[ph % PD][c][v];
            }
            if (!G || t + PD < tend) load(t + PD, pm[ph % PD], pj[ph % PD]);
            auto &L = lds[t & 1];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                L[kXm][rw][pl + v] = m[sr][v];
                L[kXmq][rw][pl + v] = m[sq][v];
#pragma unroll
                for (int c = 0; c < 3; ++c) L[kXjx + c][rw][pl + v] = j[c][sr][v];
                L[kXmu][rw][pl + v] = mu[sr][v];
            }
            __syncthreads();
            // mu of plane t - r into slot s0
            if (age >= 2 * R && rows_ok(1)) {
                T e[V + 2 * R];
                gather_x<T, V, R>(m[sr], e);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    T S[R];
                    static_for<1, R + 1>([&](auto jc) {
                        constexpr int jj = decltype(jc)::value;
                        constexpr int sp = Slot<K, R - jj>::template at<ph>, sm = Slot<K, R + jj>::template at<ph>;
                        T acc = e[R + v + jj] + e[R + v - jj];
                        acc = acc + (L[kXm][rw + jj][pl + v] + L[kXm][rw - jj][pl + v]);
                        acc = acc + (m[sp][v] + m[sm][v]);
                        S[jj - 1] = acc;
                    });
                    const T c0 = m[sr][v];
                    mu[s0][v] = ch_mu<T, R>(a, c0, S, c0 * ctr);
                }
            }
            // the update of plane q = t - 2r
            if (age >= 4 * R && rows_ok(2)) {
                const int32_t q = t - 2 * R;
                const int64_t ooff = (int64_t)wrap32(q, nz) * plane + rowoff;
                T emu[V + 2 * R], res[V];
                gather_x<T, V, R>(mu[sr], emu);
                {
                    T em[V + 2 * R], ejx[V + 2 * R];
                    gather_x<T, V, R>(m[sq], em);
                    gather_x<T, V, R>(j[0][sr], ejx);
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        T Sm[R];
                        static_for<1, R + 1>([&](auto jc) {
                            constexpr int jj = decltype(jc)::value;
                            constexpr int sp = Slot<K, R - jj>::template at<ph>, sm = Slot<K, R + jj>::template at<ph>;
                            T acc = emu[R + v + jj] + emu[R + v - jj];
                            acc = acc + (L[kXmu][rw + jj][pl + v] + L[kXmu][rw - jj][pl + v]);
                            acc = acc + (mu[sp][v] + mu[sm][v]);
                            Sm[jj - 1] = acc;
                        });
                        T div = T(0);
                        static_for<1, R + 1>([&](auto kc) {
                            constexpr int k = decltype(kc)::value;
                            div = fma(a.w1[k - 1], em[R + v + k] * ejx[R + v + k] - em[R + v - k] * ejx[R + v - k], div);
                        });
                        static_for<1, R + 1>([&](auto kc) {
                            constexpr int k = decltype(kc)::value;
                            div = fma(a.w1[k - 1], L[kXmq][rw + k][pl + v] * L[kXjx + 1][rw + k][pl + v] -
                                                       L[kXmq][rw - k][pl + v] * L[kXjx + 1][rw - k][pl + v], div);
                        });
                        static_for<1, R + 1>([&](auto kc) {
                            constexpr int k = decltype(kc)::value;
                            constexpr int mp = Slot<K, 2 * R - k>::template at<ph>, mm = Slot<K, 2 * R + k>::template at<ph>;
                            constexpr int jp = Slot<K, R - k>::template at<ph>, jm = Slot<K, R + k>::template at<ph>;
                            div = fma(a.w1[k - 1], m[mp][v] * j[2][jp][v] - m[mm][v] * j[2][jm][v], div);
                        });
                        res[v] = fma(-a.k2, div, ch_update<T, R>(a, m[sq][v], Sm, mu[sr][v] * ctr));
                    }
                }
                if (out_row) store_row<T, V>(out[0] + ooff, xl, om, res);
                static_for<0, 3>([&](auto axc) {
                    constexpr int ax = decltype(axc)::value;
                    T ej[V + 2 * R];
                    gather_x<T, V, R>(j[ax][sr], ej);
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        T Sj[R];
                        T grad = T(0);
                        static_for<1, R + 1>([&](auto jc) {
                            constexpr int jj = decltype(jc)::value;
                            constexpr int sp = Slot<K, R - jj>::template at<ph>, sm = Slot<K, R + jj>::template at<ph>;
                            T acc = ej[R + v + jj] + ej[R + v - jj];
                            acc = acc + (L[kXjx + ax][rw + jj][pl + v] + L[kXjx + ax][rw - jj][pl + v]);
                            acc = acc + (j[ax][sp][v] + j[ax][sm][v]);
                            Sj[jj - 1] = acc;
                        });
                        static_for<1, R + 1>([&](auto kc) {
                            constexpr int k = decltype(kc)::value;
                            constexpr int sp = Slot<K, R - k>::template at<ph>, sm = Slot<K, R + k>::template at<ph>;
                            T d;
                            if constexpr (ax == 0)
                                d = emu[R + v + k] - emu[R + v - k];
                            else if constexpr (ax == 1)
                                d = L[kXmu][rw + k][pl + v] - L[kXmu][rw - k][pl + v];
                            else
                                d = mu[sp][v] - mu[sm][v];
                            grad = fma(a.w1[k - 1], d, grad);
                        });
                        const T j0 = j[ax][sr][v];
                        res[v] = fma(a.k2 * m[sq][v], grad, ch_update<T, R>(a, j0, Sj, j0 * ctr));
                    }
                    if (out_row) store_row<T, V>(out[1 + ax] + ooff, xl, om, res);
                });
            }
        }
    };
    int32_t tb = tb0;
    for (; tb + K + PD <= tend; tb += K)
        static_for<0, K>([&](auto phc) { phase(phc, std::false_type{}, tb); });
    for (; tb < tend; tb += K)
        static_for<0, K>([&](auto phc) { phase(phc, std::true_type{}, tb); });
}

template <typename T, int R>
__global__ void __launch_bounds__((64 * MH3March<T, R>::NW)) k_mh3d_march(StepArgs<T> a)
{
    using TL = MH3March<T, R>;
    __shared__ T lds[2][kXPlanes][TL::NR][TL::RW];
    const int32_t item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= a.items) return;  // uniform over the workgroup
    const int32_t strip = item % a.strips, rest = item / a.strips;
    const int32_t ytile = rest % a.ytiles, chunk = rest / a.ytiles;
    const int lx = (int)(threadIdx.x & 63) % TL::LPR;
    const int rw = tile_row<TL::RPW, TL::LPR>();
    const int64_t xb = (int64_t)strip * a.ow - TL::HV;
    const int64_t yrow = (int64_t)ytile * (TL::NR - 2 * TL::H) - TL::H + rw;
    const bool out_row = rw >= TL::H && rw < TL::NR - TL::H && yrow < a.ny;
    const int64_t rowoff = wrap_any(yrow, a.ny) * a.pitch;
    const int32_t z0 = chunk * a.clen, z1 = min(z0 + a.clen, (int32_t)a.nz);
    // the FAST choice is uniform over the workgroup (it depends on the strip only)
    if (xb >= 0 && xb + TL::RW <= a.nx)
        mh3d_march<T, R, true>(a, xb, lx, rw, rowoff, out_row, z0, z1, lds);
    else
        mh3d_march<T, R, false>(a, xb, lx, rw, rowoff, out_row, z0, z1, lds);
}

// Launch geometry of the march: strips, outputs per strip, y tiles and z
// chunks (at least 16 planes each, enough work items to fill the chip).
template <typename T, int R>
bool plan_mh3d_march(StepArgs<T> &a)
{
    using TL = MH3March<T, R>;
    const int64_t st = cdiv(a.nx, TL::OWMAX);
    const int64_t yt = cdiv(a.ny, TL::NR - 2 * TL::H);
    const int64_t chunks = std::max<int64_t>(1, std::min<int64_t>(cdiv(kMH3Items, st * yt), a.nz / 16));
    const int64_t clen = cdiv(a.nz, chunks);
    const int64_t items = st * yt * cdiv(a.nz, clen);
    if (items > (int64_t)INT32_MAX) return false;
    a.strips = (int32_t)st;
    a.ow = (int32_t)(cdiv(cdiv(a.nx, st), TL::V) * TL::V);
    a.ytiles = (int32_t)yt;
    a.clen = (int32_t)clen;
    a.chunks = (int32_t)cdiv(a.nz, clen);
    a.items = (int32_t)items;
    return true;
}

// The march runs r = 2 (on 512^3 1.55x faster than the column tiles in FP64,
// on par in FP32); the column tiles run r = 1, where they are 1.2-1.3x faster.
template <int R>
constexpr bool mh3d_marches()
{
    return R == 2;
}

}  // namespace

bool mh3d_available(const Launch &L) { return L.kind == kMH && L.ndim == 3 && L.r >= 1 && L.r <= 2; }

hipError_t launch_mh3d(const Launch &L, const void *args, hipStream_t s)
{
    hipError_t err = hipErrorInvalidValue;
    if (!mh3d_available(L)) return err;
    dispatch_prec(L.fp32, [&](auto tz) {
        using T = decltype(tz);
        const StepArgs<T> &a = *static_cast<const StepArgs<T> *>(args);
        dispatch_r(L.r, RList<1, 2>{}, [&](auto rc) {
            constexpr int R = decltype(rc)::value;
            if constexpr (mh3d_marches<R>()) {
                StepArgs<T> b = a;
                if (!plan_mh3d_march<T, R>(b)) return;
                hipLaunchKernelGGL((k_mh3d_march<T, R>), dim3((unsigned)b.items), dim3(64 * MH3March<T, R>::NW), 0,
                                   s, b);
                err = hipGetLastError();
            } else {
                using TL = MH3Tile<T, R>;
                const int64_t tx = cdiv(a.nx, TL::TX), ty = cdiv(a.ny, TL::TY);
                const int64_t tiles = tx * ty;
                // z chunks: enough work items to fill the chip, at least 16 planes each
                const int64_t chunks =
                    std::max<int64_t>(1, std::min<int64_t>(cdiv(kMH3Items, tiles), a.nz / 16));
                const int64_t clen = cdiv(a.nz, chunks);
                const int64_t items = tiles * cdiv(a.nz, clen);
                if (items > (int64_t)INT32_MAX || tx > INT32_MAX || ty > INT32_MAX) return;
                hipLaunchKernelGGL((k_mh3d<T, R>), dim3((unsigned)items), dim3(TL::THREADS), 0, s, a,
                                   (int32_t)tx, (int32_t)ty, (int32_t)clen);
                err = hipGetLastError();
            }
        });
    });
    return err;
}

}  // namespace pf
