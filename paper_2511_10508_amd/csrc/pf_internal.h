// Internal interface between the host runtime and the HIP kernels of libpfmi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pf {

constexpr int kAC = 1, kCH = 2, kGS = 3, kMC = 4, kMH = 5;
// Kernel kind of Cahn-Hilliard with the direct biharmonic stencil (a
// descriptor flag on PF_CH; internal to the kernels and launchers).
constexpr int kCHD = 16;
// The two passes of Cahn-Hilliard with mu through a field-sized buffer (3D):
// kCHMU takes c and writes mu (and reduces c); kCHUP takes mu (stencil) and c
// (centre values only) and writes the stepped c.
constexpr int kCHMU = 17, kCHUP = 18;
constexpr int kMaxFields = 4;       // Model H in 3D: m and three components of j

// Fields a kernel family reduces and steps as a fixed set: Gray-Scott (u, v)
// and Model C (phi, rho) have two.  Model H has 1 + ndim (m and j), stepped by
// its own kernels (the 1D strip kernel, the 2D and 3D marching kernels, the per-site
// kernels elsewhere); its reductions cover m.
constexpr int nfields_kind(int kind) { return (kind == kGS || kind == kMC || kind == kCHUP) ? 2 : 1; }
constexpr int kMaxR = 8;            // stencil radius r = order / 2 (order <= 16)
constexpr int kNumQ = 3;            // reduction quantities per partial slot
constexpr int kWaves2D = 4;         // waves per workgroup, 2D kernels
constexpr int kWaves3D = 16;        // waves per workgroup of the 3D kernels (two tile rows each)

// Reduction quantities of one partial slot:
//   q0 = sum of field 0, q1 = sum of field 1 (GS) or of the energy density
//   (AC, CH), q2 = number of non-finite values.  Each is an FP64 (hi, lo)
//   pair; the runtime scales the sums by dx^d.

// Arguments of one model's step, shared by the single-model and batched
// launches.  All sizes in elements.  Weights and constants are in the storage
// precision T (rounded once from FP64 on the host).
template <typename T>
struct StepArgs {
    T *buf[kMaxFields][2];   // [field][parity]
    int64_t nx, ny, nz;      // grid extents (nz = 1 in 2D)
    int64_t pitch;           // row stride
    int64_t plane;           // plane stride = pitch * ny
    int32_t parity;          // input buffer of this launch (output = 1 - parity)
    int32_t strips;          // x strips
    int32_t ow;              // outputs per strip
    int32_t ytiles;          // 3D: tiles along y
    int32_t chunks;          // chunks along the marching axis
    int32_t clen;            // chunk length
    int32_t items;           // work items (2D: waves, 3D: workgroups)
    int32_t red;             // fuse reductions into this launch
    T wi[kMaxR];             // w_j / dx^2 (inner Laplacian: CH chemical potential)
    T wu[kMaxR];             // update weights of field 0 (dt-scaled)
    T wv[kMaxR];             // update weights of field 1 (GS, MC)
    T w4[kMaxR + 1];         // -dt w4_j/dx^4 (direct biharmonic, j = 1..r+1)
    T w1[kMaxR];             // w1_j/dx (Model H: first derivatives, j = 1..r)
    T k0, k1, k2, k3;        // model constants (see kernels)
    double w64[kMaxR];       // w_j / dx^2 in FP64 (energy)
    double w64sum;           // sum_j w64[j] (energy by parts)
    double c1, c2;           // FP64 Landau constants (energy)
    double2 *part;           // partial sums [q][slot]
    int64_t pstride;         // slots per quantity
};

// Batched (serving) launch: a table of StepArgs, one per request of one
// kernel class, with work-item prefix sums; a launch processes step `k` of the
// current tick for every request whose `steps[i]` exceeds k.  Everything the
// kernel reads lives in device memory (the struct holds only pointers), so a
// captured graph stays valid when the table's contents change.
template <typename T>
struct BatchTable {
    StepArgs<T> *args;       // device array [n]
    int32_t *count;          // device scalar n
    int32_t *item_start;     // device array [n + 1]
    int32_t *steps;          // device array [n]: steps of this tick
};

// Kernel-family launchers (defined in kernels_*.hip).  Every launcher returns
// the hipError_t of the launch.
//   family 0: fused marching kernels; family 1: per-site generic kernels.
struct Launch {
    int kind, ndim, r, fp32;
};

// Fused marching family.  plan_* fills the decomposition for a chunk length
// and returns false when the family does not cover this (kind, ndim, r).
// tb = time steps fused per launch (1, or 2 where time_block_available).
bool time_block_available(const Launch &L);
bool plan_fused2d(const Launch &L, int64_t nx, int64_t ny, int32_t clen, int tb, int32_t *strips,
                  int32_t *ow, int32_t *chunks, int32_t *items, int32_t *blocks, int32_t *threads);
// 3D tiles hold one or two rows per wave (rpw); every 3D kernel has rpw = 2,
// some also rpw = 1 (rows_per_wave_available); rows_per_wave_default is the
// layout used until one is set or tuned.
bool rows_per_wave_available(const Launch &L, int tb, int rpw);
int rows_per_wave_default(const Launch &L, int tb);
// the layout of the batched (serving) 3D kernel of L's class: 2 or 4
int rows_per_wave_batched(const Launch &L);
// Two passes (3D Cahn-Hilliard, composed form, one step per launch, two rows
// per wave): mu goes through a field-sized buffer instead of staying in
// registers, and both passes have the halo of one radius-r stencil instead
// of two.  plan_fused3d with passes = 2 plans the tiles of both passes.
bool two_pass_available(const Launch &L);
bool plan_fused3d(const Launch &L, int64_t nx, int64_t ny, int64_t nz, int32_t clen, int tb,
                  int rpw, int passes, int32_t *strips, int32_t *ow, int32_t *ytiles,
                  int32_t *chunks, int32_t *items, int32_t *blocks, int32_t *threads);
// 1D: strips of one row, `clen` strips per wave (chunks = items = waves).
bool plan_fused1d(const Launch &L, int64_t nx, int32_t clen, int tb, int32_t *strips, int32_t *ow,
                  int32_t *chunks, int32_t *items, int32_t *blocks, int32_t *threads);
hipError_t launch_fused1d(const Launch &L, const void *args, int32_t blocks, int32_t threads,
                          int red, int tb, hipStream_t s);
hipError_t launch_fused2d(const Launch &L, const void *args, int32_t blocks, int32_t threads,
                          int red, int tb, hipStream_t s);
// 3D Cahn-Hilliard with the direct biharmonic (r <= 3): one z-marching pass
// (kernels_chd3d.hip), the 3D march with four rows per wave (rpw 4, the
// default) or one column per thread over column tiles (rpw 2);
// plan_fused3d and launch_fused3d route kCHD here.
bool chd3d_available(const Launch &L);
bool plan_chd3d(const Launch &L, int64_t nx, int64_t ny, int64_t nz, int32_t clen, int rpw,
                int32_t *strips, int32_t *ow, int32_t *ytiles, int32_t *chunks, int32_t *items,
                int32_t *blocks, int32_t *threads);
hipError_t launch_chd3d(const Launch &L, const void *args, int32_t blocks, int32_t threads, int red,
                        int rpw, hipStream_t s);
// mu: the field-sized mu buffer of a two-pass plan (same pitch and plane
// stride as the fields), nullptr for the fused single pass.
hipError_t launch_fused3d(const Launch &L, const void *args, int32_t blocks, int32_t threads,
                          int red, int tb, int rpw, void *mu, hipStream_t s);
// Batched (serving) launches: step k of the tick for every request of the
// table.  tb = 2 (where time_block_available): the launch advances requests
// with two or more steps left in the tick by a two-step sweep and those with
// one left by a single step (their plan, made for two steps, covers the
// single-step kernel); k counts steps, so the tick's launches are k = 0, 2, ..
hipError_t launch_fused2d_batched(const Launch &L, const void *table, int32_t k, int32_t blocks,
                                  int tb, hipStream_t s);
hipError_t launch_fused3d_batched(const Launch &L, const void *table, int32_t k, int32_t blocks,
                                  int tb, hipStream_t s);

// Tiny-grid serving class: the whole grid of a request in one workgroup's LDS
// (kTinyLdsBytes), all of a tick's steps of the request in one launch
// (table steps[i] of them), the result written into the other buffer of
// each field (one buffer flip per launch).  tiny_available: 2D / 3D AC, CH,
// GS, Model C with r <= 4 and nx <= 1024 whose two copies of the fields
// (plus mu or g) fit the LDS.
constexpr int kTinyLdsBytes = 128 * 1024;
bool tiny_available(const Launch &L, int64_t nx, int64_t ny, int64_t nz);
hipError_t launch_tiny(const Launch &L, const void *table, int32_t blocks, hipStream_t s);

// Many steps of one small Allen-Cahn model in one launch: 2D, r <= 2, ny a
// multiple of 16 with (ny / 16) * nx <= 1024, the grid (one copy) in
// kTinyLdsBytes of LDS; each thread holds a 16-row segment of one column in
// registers between two barriers.  On 64 or 128 columns (r <= columns / 64)
// and 64 or 128 rows one wave holds a band of whole rows instead
// (x-neighbours by lane rotation, only the bands' edge rows through LDS, one
// barrier per step).
// `args` is the
// model's StepArgs; the launch reads buf[parity] and leaves the state after
// `steps` steps in buf[parity ^ (steps & 1)].
bool lds_steps_available(const Launch &L, int64_t nx, int64_t ny, int64_t nz);
hipError_t launch_lds_steps(const Launch &L, const void *args, int32_t steps, hipStream_t s);

// Generic per-site family (any r <= kMaxR, 1D, 2D and 3D).  CH runs two
// passes through `scratch`: one field-sized buffer of T (same pitch as the
// fields), ndim of them for the direct biharmonic.
hipError_t launch_generic(const Launch &L, const void *args, void *scratch, hipStream_t s);

// Semi-implicit Fourier spectral step (Models A and B): the explicit term of
// buf[0][parity] into g (pitched like the fields), and the implicit update of
// the half spectrum uh from the explicit term's spectrum nh (written to both).
struct SpecArgs {
    void *uh;              // half spectrum of the state (u_scale uh), updated in place
    void *nh;              // half spectrum of the explicit term; receives the update too
    int64_t nxh, ny, nz;   // nx/2 + 1, ny, nz
    double sx, sy, sz;     // 2 pi / (n_a dx)
    double dt, inv_n;      // time step, 1 / (nx ny nz)
    double u_scale;        // 1 / (nx ny nz) for a fresh transform, 1 for the kept spectrum
};
hipError_t launch_spectral_nonlinear(const Launch &L, const void *args, void *g, hipStream_t s);
hipError_t launch_spectral_update(const Launch &L, const SpecArgs &a, hipStream_t s);

// Standalone reductions of the state buf[.][parity] (no step).
hipError_t launch_reduce_state(const Launch &L, const void *args, hipStream_t s);
int64_t reduce_partial_slots(int64_t nsites);

// Fixed-order compensated combination of `slots` partials per quantity into
// out[q] (double2 hi, lo), q = 0..kNumQ-1, through `part2` (kNumQ * kFinSlots
// pairs of second-level scratch).
constexpr int kFinSlots = 256;
hipError_t launch_finalize(const double2 *part, int64_t pstride, int64_t slots, double2 *part2,
                           double2 *out, hipStream_t s);

// Counter-based initial conditions.
struct InitArgs {
    void *f0, *f1;            // field buffers
    int64_t nx, ny, nz, pitch, plane;
    int32_t fp32, nfields;    // nfields: 1 or 2 (f0, f1)
    int32_t ic;               // 1 uniform, 2 GS cubes, 3 const
    uint64_t key0, key1;      // per-stream keys (SplitMix64 of seed, stream)
    double lo, span;          // x = lo + span * u01 (span = hi - lo rounded on the host)
    double v0, v1;            // const values / (cubes) outside values
    double in0, in1;          // (cubes) inside values
    int32_t ncubes, side;
    int32_t cube[64][3];      // cube corners (x, y, z)
};
hipError_t launch_init(const InitArgs &a, hipStream_t s);

// Plain streaming copy (16-byte vectors), for bandwidth calibration.
hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t s);

}  // namespace pf
