/*
 * pfmi — explicit finite-difference phase-field / reaction-diffusion steps
 * on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libpfmi.so.  Plain pointers and sizes only; no C++ exceptions
 * cross this boundary.  Every call returns a pf_status (or a plain value
 * where noted); on failure pf_last_error() gives a thread-local message.
 *
 * Method (SymPhas 2.0, arXiv 2511.10508):
 *   Model A, Allen-Cahn, Eq. (model-a):  dphi/dt = lap phi + c1 phi - c2 phi^3
 *   Model B, Cahn-Hilliard, Eq. (model-b): drho/dt = lap(-lap rho - c1 rho + c2 rho^3)
 *   Gray-Scott (named in the paper's Introduction as a reaction-diffusion
 *   model; standard two-species form):
 *       du/dt = Du lap u - u v^2 + F (1 - u)
 *       dv/dt = Dv lap v + u v^2 - (F + k) v
 * on a uniform periodic 1D, 2D or 3D grid.  lap is the star-shaped sum of 1D
 * centred second-derivative stencils of any even accuracy order p
 * (Sec. "Compile-Time Stencil Generation": weights from polynomial
 * interpolation, symmetric unknowns); the Cahn-Hilliard biharmonic is that
 * Laplacian applied twice.  Time stepping is forward Euler with every
 * right-hand side taken from the state at the start of the step.  All fields
 * stay resident on the device; data reaches the host only through
 * pf_get_field / pf_reduce (Sec. "CUDA Implementation": device residency).
 *
 * Memory layout on the device: one array per field and per ping-pong
 * buffer, x fastest, rows of `pitch` elements (pitch >= nx, a multiple of
 * 16 bytes), planes of pitch * ny elements.  Storage is FP64 or FP32.
 */
#ifndef PFMI_H
#define PFMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_ABI_VERSION 1

typedef enum {
    PF_OK = 0,
    PF_ERR_ARG = 1,          /* invalid argument or descriptor */
    PF_ERR_UNSTABLE = 2,     /* dt above the explicit-stability limit */
    PF_ERR_NOMEM = 3,        /* device or host allocation failed / over budget */
    PF_ERR_DEVICE = 4,       /* a HIP call failed */
    PF_ERR_STATE = 5,        /* call not valid in the object's current state */
    PF_ERR_UNSUPPORTED = 6,  /* combination not supported (e.g. energy of Gray-Scott) */
    PF_ERR_BUSY = 7,         /* resource busy (server queue full) */
    PF_ERR_NOTFOUND = 8      /* unknown ticket */
} pf_status;

/* Model kinds: Allen-Cahn (Eq. model-a), Cahn-Hilliard (Eq. model-b),
 * Gray-Scott, Model C (Eq. model-c), Model H (Eq. model-h). */
enum { PF_AC = 1, PF_CH = 2, PF_GS = 3, PF_MC = 4, PF_MH = 5 };
/* Storage / arithmetic precision of the bulk step. */
enum { PF_FP64 = 0, PF_FP32 = 1 };
/* Descriptor flags. */
enum {
    PF_ALLOW_UNSTABLE = 1u,    /* accept dt above the stability limit */
    PF_USE_GRAPH = 2u,         /* pf_step replays captured HIP graphs of steps */
    PF_REDUCE_EACH_STEP = 4u,  /* fuse the reductions into every step (history) */
    PF_FORCE_GENERIC = 8u,     /* use the simple per-site kernels (testing) */
    PF_BIHARMONIC_DIRECT = 16u, /* Cahn-Hilliard only: direct biharmonic stencil */
    PF_SPECTRAL = 32u           /* Allen-Cahn / Cahn-Hilliard: semi-implicit Fourier step */
};
/* Initial conditions for pf_init (counter-based SplitMix64 generator). */
enum { PF_IC_UNIFORM = 1, PF_IC_GS_CUBES = 2, PF_IC_CONST = 3 };
/* Reduction selectors for pf_reduce. */
enum { PF_RED_MASS0 = 0, PF_RED_MASS1 = 1, PF_RED_ENERGY = 2, PF_RED_NONFINITE = 3 };

/*
 * Model descriptor.  struct_size must be sizeof(pf_desc) (ABI check).
 *   kind      PF_AC, PF_CH, PF_GS, PF_MC or PF_MH
 *   nfields   1 for AC and CH, 2 for GS (u, v) and MC (phi, rho), 1 + ndim
 *             for MH (m, then the components of j); anything else ->
 *             PF_ERR_ARG
 *   ndim      1, 2 or 3; n[ndim..2] must be 1 (1D grids run their own
 *             kernels, marching along x)
 *   n         grid extents (x, y, z), each >= 1, N = n0 n1 n2 < 2^40
 *   dx        uniform spacing (> 0); dt time step (> 0)
 *   order     accuracy order p of the Laplacian stencil, even, 2..16
 *   precision PF_FP64 or PF_FP32 (FP32: storage, weights, parameters, the
 *             stencil, the nonlinear terms and the update in FP32; the
 *             reductions stay FP64 with compensation)
 *   params    AC, CH: {c1, c2};  GS: {Du, Dv, F, k};  MC: {c1, c2, c3} with
 *             phi_t = L phi + c1 phi - c2 phi^3 - 2 phi rho and
 *             rho_t = L(rho + c3 phi^2);  MH: {c1, c2, c3} with the
 *             transverse projector one: m_t = L mu - c3 div(m j), mu =
 *             c2 m^3 - c1 m - L m, j_t = L j + c3 m grad(mu) (grad and div
 *             by centred first-derivative stencils of accuracy `order`);
 *             nparams must match.  MH runs one fused pass on 1D rows
 *             (order <= 8) and on 2D and 3D grids (order <= 4), and the
 *             per-site kernels with one field-sized temporary (mu)
 *             otherwise; its
 *             reductions cover m (mass, non-finite count); the server does
 *             not take it.
 *   flags     PF_* flags above.  PF_BIHARMONIC_DIRECT (PF_CH only, else
 *             PF_ERR_ARG) replaces the Laplacian applied twice by the
 *             biharmonic's own stencil (Secs. "Advanced Derivative Support",
 *             "Compile-Time Stencil Generation": stencils of any derivative
 *             order): rho_t = L g - B rho, g = c2 rho^3 - c1 rho, B = sum over
 *             axes of the centred fourth derivative of accuracy `order`
 *             (radius order/2 + 1, pf_weights4) plus twice the products of
 *             the second-derivative stencils of each axis pair.  At order 2
 *             the two forms are the same stencil.  Not accepted by the server.
 *             PF_SPECTRAL (PF_AC or PF_CH; not with PF_BIHARMONIC_DIRECT,
 *             PF_USE_GRAPH or PF_FORCE_GENERIC, else PF_ERR_ARG; N < 2^30)
 *             replaces the finite-difference step by the semi-implicit
 *             Fourier spectral step (Sec. "Construction of Semi-Implicit
 *             Fourier Spectral Scheme"): with k the continuous wavenumbers
 *             2 pi m / (n dx) and K2 = |k|^2, AC: phi^ <- (phi^ + dt N^) /
 *             (1 + dt K2), N = c1 phi - c2 phi^3; CH: c^ <- (c^ - dt K2 g^) /
 *             (1 + dt K2^2), g = c2 c^3 - c1 c.  `order` is checked but
 *             unused.  Only the local term is explicit: pf_stability gives
 *             1/c1 (AC) or 2/c1^2 (CH), the limit of the step linearised
 *             about the separated states c^2 = c1/c2 (+inf for c1 = 0).  The
 *             mass reductions apply, the free energy is PF_ERR_UNSUPPORTED.
 *             The model holds two half spectra besides its fields (hipFFT
 *             plans allocate their own work space) and keeps the updated
 *             spectrum between steps, so a run of steps takes two transforms
 *             per step; after pf_init, pf_set_field or pf_field_device the
 *             next step transforms the state again.  Not accepted by the server.
 */
typedef struct pf_desc {
    uint32_t struct_size;
    int32_t kind;
    int32_t nfields;
    int32_t ndim;
    int64_t n[3];
    double dx;
    double dt;
    int32_t order;
    int32_t precision;
    int32_t nparams;
    uint32_t flags;
    double params[8];
} pf_desc;

typedef struct pf_model pf_model;

/* Library information. */
int32_t pf_abi_version(void);
const char *pf_last_error(void);            /* thread-local, never NULL */
const char *pf_status_str(pf_status s);

/*
 * Host FP64 stencil weights: the centred second-derivative weights
 * w[0..order/2] (w_{-j} = w_j) for accuracy `order`, computed by Fornberg's
 * recursion (Math. Comp. 51, 1988) on the nodes 0, +-1, .., +-r at unit
 * spacing.  `w` must hold order/2 + 1 doubles (caller-owned).
 */
pf_status pf_weights(int32_t order, double *w);

/*
 * Host FP64 centred fourth-derivative weights w4[0..order/2 + 1] (w4_{-j} =
 * w4_j) of accuracy `order` (the direct biharmonic's axis stencil), by the
 * same recursion on the nodes 0, +-1, .., +-(order/2 + 1).  `w4` must hold
 * order/2 + 2 doubles (caller-owned).  PF_ERR_ARG for a bad order or NULL.
 */
pf_status pf_weights4(int32_t order, double *w4);

/*
 * Host FP64 centred first-derivative weights w1[0..order/2] (w1_{-j} =
 * -w1_j, w1[0] = 0) of accuracy `order` (Model H's gradient and divergence),
 * by the same recursion.  `w1` must hold order/2 + 1 doubles (caller-owned).
 * PF_ERR_ARG for a bad order or NULL.
 */
pf_status pf_weights1(int32_t order, double *w1);

/*
 * Explicit-stability limit of the descriptor's model: the largest dt for
 * which the linearised forward-Euler step keeps every Fourier mode bounded
 * (Nyquist-mode symbol of the stencil; AC linearised for phi^2 <= c1/c2,
 * CH for rho^2 <= c1/c2, GS for u, v in [0, 1]).
 */
pf_status pf_stability(const pf_desc *desc, double *dt_max);

/* Device bytes a model of this descriptor holds (2 buffers per field, padded
 * pitch, plus reduction scratch, plus the field-sized temporaries of the
 * per-site kernels where the fused ones do not apply: one for Cahn-Hilliard
 * and Model H, ndim for the direct biharmonic).  A 3D Cahn-Hilliard model
 * switched to two passes (pf_set_passes, or the autotuner's choice) holds
 * one field more.  0 for an invalid descriptor. */
uint64_t pf_footprint_bytes(const pf_desc *desc);

/* Elements of one device field buffer (pitch * n1 * n2).  -1 if invalid. */
int64_t pf_buffer_elems(const pf_desc *desc);

/*
 * Create a model.  The library allocates and owns 2 * nfields device
 * buffers (ping-pong) plus reduction scratch; fields start at zero.
 * hip_stream: a hipStream_t owned by the caller, or NULL for a stream owned
 * by the model.  Errors: PF_ERR_ARG (bad descriptor), PF_ERR_UNSTABLE (dt >
 * dt_max without PF_ALLOW_UNSTABLE), PF_ERR_NOMEM, PF_ERR_DEVICE.
 */
pf_status pf_create(const pf_desc *desc, void *hip_stream, pf_model **out);

/*
 * Create a model on caller-owned device memory (e.g. torch tensors):
 * dev_bufs holds nbufs = 2 * nfields pointers, in the order field 0 buffer
 * A, field 0 buffer B, field 1 buffer A, field 1 buffer B; each of
 * pf_buffer_elems(desc) elements of the storage type, 16-byte aligned.  The
 * caller keeps them alive until pf_destroy; the library never frees them.
 */
pf_status pf_create_on(const pf_desc *desc, void *hip_stream, void *const *dev_bufs,
                       int32_t nbufs, pf_model **out);

/* Release the model (syncs its stream first).  NULL is a no-op. */
void pf_destroy(pf_model *m);

/*
 * Initialise the fields on the device from the counter-based generator:
 * every value is a pure function of (seed, stream, site index), site index
 * x + n0 (y + n1 z), so any sub-window can be reproduced on the host.
 *   PF_IC_UNIFORM  ic_params {lo, hi}: field f = lo + (hi - lo) U_f
 *   PF_IC_GS_CUBES ic_params {ncubes, side, noise}: u = 1, v = 0 except
 *                  ncubes cubes (periodic) with u = 0.5, v = 0.25, then
 *                  U[-noise, noise] added to u and v
 *   PF_IC_CONST    ic_params {value_0, value_1}
 * Asynchronous on the model's stream.  Resets pf_steps_done to 0.
 */
pf_status pf_init(pf_model *m, int32_t ic, uint64_t seed, const double *ic_params,
                  int32_t n_ic_params);

/* Copy a field between host FP64 memory (count = N doubles, x fastest,
 * caller-owned, used only during the call) and the device.  FP32 storage
 * rounds to nearest on set and widens exactly on get.  Both synchronise the
 * model's stream.  count != N -> PF_ERR_ARG. */
pf_status pf_set_field(pf_model *m, int32_t field, const double *host, int64_t count);
pf_status pf_get_field(pf_model *m, int32_t field, double *host, int64_t count);

/* Copy a box of a field to host FP64 memory: origin (x, y, z) (periodic,
 * wrapped) and extent w (wx, wy, wz); host holds wx*wy*wz doubles, x
 * fastest.  Synchronises the model's stream. */
pf_status pf_get_window(pf_model *m, int32_t field, const int64_t *origin, const int64_t *w,
                        double *host);

/* Zero-copy view of the current buffer of a field; valid until the next
 * pf_step / pf_init / pf_destroy. */
pf_status pf_field_device(pf_model *m, int32_t field, void **ptr, int64_t *pitch_elems,
                          int32_t *elem_bytes);

/*
 * Enqueue nsteps forward-Euler steps on the model's stream and return
 * (asynchronous).  With PF_REDUCE_EACH_STEP the reductions of the state at
 * the start of every step are fused into the step kernel and kept in a
 * device history (pf_reduce_history).  With PF_USE_GRAPH the launches are
 * replayed from captured HIP graphs.  A small 2D Allen-Cahn model (order <=
 * 4, ny a multiple of 16 with (ny / 16) * nx <= 1024, one copy of the grid
 * within 128 KiB) stepped without PF_REDUCE_EACH_STEP or kernel timing runs
 * up to 4096 steps per launch in one workgroup's LDS; the fields are bitwise
 * the same.
 */
pf_status pf_step(pf_model *m, int64_t nsteps);

/*
 * Allocation-free step, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Runs nsteps steps of the descriptor's model on caller-owned
 * buffers in the layout of pf_create_on (2 * nfields buffers of
 * pf_buffer_elems(desc) elements, 16-byte aligned; dev_bufs[2 f + p] is
 * buffer p of field f), starting from buffer `parity` (0 or 1) of every
 * field; the result is in buffer parity ^ (nsteps & 1).  The kernels and
 * their plan are those of a pf_create_on model with pf_set_tile(m, 0), one
 * step per launch and the default 3D tile layout, so fields and reductions
 * are bitwise that model's.  With PF_REDUCE_EACH_STEP, dev_history
 * (caller-owned device memory of 6 * nsteps doubles) receives for step k the
 * reductions of the state at its start as three (hi, lo) pairs: the sum of
 * field 0, the sum of field 1 (GS, MC) or of the energy density (AC, CH),
 * and the non-finite count (hi), not multiplied by dx^ndim; without it
 * dev_history may be NULL.  Enqueues on hip_stream (NULL = the null stream)
 * of the current device and returns; no allocation.  The reduction partials
 * live in one static 16 MiB device array per GPU, shared by every call on
 * that GPU and keeping the last call's contents: calls that overlap on one
 * GPU (other streams or threads) race and must be serialised by the caller.
 * Errors, before anything is enqueued: PF_ERR_ARG (bad descriptor or
 * arguments; PF_SPECTRAL, PF_FORCE_GENERIC or PF_USE_GRAPH; a grid whose
 * partials need more than the 16 MiB), PF_ERR_UNSTABLE, PF_ERR_UNSUPPORTED
 * (descriptors that need the per-site kernels and their field-sized
 * temporary), PF_ERR_DEVICE.
 */
pf_status pf_step_noalloc(const pf_desc *desc, void *hip_stream, void *const *dev_bufs,
                          int32_t nbufs, int32_t parity, int64_t nsteps, double *dev_history);

/*
 * Reductions of the current state, compensated in FP64 on the device and
 * combined in a fixed order: value = hi + lo (double-double).
 *   PF_RED_MASS0 / PF_RED_MASS1: dx^d sum of field 0 / 1 (MASS1: GS and MC
 *                  only, else PF_ERR_UNSUPPORTED)
 *   PF_RED_ENERGY: dx^d sum of -(1/2) x L x + (c2/4) x^4 - (c1/2) x^2 (AC, CH
 *                  only, with the Laplacian of the descriptor's order, also
 *                  for the direct biharmonic; GS, MC, MH and PF_SPECTRAL ->
 *                  PF_ERR_UNSUPPORTED)
 *   PF_RED_NONFINITE: number of NaN / Inf values (hi = count, lo = 0) of the
 *                  reduced fields (MH: m only)
 * Synchronises the stream.
 */
pf_status pf_reduce(pf_model *m, int32_t which, double *hi, double *lo);

/* Per-step reductions recorded by the last pf_step under PF_REDUCE_EACH_STEP:
 * entry k is the state at the start of step k of that call.  hi/lo hold
 * `count` doubles each (caller-owned); count must not exceed that call's
 * nsteps.  Synchronises the stream. */
pf_status pf_reduce_history(pf_model *m, int32_t which, double *hi, double *lo, int64_t count);

/* Wait for all work enqueued on the model's stream. */
pf_status pf_sync(pf_model *m);

/* Steps advanced since creation or the last pf_init / pf_set_steps_done. */
int64_t pf_steps_done(const pf_model *m);
pf_status pf_set_steps_done(pf_model *m, int64_t steps);

/* The hipStream_t the model enqueues on. */
pf_status pf_stream(pf_model *m, void **hip_stream);

/*
 * Tile shape of the step kernels: chunk = sites marched per work item along
 * the slowest axis (y in 2D, z in 3D), 0 = the library's choice.  Fields
 * do not depend on it (bitwise); fused reductions agree to their compensated
 * accuracy (the partition into partial sums changes).  pf_get_tile reports the current one and
 * the kernel family in use (0 fused marching, 1 per-site generic).
 */
pf_status pf_set_tile(pf_model *m, int32_t chunk);
pf_status pf_get_tile(pf_model *m, int32_t *chunk, int32_t *family);

/*
 * Temporal blocking: tb = 2 fuses two time steps into one sweep over the
 * fields (the intermediate state stays in registers), halving HBM traffic per
 * step; available on the fused kernels for 2D grids with order 2 or 4 and
 * 3D grids with order 2 (otherwise PF_ERR_UNSUPPORTED).  Results are bitwise those of tb = 1.  An
 * odd remainder of a pf_step call runs one single step.
 */
pf_status pf_set_time_block(pf_model *m, int32_t tb);
int32_t pf_get_time_block(const pf_model *m);

/*
 * 3D tile layout of the fused kernels: rows = tile rows held by each wave.
 * 2: each wave holds two rows of 32 lanes (32-row tiles, 512-byte row
 * segments; built for every 3D kernel).  1: one row of 64 lanes (16-row
 * tiles, 1 KiB segments; built for FP64 Allen-Cahn with order <= 4 and
 * FP64 Gray-Scott with order 2, where it is the default).  4: four rows of
 * 16 lanes (32-row tiles of 8 waves, two workgroups per CU, or one with up
 * to 256 registers a lane; 48-row tiles of 12 waves for Cahn-Hilliard with
 * order 6 and the direct biharmonic with order 2; built for Cahn-Hilliard,
 * Model C, Gray-Scott with order >= 4, Allen-Cahn with order 8 and the
 * direct biharmonic; the default for Gray-Scott and Model C with order >= 6,
 * FP32 Cahn-Hilliard with order 6 and the direct biharmonic).  The direct
 * biharmonic has one other 3D layout, 2: one thread per column of an x-y
 * tile (plus its halo) marching along z.  0 restores the default.  Fields
 * are bitwise independent of it.  PF_ERR_UNSUPPORTED for a 2D model, the
 * per-site family, or a layout not built for this model.  pf_get_tile_rows
 * returns the layout in use (0 for 2D models and the per-site family, -1 for
 * NULL).
 */
pf_status pf_set_tile_rows(pf_model *m, int32_t rows);
int32_t pf_get_tile_rows(const pf_model *m);

/*
 * Passes of a 3D Cahn-Hilliard step (composed form, order <= 6) on the fused
 * kernels.  1 (default): mu = f'(c) - L c stays in registers and LDS, and
 * the update is the second of two chained radius-r stencils in the same
 * sweep (halo 2r).  2: a first pass writes mu into a field-sized buffer (the
 * model allocates it, one more field of HBM) and reduces c, a second reads
 * mu and c and writes the stepped c; each pass has the halo of one stencil
 * and a single register ring, at the price of writing and reading mu and
 * reading c twice (the three-array layout of the paper, Sec. Benchmarks,
 * memory-footprint table).  Fields are bitwise those of one pass; fused
 * reductions agree to their compensated accuracy.  Two passes run one step
 * per launch (pf_set_time_block(m, 2) is then PF_ERR_UNSUPPORTED).
 * PF_ERR_UNSUPPORTED for other models, orders, the per-site or spectral
 * family.  pf_get_passes returns the passes in use (0 outside the fused
 * family, -1 for NULL).  Until set, one pass; the autotuner considers both.
 */
pf_status pf_set_passes(pf_model *m, int32_t passes);
int32_t pf_get_passes(const pf_model *m);

/*
 * Autotuner: times each candidate (chunk length, time-block factor, 3D tile
 * layout, passes of a 3D Cahn-Hilliard step) on the model's own buffers by re-running steps from the current
 * state (whose buffer is never written, so the state is unchanged), keeps the
 * fastest per step and records it in an in-process cache keyed by (kind,
 * ndim, order, precision, per-step reductions, size class) that later models
 * of the same class reuse.
 * trials = timed launches per candidate (<= 0: 3); where they take less
 * than 2 ms, the candidate is timed again with as many launches as fill
 * 2 ms (at most 64).
 */
pf_status pf_autotune(pf_model *m, int32_t trials);

/*
 * Kernel timing on the model's stream: while enabled, pf_step records a HIP
 * event pair around every step-kernel launch (graph replay and the
 * whole-grid LDS launches of small models are off);
 * pf_timing_read synchronises and returns the summed kernel milliseconds,
 * the number of launches and the number of time steps they advanced since
 * the last enable (any output pointer may be NULL).
 */
pf_status pf_timing_enable(pf_model *m, int32_t on);
pf_status pf_timing_read(pf_model *m, double *total_ms, int64_t *launches, int64_t *steps);

/*
 * Measurement helper: stream `bytes` from src to dst (device pointers,
 * 16-byte aligned, bytes a multiple of 16) with the library's plain copy
 * kernel on hip_stream (NULL = the null stream) and return the kernel time
 * in milliseconds measured with HIP events (synchronises).  Calibrates
 * attainable HBM bandwidth and hardware byte counters.
 */
pf_status pf_copy_probe(void *dst, const void *src, uint64_t bytes, void *hip_stream,
                        int32_t reps, double *ms_per_rep);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent simulation requests.
 *
 * A server owns one device and a stream.  Requests (a descriptor, an initial
 * condition and a step count) are admitted while their footprint fits the
 * HBM budget and a slot is free; every scheduler tick runs a block of steps
 * for all admitted requests in batched launches (one per kernel class and
 * step) replayed from a captured HIP graph.  Requests that arrive while
 * others run are admitted at the next tick.  Each request's result is
 * bitwise the same as a model stepped alone with the same tile.
 * ---------------------------------------------------------------------- */
typedef struct pf_server pf_server;

typedef struct pf_result {
    uint64_t ticket;
    int32_t status;          /* PF_OK, or the request's failure */
    int32_t _pad;
    double t_submit;         /* seconds on the server's monotonic clock */
    double t_admit;
    double t_done;           /* device completion observed by the scheduler */
    double mass[2];          /* reductions of the final state (hi + lo folded) */
    double energy;           /* AC / CH */
    int64_t nonfinite;
    int64_t steps_done;
} pf_result;

/*
 * hbm_budget: bytes of device memory the server may hold for requests
 * (0 = 90 % of free memory at creation); max_slots: most requests resident
 * at once, running or finished and not yet released (a finished request keeps
 * its memory and slot until pf_server_release); steps_per_tick: steps per
 * request per tick (0 = 64).  Served requests run the batched kernels with
 * two steps per launch where their class has a two-step kernel (2D orders 2
 * and 4, 3D order 2), and the chunk length the server's autotuner picks per
 * kernel class and size bucket on the first request of each bucket.
 * Requests whose grid fits one workgroup's LDS (2D or 3D Allen-Cahn,
 * Cahn-Hilliard, Gray-Scott or Model C, order <= 8, x extent <= 1024, both
 * copies of the fields plus mu or g within 128 KiB) form a tiny class: one
 * workgroup per request keeps the whole grid in LDS and runs up to
 * 16 x steps_per_tick of its steps per tick, touching HBM once per tick.
 * Environment: PFMI_SERVER_MAX_GRAPHS bounds the cache of captured tick
 * graphs (default 256); PFMI_SERVER_TWO_STEP=0 keeps one step per launch;
 * PFMI_SERVER_TUNE=off keeps the library's default chunk.
 */
pf_status pf_server_create(int32_t device, uint64_t hbm_budget, int32_t max_slots,
                           int32_t steps_per_tick, pf_server **out);

/* Thread-safe, non-blocking.  Footprint above the budget -> PF_ERR_NOMEM;
 * an invalid or unstable descriptor -> PF_ERR_ARG / PF_ERR_UNSTABLE; a 1D
 * grid or PF_BIHARMONIC_DIRECT -> PF_ERR_UNSUPPORTED (served requests run the
 * batched 2D and 3D kernels). */
pf_status pf_server_submit(pf_server *s, const pf_desc *desc, int32_t ic, uint64_t seed,
                           const double *ic_params, int32_t n_ic_params, int64_t nsteps,
                           uint64_t *ticket);

/* Up to max finished requests not yet reported (non-blocking). */
pf_status pf_server_poll(pf_server *s, pf_result *out, int32_t max, int32_t *n);

/* Copy a finished request's field to host FP64 memory (count = N). */
pf_status pf_server_fetch(pf_server *s, uint64_t ticket, int32_t field, double *host,
                          int64_t count);

/* Free a finished request's device memory and slot. */
pf_status pf_server_release(pf_server *s, uint64_t ticket);

/* Cancel a queued or running request (it finishes with PF_ERR_STATE). */
pf_status pf_server_cancel(pf_server *s, uint64_t ticket);

/* Block until every submitted request has finished or timeout_s passed
 * (PF_ERR_BUSY on timeout). */
pf_status pf_server_drain(pf_server *s, double timeout_s);

/* Server statistics: ticks run, batched launches, graph captures, graph replays. */
pf_status pf_server_stats(pf_server *s, int64_t *ticks, int64_t *launches, int64_t *captures,
                          int64_t *replays);

/* Stop the scheduler and free everything (pending requests are dropped). */
void pf_server_destroy(pf_server *s);

#ifdef __cplusplus
}
#endif
#endif /* PFMI_H */
