// Host runtime and C ABI of libpfmi: model objects, device buffers, the step
// loop (eager or replayed HIP graphs), reductions, initial conditions,
// kernel timing and the tile autotuner.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pfmi.h"
#include "pf_internal.h"
#include "pf_runtime.h"

namespace pf {

bool centered_d2_weights(int order, double *w);
bool centered_d4_weights(int order, double *w4);
bool centered_d1_weights(int order, double *w1);

static thread_local std::string g_err;

pf_status fail(pf_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

pf_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return PF_ERR_DEVICE;
}

#define PF_HIP(call, what)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, what);    \
    } while (0)

// ------------------------------------------------------------------ desc --
int nfields_of(int kind) { return nfields_kind(kind); }

pf_status check_desc(const pf_desc *d)
{
    if (!d) return fail(PF_ERR_ARG, "descriptor is NULL");
    if (d->struct_size != sizeof(pf_desc))
        return fail(PF_ERR_ARG, "pf_desc.struct_size does not match this library");
    if (d->kind != kAC && d->kind != kCH && d->kind != kGS && d->kind != kMC && d->kind != kMH)
        return fail(PF_ERR_ARG, "unknown model kind");
    const int nf = d->kind == kMH ? 1 + d->ndim : nfields_of(d->kind);
    if (d->nfields != nf)
        return fail(PF_ERR_ARG, "nfields does not match the model (AC, CH: 1; GS, MC: 2; MH: 1 + ndim)");
    if (d->ndim < 1 || d->ndim > 3) return fail(PF_ERR_ARG, "ndim must be 1, 2 or 3");
    for (int a = 0; a < 3; ++a)
        if (d->n[a] < 1) return fail(PF_ERR_ARG, "grid extents must be >= 1");
    if (d->ndim <= 2 && d->n[2] != 1) return fail(PF_ERR_ARG, "1D and 2D grids need n[2] == 1");
    if (d->ndim == 1 && d->n[1] != 1) return fail(PF_ERR_ARG, "1D grids need n[1] == 1");
    const double N = (double)d->n[0] * (double)d->n[1] * (double)d->n[2];
    if (N > (double)(1ll << 40)) return fail(PF_ERR_ARG, "grid too large");
    if (d->n[0] > (1ll << 30) || d->n[1] > (1ll << 30) || d->n[2] > (1ll << 30))
        return fail(PF_ERR_ARG, "grid extent too large");
    if (!(d->dx > 0.0) || !std::isfinite(d->dx)) return fail(PF_ERR_ARG, "dx must be > 0");
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(PF_ERR_ARG, "dt must be > 0");
    if (d->order < 2 || d->order > 16 || d->order % 2)
        return fail(PF_ERR_ARG, "order must be even, 2..16");
    if (d->precision != PF_FP64 && d->precision != PF_FP32)
        return fail(PF_ERR_ARG, "precision must be PF_FP64 or PF_FP32");
    const int np = d->kind == kGS ? 4 : (d->kind == kMC || d->kind == kMH) ? 3 : 2;
    if (d->nparams != np) return fail(PF_ERR_ARG, "nparams must be 2 (AC, CH), 4 (GS) or 3 (MC, MH)");
    for (int i = 0; i < np; ++i)
        if (!std::isfinite(d->params[i])) return fail(PF_ERR_ARG, "parameters must be finite");
    if ((d->flags & PF_BIHARMONIC_DIRECT) && d->kind != kCH)
        return fail(PF_ERR_ARG, "PF_BIHARMONIC_DIRECT applies to Cahn-Hilliard only");
    if (d->flags & PF_SPECTRAL) {
        if (d->kind != kAC && d->kind != kCH)
            return fail(PF_ERR_ARG, "PF_SPECTRAL applies to Allen-Cahn and Cahn-Hilliard only");
        if (d->flags & (PF_BIHARMONIC_DIRECT | PF_USE_GRAPH | PF_FORCE_GENERIC))
            return fail(PF_ERR_ARG, "PF_SPECTRAL takes no PF_BIHARMONIC_DIRECT, PF_USE_GRAPH "
                                    "or PF_FORCE_GENERIC");
        if (d->n[0] > (1 << 30) / std::max<int64_t>(1, d->n[1] * d->n[2]))
            return fail(PF_ERR_ARG, "PF_SPECTRAL grids must hold fewer than 2^30 sites");
    }
    if (d->kind == kGS)
        for (int i = 0; i < np; ++i)
            if (d->params[i] < 0.0) return fail(PF_ERR_ARG, "Gray-Scott parameters must be >= 0");
    return PF_OK;
}

double stability_limit(const pf_desc *d)
{
    // spectral scheme: the Laplacian terms are implicit and only the local
    // term is explicit; linearised about the separated states (u^2 = c1/c2,
    // explicit slope -2 c1 for AC, +2 c1 for CH) every mode stays bounded for
    // dt <= 1/c1 (AC) and dt <= 2/c1^2 (CH); c1 = 0 leaves no limit
    if (d->flags & PF_SPECTRAL) {
        const double c1 = std::fabs(d->params[0]);
        if (c1 == 0.0) return HUGE_VAL;
        return d->kind == kAC ? 1.0 / c1 : 2.0 / (c1 * c1);
    }
    double w[kMaxR + 1];
    centered_d2_weights(d->order, w);
    double sigma = w[0];
    for (int j = 1; j <= d->order / 2; ++j) sigma += 2.0 * w[j] * ((j & 1) ? -1.0 : 1.0);
    const double lam = std::fabs(sigma) * d->ndim / (d->dx * d->dx);
    double rho;
    if (d->kind == kAC || d->kind == kMC)  // MC: phi as AC about small fields, rho diffuses
        rho = lam + 2.0 * std::fabs(d->params[0]);
    else if (d->kind == kMH)  // m as CH, each j_a diffuses; couplings are higher order
        rho = std::max(lam * lam + 2.0 * std::fabs(d->params[0]) * lam, lam);
    else if (d->kind == kCH && (d->flags & PF_BIHARMONIC_DIRECT)) {
        // Nyquist symbol of the direct operator: ndim tau / dx^4 for the
        // fourth derivatives, ndim (ndim - 1) (sigma / dx^2)^2 for the mixed
        // products (tau: the fourth-derivative stencil at the Nyquist mode)
        double w4[kMaxR + 2];
        centered_d4_weights(d->order, w4);
        double tau = w4[0];
        for (int j = 1; j <= d->order / 2 + 1; ++j) tau += 2.0 * w4[j] * ((j & 1) ? -1.0 : 1.0);
        const double s1 = std::fabs(sigma) / (d->dx * d->dx);
        const double beta = d->ndim * std::fabs(tau) / (d->dx * d->dx * d->dx * d->dx) +
                            d->ndim * (d->ndim - 1) * s1 * s1;
        rho = beta + 2.0 * std::fabs(d->params[0]) * lam;
    } else if (d->kind == kCH)
        rho = lam * lam + 2.0 * std::fabs(d->params[0]) * lam;
    else
        rho = std::max(d->params[0], d->params[1]) * lam + d->params[2] + d->params[3] + 1.0;
    return 2.0 / rho;
}

// Row pitch: nx rounded up to 16 bytes, plus a padding for rows of 4 KiB or
// more so that consecutive rows do not start at the same large power-of-two
// offset.  PFMI_PITCH_PAD_BYTES overrides the padding (tuning knob).
int64_t pitch_of(const pf_desc *d)
{
    const int64_t eb = d->precision == PF_FP32 ? 4 : 8;
    const int64_t v = 16 / eb;
    int64_t p = (d->n[0] + v - 1) / v * v;
    int64_t pad = kDefaultPitchPadBytes;
    if (const char *env = std::getenv("PFMI_PITCH_PAD_BYTES")) pad = std::atoll(env);
    if (p * eb >= 4096 && pad > 0) p += (pad / eb + v - 1) / v * v;
    return p;
}

int64_t buffer_elems(const pf_desc *d) { return pitch_of(d) * d->n[1] * d->n[2]; }

int elem_bytes(const pf_desc *d) { return d->precision == PF_FP32 ? 4 : 8; }

// ------------------------------------------------------------ SplitMix64 --
static uint64_t mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static const uint64_t kGolden = 0x9E3779B97F4A7C15ull;
static uint64_t stream_key(uint64_t seed, uint64_t stream) { return mix64(seed + (stream + 1) * kGolden); }
static double u01_host(uint64_t key, uint64_t idx)
{
    return (double)(mix64(key + (idx + 1) * kGolden) >> 11) * 0x1.0p-53;
}

// ----------------------------------------------------------------- model --
Model::~Model() {}

static size_t tsize(const Model *m) { return m->fp32 ? 4 : 8; }

template <typename T>
static void fill_args(Model *m, StepArgs<T> &a)
{
    const pf_desc &d = m->desc;
    std::memset(&a, 0, sizeof(a));
    for (int f = 0; f < kMaxFields; ++f)
        for (int p = 0; p < 2; ++p)
            a.buf[f][p] = static_cast<T *>(m->buf[f < m->nf ? f : 0][p]);
    a.nx = d.n[0];
    a.ny = d.n[1];
    a.nz = d.n[2];
    a.pitch = m->pitch;
    a.plane = m->pitch * d.n[1];
    const int r = d.order / 2;
    double w[kMaxR + 1];
    centered_d2_weights(d.order, w);
    const double idx2 = 1.0 / (d.dx * d.dx);
    a.w64sum = 0.0;
    for (int j = 1; j <= r; ++j) {
        const double wl = w[j] * idx2;
        a.w64[j - 1] = wl;
        a.w64sum += wl;
        a.wi[j - 1] = (T)wl;
        if (d.kind == kGS) {
            a.wu[j - 1] = (T)(d.dt * d.params[0] * wl);
            a.wv[j - 1] = (T)(d.dt * d.params[1] * wl);
        } else if (d.kind == kMC) {
            a.wu[j - 1] = (T)(d.dt * wl);
            a.wv[j - 1] = (T)(d.dt * wl);
        } else {
            a.wu[j - 1] = (T)(d.dt * wl);
        }
    }
    if (d.kind == kMH) {
        double w1[kMaxR + 1];
        centered_d1_weights(d.order, w1);
        for (int j = 1; j <= r; ++j) a.w1[j - 1] = (T)(w1[j] / d.dx);
    }
    if (m->L.kind == kCHD) {
        double w4[kMaxR + 2];
        centered_d4_weights(d.order, w4);
        const double idx4 = idx2 * idx2;
        for (int j = 1; j <= r + 1; ++j) a.w4[j - 1] = (T)(-d.dt * w4[j] * idx4);
    }
    if (d.kind == kAC) {
        a.k0 = (T)(d.dt * d.params[0]);
        a.k1 = (T)(d.dt * d.params[1]);
    } else if (d.kind == kCH || d.kind == kMH) {
        a.k0 = (T)d.params[0];
        a.k1 = (T)d.params[1];
        a.k2 = (T)(d.dt * (d.kind == kMH ? d.params[2] : 0.0));
    } else if (d.kind == kMC) {
        a.k0 = (T)(d.dt * d.params[0]);
        a.k1 = (T)(d.dt * d.params[1]);
        a.k2 = (T)(2.0 * d.dt);
        a.k3 = (T)d.params[2];
    } else {
        a.k0 = (T)(d.dt * d.params[2]);
        a.k1 = (T)(d.dt * (d.params[2] + d.params[3]));
        a.k2 = (T)d.dt;
    }
    a.c1 = (d.kind == kAC || d.kind == kCH) ? d.params[0] : 0.0;
    a.c2 = (d.kind == kAC || d.kind == kCH) ? d.params[1] : 0.0;
    a.part = m->part;
    a.pstride = m->pstride;
}

// Plan the fused decomposition for the model's chunk length.
static bool plan(Model *m)
{
    Launch L = m->L;
    const pf_desc &d = m->desc;
    m->family = 1;
    m->lds_steps = false;
    if (d.flags & PF_SPECTRAL) {
        m->family = 2;
        m->tb = 1;
        return true;
    }
    if (!time_block_available(L)) m->tb = 1;
    if (d.flags & PF_FORCE_GENERIC) {
        m->tb = 1;
        return true;
    }
    int32_t strips, ow, ytiles = 1, chunks, items, blocks, threads;
    bool ok;
    if (d.ndim == 1)
        ok = plan_fused1d(L, d.n[0], m->clen, m->tb, &strips, &ow, &chunks, &items, &blocks,
                          &threads);
    else if (d.ndim == 2)
        ok = plan_fused2d(L, d.n[0], d.n[1], m->clen, m->tb, &strips, &ow, &chunks, &items,
                          &blocks, &threads);
    else {
        m->passes = m->passes_req == 2 && two_pass_available(L) ? 2 : 1;
        if (m->passes == 2) {
            m->tb = 1;
            m->rpw = 2;
        } else {
            m->rpw = m->rpw_req && rows_per_wave_available(L, m->tb, m->rpw_req)
                         ? m->rpw_req
                         : rows_per_wave_default(L, m->tb);
        }
        ok = plan_fused3d(L, d.n[0], d.n[1], d.n[2], m->clen, m->tb, m->rpw, m->passes, &strips,
                          &ow, &ytiles, &chunks, &items, &blocks, &threads);
    }
    if (!ok) {
        m->tb = 1;
        m->passes = 1;
        return true;
    }
    m->family = 0;
    m->lds_steps = lds_steps_available(L, d.n[0], d.n[1], d.n[2]);
    m->strips = strips;
    m->ow = ow;
    m->ytiles = ytiles;
    m->chunks = chunks;
    m->items = items;
    m->blocks = blocks;
    m->threads = threads;
    m->fused_slots = d.ndim == 3 ? (int64_t)items * kWaves3D : (int64_t)items;
    return true;
}

// Default chunk length along the marching axis: long enough to amortise the
// 2H warm-up rows, short enough that small grids still expose thousands of
// work items (about 4096 waves in 2D, 1024 workgroups in 3D, whose tiles
// are half as wide as a 2D strip and 32 rows high).
int32_t default_chunk(const pf_desc *d)
{
    if (d->ndim == 1) {
        // strips per wave: about 8192 waves (8 per SIMD)
        const int64_t strips = std::max<int64_t>(1, d->n[0] / (d->precision == PF_FP32 ? 224 : 112));
        return (int32_t)std::max<int64_t>(1, std::min<int64_t>(256, strips / 8192));
    }
    const int64_t march = d->ndim == 2 ? d->n[1] : d->n[2];
    const int64_t cols = (d->precision == PF_FP32 ? 256 : 128) / (d->ndim == 2 ? 1 : 2);
    const int64_t strips = std::max<int64_t>(1, (d->n[0] + cols - 1) / cols);
    const int64_t cmin = 8;
    int64_t cmax, c;
    if (d->ndim == 2) {
        cmax = 512;
        c = march * strips / 4096;
    } else {
        cmax = 64;
        const int64_t ytiles = std::max<int64_t>(1, (d->n[1] + 23) / 24);
        c = march * strips * ytiles / 1024;
    }
    c = std::max(cmin, std::min(cmax, c));
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(c, march));
}

// Tuned decompositions, keyed by model, order, precision, whether reductions
// ride on every step, and the log2 of each extent.
struct TuneChoice {
    int32_t chunk;
    int tb, rpw, passes;
};
using TuneKey = std::tuple<int, int, int, int, int, int, int, int>;
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneChoice> g_tune_cache;

static TuneKey tune_key(const pf_desc &d)
{
    auto lg = [](int64_t v) { int b = 0; while ((1ll << (b + 1)) <= v) ++b; return b; };
    return std::make_tuple(d.kind, d.ndim, d.order, d.precision,
                           (int)(d.flags & (PF_REDUCE_EACH_STEP | PF_BIHARMONIC_DIRECT)),
                           lg(d.n[0]), lg(d.n[1]),
                           lg(d.n[2]));
}

static hipError_t dev_alloc(Model *m, void **p, size_t bytes)
{
    return m->async_alloc ? hipMallocAsync(p, bytes, m->stream) : hipMalloc(p, bytes);
}

static void dev_free(Model *m, void *p)
{
    if (!p) return;
    if (m->async_alloc)
        (void)hipFreeAsync(p, m->stream);
    else
        (void)hipFree(p);
}

static pf_status ensure_partials(Model *m)
{
    const int64_t N = m->desc.n[0] * m->desc.n[1] * m->desc.n[2];
    int64_t need = std::max<int64_t>(reduce_partial_slots(N), m->family == 0 ? m->tb * m->fused_slots : 0);
    need = std::max<int64_t>(need, 1);
    if (need <= m->pstride && m->part) return PF_OK;
    if (m->part) {
        if (!m->async_alloc) PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
        dev_free(m, m->part);
        m->part = nullptr;
    }
    PF_HIP(dev_alloc(m, (void **)&m->part, sizeof(double2) * kNumQ * need), "hipMalloc(partials)");
    m->pstride = need;
    return PF_OK;
}

// Cache the launch arguments of the model's current plan.
static void refresh_args(Model *m)
{
    auto setp = [&](auto &a) {
        a.strips = m->strips;
        a.ow = m->ow;
        a.ytiles = m->ytiles;
        a.chunks = m->chunks;
        a.clen = m->clen;
        a.items = m->items;
    };
    if (m->fp32) {
        fill_args<float>(m, m->a32);
        setp(m->a32);
    } else {
        fill_args<double>(m, m->a64);
        setp(m->a64);
    }
}

// Field-sized mu buffer(s): the per-site family's CH, direct-biharmonic and
// Model H temporaries, or the mu buffer of a two-pass fused plan.
static pf_status ensure_scratch(Model *m)
{
    const bool need = m->family == 0 ? m->passes == 2
                                     : (m->L.kind == kCH || m->L.kind == kCHD || m->L.kind == kMH);
    if (!need || m->scratch) return PF_OK;
    const size_t nbuf = m->L.kind == kCHD ? (size_t)m->desc.ndim : 1;
    PF_HIP(dev_alloc(m, &m->scratch, nbuf * tsize(m) * (size_t)m->elems), "hipMalloc(scratch)");
    return PF_OK;
}

pf_status set_chunk(Model *m, int32_t chunk)
{
    m->clen = chunk > 0 ? chunk : default_chunk(&m->desc);
    plan(m);
    m->graphs_valid = false;
    pf_status st = ensure_partials(m);
    // a two-pass plan gets its mu buffer now, not inside a graph capture
    if (st == PF_OK && m->family == 0 && m->passes == 2) st = ensure_scratch(m);
    refresh_args(m);
    return st;
}

// Launch `tb` fused steps from parity `par` (writes 1 - par).  red: fuse the
// reductions of the state at the start of each of those steps; the finalised
// results go to res[0 .. kNumQ) and, for tb = 2, res[kNumQ .. 2 kNumQ).
static pf_status launch_step(Model *m, int par, bool red, double2 *res, bool timed, int tb = 1)
{
    const pf_desc &d = m->desc;
    union {
        StepArgs<double> d64;
        StepArgs<float> d32;
    } u;
    void *ap;
    if (m->fp32) {
        u.d32 = m->a32;
        u.d32.parity = par;
        u.d32.red = red;
        ap = &u.d32;
    } else {
        u.d64 = m->a64;
        u.d64.parity = par;
        u.d64.red = red;
        ap = &u.d64;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        if (m->ev_used + 2 > m->events.size()) {
            hipEvent_t a, b;
            PF_HIP(hipEventCreate(&a), "hipEventCreate");
            PF_HIP(hipEventCreate(&b), "hipEventCreate");
            m->events.push_back(a);
            m->events.push_back(b);
        }
        e0 = m->events[m->ev_used];
        e1 = m->events[m->ev_used + 1];
        m->ev_used += 2;
    }
    if (m->family == 0) {
        if (m->passes == 2) {
            pf_status st = ensure_scratch(m);
            if (st != PF_OK) return st;
        }
        if (timed) PF_HIP(hipEventRecord(e0, m->stream), "hipEventRecord");
        hipError_t e = d.ndim == 1   ? launch_fused1d(m->L, ap, m->blocks, m->threads, red, tb, m->stream)
                       : d.ndim == 2 ? launch_fused2d(m->L, ap, m->blocks, m->threads, red, tb, m->stream)
                                     : launch_fused3d(m->L, ap, m->blocks, m->threads, red, tb, m->rpw,
                                                      m->passes == 2 ? m->scratch : nullptr, m->stream);
        if (e != hipSuccess) return hip_fail(e, "step kernel launch");
        if (timed) PF_HIP(hipEventRecord(e1, m->stream), "hipEventRecord");
        if (red) {
            for (int s = 0; s < tb; ++s) {
                hipError_t f = launch_finalize(m->part + (int64_t)s * m->fused_slots, m->pstride, m->fused_slots,
                                               m->part2, res + kNumQ * s, m->stream);
                if (f != hipSuccess) return hip_fail(f, "finalize launch");
            }
        }
    } else {
        if (red) {
            hipError_t e = launch_reduce_state(m->L, ap, m->stream);
            if (e != hipSuccess) return hip_fail(e, "reduce launch");
            const int64_t N = d.n[0] * d.n[1] * d.n[2];
            e = launch_finalize(m->part, m->pstride, reduce_partial_slots(N), m->part2, res, m->stream);
            if (e != hipSuccess) return hip_fail(e, "finalize launch");
        }
        if (m->family == 2) {
            if (timed) PF_HIP(hipEventRecord(e0, m->stream), "hipEventRecord");
            pf_status st = spectral_step(m, par, ap);
            if (st != PF_OK) return st;
            if (timed) PF_HIP(hipEventRecord(e1, m->stream), "hipEventRecord");
        } else if ((mh2d_available(m->L) || mh3d_available(m->L)) && !(d.flags & PF_FORCE_GENERIC)) {
            if (timed) PF_HIP(hipEventRecord(e0, m->stream), "hipEventRecord");
            hipError_t e = d.ndim == 2 ? launch_mh2d(m->L, ap, m->stream) : launch_mh3d(m->L, ap, m->stream);
            if (e != hipSuccess) return hip_fail(e, "Model H step launch");
            if (timed) PF_HIP(hipEventRecord(e1, m->stream), "hipEventRecord");
        } else {
            pf_status st = ensure_scratch(m);
            if (st != PF_OK) return st;
            if (timed) PF_HIP(hipEventRecord(e0, m->stream), "hipEventRecord");
            hipError_t e = launch_generic(m->L, ap, m->scratch, m->stream);
            if (e != hipSuccess) return hip_fail(e, "generic step launch");
            if (timed) PF_HIP(hipEventRecord(e1, m->stream), "hipEventRecord");
        }
    }
    m->launches++;
    m->timed_steps += timed ? tb : 0;
    return PF_OK;
}

static pf_status ensure_history(Model *m, int64_t n)
{
    if (n <= m->hist_cap) return PF_OK;
    if (m->hist) {
        PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
        PF_HIP(hipFree(m->hist), "hipFree(history)");
        m->hist = nullptr;
    }
    const int64_t cap = std::max<int64_t>(n, 1024);
    PF_HIP(hipMalloc((void **)&m->hist, sizeof(double2) * kNumQ * cap), "hipMalloc(history)");
    m->hist_cap = cap;
    return PF_OK;
}

static void destroy_graphs(Model *m)
{
    for (auto &g : m->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    m->graphs.clear();
    m->graphs_valid = false;
}

// Capture `k` steps starting at parity `par` (reductions into the staging
// history rows 0..k-1 when red) as one graph.
static pf_status capture_graph(Model *m, int par, int k, bool red, Model::Graph &g)
{
    g.par = par;
    g.steps = k;
    g.red = red;
    PF_HIP(hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    pf_status st = PF_OK;
    int p = par;
    g.launches = 0;
    for (int i = 0; i < k && st == PF_OK; i += m->tb) {
        st = launch_step(m, p, red, m->stage + kNumQ * i, false, m->tb);
        p ^= 1;
        g.launches++;
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(m->stream, &graph);
    if (st != PF_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    g.graph = graph;
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    m->captures++;
    return PF_OK;
}

constexpr int32_t kLdsLaunchSteps = 4096;  // steps per launch of the whole-grid LDS kernel

pf_status do_steps(Model *m, int64_t nsteps)
{
    if (nsteps < 0) return fail(PF_ERR_ARG, "nsteps must be >= 0");
    TraceRange range("pf_step");
    const bool each = (m->desc.flags & PF_REDUCE_EACH_STEP) != 0;
    if (each) {
        pf_status st = ensure_history(m, nsteps);
        if (st != PF_OK) return st;
        m->hist_len = nsteps;
    }
    const bool use_graph = (m->desc.flags & PF_USE_GRAPH) != 0 && !m->timing;
    int64_t done = 0;
    if (m->lds_steps && !each && !m->timing) {
        // the whole grid in one workgroup's LDS, up to kLdsLaunchSteps steps per launch
        while (done < nsteps) {
            const int32_t k = (int32_t)std::min<int64_t>(nsteps - done, kLdsLaunchSteps);
            StepArgs<double> a64 = m->a64;
            StepArgs<float> a32 = m->a32;
            a64.parity = a32.parity = m->parity;
            const hipError_t e = launch_lds_steps(m->L, m->fp32 ? (const void *)&a32 : (const void *)&a64, k,
                                                  m->stream);
            if (e != hipSuccess) return hip_fail(e, "LDS step kernel launch");
            m->parity ^= (k & 1);
            m->steps_done += k;
            done += k;
        }
        return PF_OK;
    }
    if (use_graph && nsteps >= 2 * kGraphSteps) {
        if (!m->stage) PF_HIP(hipMalloc((void **)&m->stage, sizeof(double2) * kNumQ * kGraphSteps),
                              "hipMalloc(stage)");
        if (!m->graphs_valid) {
            destroy_graphs(m);
            m->graphs.resize(2);
            for (int p = 0; p < 2; ++p) {
                pf_status st = capture_graph(m, p, kGraphSteps, each, m->graphs[p]);
                if (st != PF_OK) {
                    destroy_graphs(m);
                    return st;
                }
            }
            m->graphs_valid = true;
        }
        while (nsteps - done >= kGraphSteps) {
            Model::Graph &g = m->graphs[m->parity];
            PF_HIP(hipGraphLaunch(g.exec, m->stream), "hipGraphLaunch");
            m->replays++;
            if (each)
                PF_HIP(hipMemcpyAsync(m->hist + kNumQ * done, m->stage,
                                      sizeof(double2) * kNumQ * kGraphSteps,
                                      hipMemcpyDeviceToDevice, m->stream),
                       "hipMemcpyAsync(history)");
            m->parity ^= (g.launches & 1);
            done += kGraphSteps;
            m->steps_done += kGraphSteps;
        }
    }
    while (done < nsteps) {
        const int tb = (m->tb == 2 && nsteps - done >= 2) ? 2 : 1;
        pf_status st = launch_step(m, m->parity, each, each ? m->hist + kNumQ * done : nullptr,
                                   m->timing, tb);
        if (st != PF_OK) return st;
        m->parity ^= 1;
        m->steps_done += tb;
        done += tb;
    }
    return PF_OK;
}

// pf_step_noalloc, host half: a model object that borrows the caller's
// buffers and stream, planned as pf_create_on plans it with the default tile
// (pf_set_tile(m, 0)), one step per launch and the default 3D tile layout.
// Everything is checked here, before any device call; `pairs_need` returns
// the reduction scratch (double2 pairs) the steps need (0 without
// PF_REDUCE_EACH_STEP).  Allocates nothing.
pf_status borrow_plan(Model *m, const pf_desc *d, void *stream, void *const *bufs, int32_t nbufs,
                      int32_t parity, int64_t nsteps, const void *hist, int64_t *pairs_need)
{
    pf_status st = check_desc(d);
    if (st != PF_OK) return st;
    if (!(d->flags & PF_ALLOW_UNSTABLE) && d->dt > stability_limit(d))
        return fail(PF_ERR_UNSTABLE, "dt exceeds the explicit-stability limit");
    if (d->flags & (PF_SPECTRAL | PF_FORCE_GENERIC | PF_USE_GRAPH))
        return fail(PF_ERR_ARG, "pf_step_noalloc takes no PF_SPECTRAL, PF_FORCE_GENERIC or PF_USE_GRAPH");
    if (!bufs || nbufs != 2 * d->nfields) return fail(PF_ERR_ARG, "nbufs must be 2 * nfields");
    if (parity != 0 && parity != 1) return fail(PF_ERR_ARG, "parity must be 0 or 1");
    if (nsteps < 0) return fail(PF_ERR_ARG, "nsteps must be >= 0");
    const bool red = (d->flags & PF_REDUCE_EACH_STEP) != 0;
    if (red && nsteps > 0 && !hist) return fail(PF_ERR_ARG, "PF_REDUCE_EACH_STEP needs a history buffer");
    m->desc = *d;
    m->nf = d->nfields;
    m->fp32 = d->precision == PF_FP32;
    m->L = Launch{(d->kind == kCH && (d->flags & PF_BIHARMONIC_DIRECT)) ? kCHD : d->kind, d->ndim,
                  d->order / 2, m->fp32 ? 1 : 0};
    m->pitch = pitch_of(d);
    m->elems = buffer_elems(d);
    m->stream = static_cast<hipStream_t>(stream);
    m->own_stream = false;
    m->own_bufs = false;
    for (int f = 0; f < m->nf; ++f)
        for (int p = 0; p < 2; ++p) {
            void *b = bufs[2 * f + p];
            if (!b || (reinterpret_cast<uintptr_t>(b) & 15))
                return fail(PF_ERR_ARG, "device buffers must be non-NULL and 16-byte aligned");
            m->buf[f][p] = b;
        }
    m->tb = 1;
    m->rpw_req = 0;
    m->passes_req = 1;  // the mu buffer of two passes would be an allocation
    m->clen = default_chunk(d);
    plan(m);
    if (m->family != 0)
        return fail(PF_ERR_UNSUPPORTED, "this descriptor runs kernels that need a field-sized "
                                        "temporary; pf_step_noalloc covers the fused kernels");
    m->parity = parity;
    *pairs_need = red ? (int64_t)kNumQ * (m->fused_slots + kFinSlots) : 0;
    return PF_OK;
}

// pf_step_noalloc, device half: the reduction partials in `scratch` (every
// pair a step reads is written earlier in the same step, so nothing needs
// clearing), nsteps launches, the finalised reductions of step k (the state
// at its start) to hist[kNumQ k .. kNumQ k + kNumQ).
pf_status borrow_run(Model *m, double2 *scratch, int64_t nsteps, double2 *hist)
{
    const bool red = (m->desc.flags & PF_REDUCE_EACH_STEP) != 0;
    m->part = red ? scratch : nullptr;
    m->pstride = red ? m->fused_slots : 0;
    m->part2 = red ? scratch + (int64_t)kNumQ * m->fused_slots : nullptr;
    refresh_args(m);
    for (int64_t k = 0; k < nsteps; ++k) {
        pf_status st = launch_step(m, m->parity, red, red ? hist + (int64_t)kNumQ * k : nullptr, false, 1);
        if (st != PF_OK) return st;
        m->parity ^= 1;
    }
    return PF_OK;
}

pf_status reduce_now(Model *m, double2 *host_out)
{
    union {
        StepArgs<double> d64;
        StepArgs<float> d32;
    } u;
    void *ap;
    if (m->fp32) {
        u.d32 = m->a32;
        u.d32.parity = m->parity;
        ap = &u.d32;
    } else {
        u.d64 = m->a64;
        u.d64.parity = m->parity;
        ap = &u.d64;
    }
    const int64_t N = m->desc.n[0] * m->desc.n[1] * m->desc.n[2];
    hipError_t e = launch_reduce_state(m->L, ap, m->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
    e = launch_finalize(m->part, m->pstride, reduce_partial_slots(N), m->part2, m->res, m->stream);
    if (e != hipSuccess) return hip_fail(e, "finalize launch");
    PF_HIP(hipMemcpyAsync(host_out, m->res, sizeof(double2) * kNumQ, hipMemcpyDeviceToHost, m->stream),
           "hipMemcpyAsync(reductions)");
    PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PF_OK;
}

double volume(const pf_desc &d)
{
    double v = 1.0;
    for (int a = 0; a < d.ndim; ++a) v *= d.dx;
    return v;
}

pf_status pick_quantity(const Model *m, int32_t which, const double2 *q, double *hi, double *lo)
{
    const pf_desc &d = m->desc;
    const double vol = volume(d);
    switch (which) {
    case PF_RED_MASS0:
        *hi = q[0].x * vol;
        *lo = q[0].y * vol;
        return PF_OK;
    case PF_RED_MASS1:
        if (nfields_of(d.kind) != 2) return fail(PF_ERR_UNSUPPORTED, "mass of field 1 needs Gray-Scott or Model C");
        *hi = q[1].x * vol;
        *lo = q[1].y * vol;
        return PF_OK;
    case PF_RED_ENERGY:
        if (d.kind == kGS || d.kind == kMC || d.kind == kMH)
            return fail(PF_ERR_UNSUPPORTED, "free energy is reduced for Allen-Cahn and Cahn-Hilliard only");
        if (d.flags & PF_SPECTRAL)
            return fail(PF_ERR_UNSUPPORTED, "no free energy for the spectral scheme");
        *hi = q[1].x * vol;
        *lo = q[1].y * vol;
        return PF_OK;
    case PF_RED_NONFINITE:
        *hi = q[2].x;
        *lo = 0.0;
        return PF_OK;
    default:
        return fail(PF_ERR_ARG, "unknown reduction");
    }
}

pf_status model_create(const pf_desc *desc, void *stream, void *const *bufs, int32_t nbufs,
                       Model **out, bool async_alloc)
{
    pf_status st = check_desc(desc);
    if (st != PF_OK) return st;
    if (!out) return fail(PF_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!(desc->flags & PF_ALLOW_UNSTABLE)) {
        const double lim = stability_limit(desc);
        if (desc->dt > lim) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "dt = %g exceeds the explicit-stability limit %g", desc->dt, lim);
            return fail(PF_ERR_UNSTABLE, msg);
        }
    }
    Model *m = new Model();
    m->async_alloc = async_alloc && stream != nullptr;
    m->desc = *desc;
    m->nf = desc->nfields;
    m->fp32 = desc->precision == PF_FP32;
    m->L = Launch{(desc->kind == kCH && (desc->flags & PF_BIHARMONIC_DIRECT)) ? kCHD : desc->kind,
                  desc->ndim, desc->order / 2, m->fp32 ? 1 : 0};
    m->pitch = pitch_of(desc);
    m->elems = buffer_elems(desc);
    hipError_t e;
    if (stream) {
        m->stream = static_cast<hipStream_t>(stream);
    } else {
        e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete m;
            return hip_fail(e, "hipStreamCreate");
        }
        m->own_stream = true;
    }
    const size_t bytes = tsize(m) * (size_t)m->elems;
    if (bufs) {
        if (nbufs != 2 * m->nf) {
            pf_destroy_model(m);
            return fail(PF_ERR_ARG, "nbufs must be 2 * nfields");
        }
        for (int f = 0; f < m->nf; ++f)
            for (int p = 0; p < 2; ++p) {
                void *b = bufs[2 * f + p];
                if (!b || (reinterpret_cast<uintptr_t>(b) & 15)) {
                    pf_destroy_model(m);
                    return fail(PF_ERR_ARG, "device buffers must be non-NULL and 16-byte aligned");
                }
                m->buf[f][p] = b;
            }
        m->own_bufs = false;
    } else {
        for (int f = 0; f < m->nf; ++f)
            for (int p = 0; p < 2; ++p) {
                e = dev_alloc(m, &m->buf[f][p], bytes);
                if (e != hipSuccess) {
                    pf_destroy_model(m);
                    hip_fail(e, "hipMalloc(field)");
                    return PF_ERR_NOMEM;
                }
                if (m->async_alloc) continue;  // the caller initialises the fields
                e = hipMemsetAsync(m->buf[f][p], 0, bytes, m->stream);
                if (e != hipSuccess) {
                    pf_destroy_model(m);
                    return hip_fail(e, "hipMemsetAsync(field)");
                }
            }
        m->own_bufs = true;
    }
    e = dev_alloc(m, (void **)&m->res, sizeof(double2) * kNumQ);
    if (e == hipSuccess) e = dev_alloc(m, (void **)&m->part2, sizeof(double2) * kNumQ * kFinSlots);
    if (e != hipSuccess) {
        pf_destroy_model(m);
        return hip_fail(e, "hipMalloc(result)");
    }
    int32_t chunk = 0;
    // served requests take the batched kernels' layout (two tile rows per
    // wave in 3D, two-step sweeps where the class has them); the serving
    // autotuner sets their chunk after admission
    if (m->async_alloc) {
        m->rpw_req = desc->ndim == 3 ? rows_per_wave_batched(m->L) : 2;
        m->passes_req = 1;
        m->tb = time_block_available(m->L) ? 2 : 1;
    }
    if (!m->async_alloc) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(tune_key(*desc));
        if (it != g_tune_cache.end()) {
            chunk = it->second.chunk;
            m->tb = it->second.tb;
            m->rpw_req = it->second.rpw;
            m->passes_req = it->second.passes;
        }
    }
    st = set_chunk(m, chunk);
    if (st == PF_OK && (desc->flags & PF_SPECTRAL)) st = spectral_setup(m);
    if (st != PF_OK) {
        pf_destroy_model(m);
        return st;
    }
    if (!m->async_alloc) {
        e = hipStreamSynchronize(m->stream);
        if (e != hipSuccess) {
            pf_destroy_model(m);
            return hip_fail(e, "hipStreamSynchronize");
        }
    }
    *out = m;
    return PF_OK;
}

void model_release_async(Model *m)
{
    if (!m) return;
    for (int f = 0; f < kMaxFields; ++f)
        for (int p = 0; p < 2; ++p)
            if (m->own_bufs) dev_free(m, m->buf[f][p]);
    dev_free(m, m->part);
    dev_free(m, m->part2);
    dev_free(m, m->res);
    dev_free(m, m->hist);
    dev_free(m, m->stage);
    dev_free(m, m->scratch);
    spectral_release(m);
    destroy_graphs(m);
    for (auto ev : m->events) (void)hipEventDestroy(ev);
    delete m;
}

void pf_destroy_model(Model *m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    if (m->async_alloc) {
        const bool own = m->own_stream;
        hipStream_t st = m->stream;
        model_release_async(m);
        if (own && st) (void)hipStreamDestroy(st);
        return;
    }
    destroy_graphs(m);
    if (m->own_bufs)
        for (int f = 0; f < kMaxFields; ++f)
            for (int p = 0; p < 2; ++p)
                if (m->buf[f][p]) (void)hipFree(m->buf[f][p]);
    if (m->part) (void)hipFree(m->part);
    if (m->res) (void)hipFree(m->res);
    if (m->part2) (void)hipFree(m->part2);
    if (m->hist) (void)hipFree(m->hist);
    if (m->stage) (void)hipFree(m->stage);
    if (m->scratch) (void)hipFree(m->scratch);
    spectral_release(m);
    for (auto ev : m->events) (void)hipEventDestroy(ev);
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
}

pf_status init_fields(Model *m, int32_t ic, uint64_t seed, const double *p, int32_t np)
{
    const pf_desc &d = m->desc;
    InitArgs a;
    std::memset(&a, 0, sizeof(a));
    a.f0 = m->buf[0][m->parity];
    a.f1 = m->nf > 1 ? m->buf[1][m->parity] : nullptr;
    a.nx = d.n[0];
    a.ny = d.n[1];
    a.nz = d.n[2];
    a.pitch = m->pitch;
    a.plane = m->pitch * d.n[1];
    a.fp32 = m->fp32;
    a.nfields = std::min(2, m->nf);  // fields 0 and 1 here, the rest below
    a.ic = ic;
    a.key0 = stream_key(seed, 0);
    a.key1 = stream_key(seed, 1);
    if (ic == PF_IC_UNIFORM) {
        if (np < 2 || !p) return fail(PF_ERR_ARG, "uniform IC needs {lo, hi}");
        a.lo = p[0];
        a.span = p[1] - p[0];
    } else if (ic == PF_IC_GS_CUBES) {
        if (d.kind != kGS) return fail(PF_ERR_ARG, "cube IC is for Gray-Scott");
        if (np < 3 || !p) return fail(PF_ERR_ARG, "cube IC needs {ncubes, side, noise}");
        const int nc = (int)p[0];
        if (nc < 0 || nc > 64) return fail(PF_ERR_ARG, "ncubes must be 0..64");
        if (p[1] < 1) return fail(PF_ERR_ARG, "cube side must be >= 1");
        a.ncubes = nc;
        a.side = (int32_t)p[1];
        a.lo = -p[2];
        a.span = p[2] - (-p[2]);
        a.v0 = 1.0;
        a.v1 = 0.0;
        a.in0 = 0.5;
        a.in1 = 0.25;
        const uint64_t k2 = stream_key(seed, 2);
        const int64_t ext[3] = {d.n[0], d.n[1], d.n[2]};
        for (int c = 0; c < nc; ++c)
            for (int ax = 0; ax < 3; ++ax) {
                const double u = u01_host(k2, (uint64_t)(3 * c + ax));
                int64_t v = (int64_t)std::floor(u * (double)ext[ax]);
                a.cube[c][ax] = (int32_t)std::min<int64_t>(v, ext[ax] - 1);
            }
    } else if (ic == PF_IC_CONST) {
        if (np < m->nf || !p) return fail(PF_ERR_ARG, "const IC needs one value per field");
        a.v0 = p[0];
        a.v1 = m->nf > 1 ? p[1] : 0.0;
    } else {
        return fail(PF_ERR_ARG, "unknown initial condition");
    }
    hipError_t e = launch_init(a, m->stream);
    if (e != hipSuccess) return hip_fail(e, "init launch");
    // Model H: fields 2 and 3 (j_y, j_z) from streams 2 and 3, as fields 0, 1
    for (int f = 2; f < m->nf && e == hipSuccess; f += 2) {
        a.f0 = m->buf[f][m->parity];
        a.f1 = f + 1 < m->nf ? m->buf[f + 1][m->parity] : nullptr;
        a.nfields = std::min(2, m->nf - f);
        a.key0 = stream_key(seed, (uint64_t)f);
        a.key1 = stream_key(seed, (uint64_t)f + 1);
        if (ic == PF_IC_CONST) {
            a.v0 = p[f];
            a.v1 = f + 1 < m->nf ? p[f + 1] : 0.0;
        }
        e = launch_init(a, m->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "init launch");
    m->steps_done = 0;
    spectral_invalidate(m);
    return PF_OK;
}

// Times every candidate (chunk length, time-block factor) on the model's own
// buffers: each trial re-runs steps from the current parity, whose buffer is
// never written, so the state is untouched.  Keeps the fastest per step.
constexpr float kTuneMinMs = 2.0f;  // least timed span per autotuner candidate

pf_status autotune(Model *m, int32_t trials)
{
    if (m->family != 0) return PF_OK;
    TraceRange range("pf_autotune");
    const pf_desc &d = m->desc;
    const bool red = (d.flags & PF_REDUCE_EACH_STEP) != 0;
    // chunk candidates up to the marching extent (1D: strips per wave)
    const int64_t march = d.ndim == 1 ? std::max<int64_t>(1, d.n[0] / (m->fp32 ? 224 : 112))
                          : d.ndim == 2 ? d.n[1] : d.n[2];
    std::vector<int32_t> cand;
    const int32_t base[] = {16, 32, 64, 128, 256, 512, 1024};
    for (int32_t c : base)
        if (c <= march * 2 || cand.empty()) cand.push_back((int32_t)std::min<int64_t>(c, march));
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    std::vector<int> tbs = {1};
    if (time_block_available(m->L)) tbs.push_back(2);
    if (trials < 1) trials = 3;
    const int32_t keep_c = m->clen;
    const int keep_tb = m->tb, keep_rpw = m->rpw_req, keep_passes = m->passes_req;
    hipEvent_t a, b;
    PF_HIP(hipEventCreate(&a), "hipEventCreate");
    PF_HIP(hipEventCreate(&b), "hipEventCreate");
    double2 *scratch = nullptr;
    if (red) PF_HIP(hipMalloc((void **)&scratch, sizeof(double2) * kNumQ * 2), "hipMalloc(tune)");
    float best = 1e30f;
    TuneChoice bestc{keep_c, keep_tb, keep_rpw, keep_passes};
    pf_status st = PF_OK;
    // (tb, rpw, passes): every time block and 3D tile layout in one pass, and
    // the two-pass form where it exists
    std::vector<std::array<int, 3>> forms;
    for (int tb : tbs)
        for (int rpw : {2, 1, 4})
            if (d.ndim != 3 ? rpw == 2 : rows_per_wave_available(m->L, tb, rpw)) forms.push_back({tb, rpw, 1});
    if (two_pass_available(m->L) && !(d.flags & PF_FORCE_GENERIC)) forms.push_back({1, 2, 2});
    for (const auto &fm : forms) {
        const int tb = fm[0], rpw = fm[1], passes = fm[2];
        {
            for (int32_t c : cand) {
                m->tb = tb;
                m->rpw_req = d.ndim == 3 ? rpw : 0;
                m->passes_req = passes;
                st = set_chunk(m, c);
                if (st != PF_OK || m->family != 0 || m->tb != tb || m->passes != passes) break;
                st = launch_step(m, m->parity, red, scratch, false, tb);
                if (st != PF_OK) break;
                // time `trials` launches; where they take less than kTuneMinMs,
                // time again with enough launches to fill it (short launches
                // differ by a few percent from one to the next)
                int reps = trials;
                float ms = 0;
                for (int pass = 0; pass < 2 && st == PF_OK; ++pass) {
                    (void)hipEventRecord(a, m->stream);
                    for (int t = 0; t < reps && st == PF_OK; ++t)
                        st = launch_step(m, m->parity, red, scratch, false, tb);
                    (void)hipEventRecord(b, m->stream);
                    (void)hipEventSynchronize(b);
                    (void)hipEventElapsedTime(&ms, a, b);
                    if (pass > 0 || ms >= kTuneMinMs || !(ms > 0.f)) break;
                    reps = std::min(64, (int)std::ceil(reps * kTuneMinMs / ms));
                }
                ms /= (float)reps * tb;
                if (st == PF_OK && ms < best) {
                    best = ms;
                    bestc = {c, tb, m->rpw_req, passes};
                }
            }
            if (st != PF_OK) break;
        }
        if (st != PF_OK) break;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (scratch) (void)hipFree(scratch);
    if (st != PF_OK) return st;
    m->tb = bestc.tb;
    m->rpw_req = bestc.rpw;
    m->passes_req = bestc.passes;
    if (m->passes_req != 2 && m->scratch && m->family == 0) {  // the mu buffer of a tried two-pass plan
        dev_free(m, m->scratch);
        m->scratch = nullptr;
    }
    st = set_chunk(m, bestc.chunk);
    if (st != PF_OK) return st;
    m->launches = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[tune_key(d)] = bestc;
    }
    return PF_OK;
}

}  // namespace pf

// ===================================================================== ABI
using namespace pf;

#define PF_API extern "C" __attribute__((visibility("default")))

PF_API int32_t pf_abi_version(void) { return PF_ABI_VERSION; }

PF_API const char *pf_last_error(void) { return g_err.c_str(); }

PF_API const char *pf_status_str(pf_status s)
{
    switch (s) {
    case PF_OK: return "ok";
    case PF_ERR_ARG: return "invalid argument";
    case PF_ERR_UNSTABLE: return "time step above the stability limit";
    case PF_ERR_NOMEM: return "out of memory";
    case PF_ERR_DEVICE: return "device error";
    case PF_ERR_STATE: return "invalid state";
    case PF_ERR_UNSUPPORTED: return "unsupported";
    case PF_ERR_BUSY: return "busy";
    case PF_ERR_NOTFOUND: return "not found";
    }
    return "unknown status";
}

PF_API pf_status pf_weights(int32_t order, double *w)
{
    if (!w) return fail(PF_ERR_ARG, "w is NULL");
    if (!centered_d2_weights(order, w)) return fail(PF_ERR_ARG, "order must be even, 2..16");
    return PF_OK;
}

PF_API pf_status pf_weights1(int32_t order, double *w1)
{
    if (!w1) return fail(PF_ERR_ARG, "w1 is NULL");
    if (!centered_d1_weights(order, w1)) return fail(PF_ERR_ARG, "order must be even, 2..16");
    return PF_OK;
}

PF_API pf_status pf_weights4(int32_t order, double *w4)
{
    if (!w4) return fail(PF_ERR_ARG, "w4 is NULL");
    if (!centered_d4_weights(order, w4)) return fail(PF_ERR_ARG, "order must be even, 2..16");
    return PF_OK;
}

PF_API pf_status pf_stability(const pf_desc *desc, double *dt_max)
{
    pf_status st = check_desc(desc);
    if (st != PF_OK) return st;
    if (!dt_max) return fail(PF_ERR_ARG, "dt_max is NULL");
    *dt_max = stability_limit(desc);
    return PF_OK;
}

PF_API int64_t pf_buffer_elems(const pf_desc *desc)
{
    if (check_desc(desc) != PF_OK) return -1;
    return buffer_elems(desc);
}

// Field-sized scratch arrays of the per-site generic kernels (CH: mu; the
// direct biharmonic: mu_a of every axis), held where the fused kernels do not
// cover the descriptor (1D and 2D: r <= 4; 3D: CH r <= 3, direct form r <= 2).
static int generic_scratch_arrays(const pf_desc *d)
{
    if (d->kind == kMH) {  // mu, except on 1D rows (fused, r <= 4), 2D tiles and 3D marches (r <= 2)
        const int r = d->order / 2;
        const bool one_pass = !(d->flags & PF_FORCE_GENERIC) &&
                              ((d->ndim == 1 && r <= 4) || (d->ndim >= 2 && r <= 2));
        return one_pass ? 0 : 1;
    }
    if (d->kind != kCH) return 0;
    const bool direct = (d->flags & PF_BIHARMONIC_DIRECT) != 0;
    const int r = d->order / 2;
    bool fused = !(d->flags & PF_FORCE_GENERIC) && r <= 4;
    if (d->ndim == 3) fused = fused && r <= 3;
    if (fused) return 0;
    return direct ? d->ndim : 1;
}

PF_API uint64_t pf_footprint_bytes(const pf_desc *desc)
{
    if (check_desc(desc) != PF_OK) return 0;
    const uint64_t P = (uint64_t)elem_bytes(desc);
    const uint64_t N = (uint64_t)(desc->n[0] * desc->n[1] * desc->n[2]);
    uint64_t bytes = (2ull * desc->nfields + (uint64_t)generic_scratch_arrays(desc)) *
                     (uint64_t)buffer_elems(desc) * P;
    if (desc->flags & PF_SPECTRAL) bytes += spectral_bytes(desc);
    // reduction partials (per-wave pairs) and the result block
    bytes += sizeof(double2) * kNumQ * (uint64_t)std::max<int64_t>(reduce_partial_slots((int64_t)N), N / 64 + 1);
    bytes += sizeof(double2) * kNumQ;
    return bytes;
}

PF_API pf_status pf_create(const pf_desc *desc, void *hip_stream, pf_model **out)
{
    Model *m = nullptr;
    pf_status st = model_create(desc, hip_stream, nullptr, 0, &m);
    if (out) *out = reinterpret_cast<pf_model *>(m);
    return st;
}

PF_API pf_status pf_create_on(const pf_desc *desc, void *hip_stream, void *const *dev_bufs,
                              int32_t nbufs, pf_model **out)
{
    if (!dev_bufs) return fail(PF_ERR_ARG, "dev_bufs is NULL");
    Model *m = nullptr;
    pf_status st = model_create(desc, hip_stream, dev_bufs, nbufs, &m);
    if (out) *out = reinterpret_cast<pf_model *>(m);
    return st;
}

PF_API void pf_destroy(pf_model *m) { pf_destroy_model(reinterpret_cast<Model *>(m)); }

static Model *M(pf_model *m) { return reinterpret_cast<Model *>(m); }

PF_API pf_status pf_init(pf_model *m, int32_t ic, uint64_t seed, const double *ic_params,
                         int32_t n_ic_params)
{
    if (!m) return fail(PF_ERR_ARG, "model is NULL");
    return init_fields(M(m), ic, seed, ic_params, n_ic_params);
}

PF_API pf_status pf_set_field(pf_model *mm, int32_t field, const double *host, int64_t count)
{
    Model *m = M(mm);
    if (!m || !host) return fail(PF_ERR_ARG, "NULL argument");
    if (field < 0 || field >= m->nf) return fail(PF_ERR_ARG, "field index out of range");
    const pf_desc &d = m->desc;
    const int64_t N = d.n[0] * d.n[1] * d.n[2];
    if (count != N) return fail(PF_ERR_ARG, "count must equal the number of sites");
    const size_t ts = tsize(m);
    std::vector<unsigned char> stage;
    const void *src = host;
    if (m->fp32) {
        stage.resize(ts * (size_t)N);
        float *s = reinterpret_cast<float *>(stage.data());
        for (int64_t i = 0; i < N; ++i) s[i] = (float)host[i];
        src = s;
    }
    spectral_invalidate(m);
    PF_HIP(hipMemcpy2DAsync(m->buf[field][m->parity], ts * m->pitch, src, ts * d.n[0], ts * d.n[0],
                            d.n[1] * d.n[2], hipMemcpyHostToDevice, m->stream),
           "hipMemcpy2DAsync(set_field)");
    PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PF_OK;
}

PF_API pf_status pf_get_field(pf_model *mm, int32_t field, double *host, int64_t count)
{
    Model *m = M(mm);
    if (!m || !host) return fail(PF_ERR_ARG, "NULL argument");
    if (field < 0 || field >= m->nf) return fail(PF_ERR_ARG, "field index out of range");
    const pf_desc &d = m->desc;
    const int64_t N = d.n[0] * d.n[1] * d.n[2];
    if (count != N) return fail(PF_ERR_ARG, "count must equal the number of sites");
    const size_t ts = tsize(m);
    if (m->fp32) {
        std::vector<float> stage((size_t)N);
        PF_HIP(hipMemcpy2DAsync(stage.data(), ts * d.n[0], m->buf[field][m->parity], ts * m->pitch,
                                ts * d.n[0], d.n[1] * d.n[2], hipMemcpyDeviceToHost, m->stream),
               "hipMemcpy2DAsync(get_field)");
        PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
        for (int64_t i = 0; i < N; ++i) host[i] = (double)stage[i];
    } else {
        PF_HIP(hipMemcpy2DAsync(host, ts * d.n[0], m->buf[field][m->parity], ts * m->pitch,
                                ts * d.n[0], d.n[1] * d.n[2], hipMemcpyDeviceToHost, m->stream),
               "hipMemcpy2DAsync(get_field)");
        PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    }
    return PF_OK;
}

PF_API pf_status pf_get_window(pf_model *mm, int32_t field, const int64_t *origin, const int64_t *w,
                               double *host)
{
    Model *m = M(mm);
    if (!m || !origin || !w || !host) return fail(PF_ERR_ARG, "NULL argument");
    if (field < 0 || field >= m->nf) return fail(PF_ERR_ARG, "field index out of range");
    const pf_desc &d = m->desc;
    for (int a = 0; a < 3; ++a)
        if (w[a] < 1 || w[a] > d.n[a]) return fail(PF_ERR_ARG, "window extent must be 1..n");
    const size_t ts = tsize(m);
    std::vector<unsigned char> row(ts * (size_t)d.n[0]);
    PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    int64_t k = 0;
    for (int64_t z = 0; z < w[2]; ++z)
        for (int64_t y = 0; y < w[1]; ++y) {
            const int64_t zz = ((origin[2] + z) % d.n[2] + d.n[2]) % d.n[2];
            const int64_t yy = ((origin[1] + y) % d.n[1] + d.n[1]) % d.n[1];
            const unsigned char *src = static_cast<const unsigned char *>(m->buf[field][m->parity]) +
                                       ts * (size_t)(zz * m->pitch * d.n[1] + yy * m->pitch);
            PF_HIP(hipMemcpy(row.data(), src, ts * (size_t)d.n[0], hipMemcpyDeviceToHost),
                   "hipMemcpy(window row)");
            for (int64_t x = 0; x < w[0]; ++x) {
                const int64_t xx = ((origin[0] + x) % d.n[0] + d.n[0]) % d.n[0];
                host[k++] = m->fp32 ? (double)reinterpret_cast<const float *>(row.data())[xx]
                                    : reinterpret_cast<const double *>(row.data())[xx];
            }
        }
    return PF_OK;
}

PF_API pf_status pf_field_device(pf_model *mm, int32_t field, void **ptr, int64_t *pitch_elems,
                                 int32_t *eb)
{
    Model *m = M(mm);
    if (!m) return fail(PF_ERR_ARG, "model is NULL");
    if (field < 0 || field >= m->nf) return fail(PF_ERR_ARG, "field index out of range");
    if (ptr) *ptr = m->buf[field][m->parity];
    spectral_invalidate(m);  // the caller may write through the view
    if (pitch_elems) *pitch_elems = m->pitch;
    if (eb) *eb = (int32_t)tsize(m);
    return PF_OK;
}

PF_API pf_status pf_step(pf_model *m, int64_t nsteps)
{
    if (!m) return fail(PF_ERR_ARG, "model is NULL");
    return do_steps(M(m), nsteps);
}

PF_API pf_status pf_reduce(pf_model *mm, int32_t which, double *hi, double *lo)
{
    Model *m = M(mm);
    if (!m || !hi || !lo) return fail(PF_ERR_ARG, "NULL argument");
    double2 q[kNumQ];
    pf_status st = reduce_now(m, q);
    if (st != PF_OK) return st;
    return pick_quantity(m, which, q, hi, lo);
}

PF_API pf_status pf_reduce_history(pf_model *mm, int32_t which, double *hi, double *lo,
                                   int64_t count)
{
    Model *m = M(mm);
    if (!m || !hi || !lo) return fail(PF_ERR_ARG, "NULL argument");
    if (!(m->desc.flags & PF_REDUCE_EACH_STEP)) return fail(PF_ERR_STATE, "PF_REDUCE_EACH_STEP not set");
    if (count < 0 || count > m->hist_len) return fail(PF_ERR_ARG, "count exceeds the recorded steps");
    std::vector<double2> h((size_t)count * kNumQ);
    if (count) {
        PF_HIP(hipMemcpyAsync(h.data(), m->hist, sizeof(double2) * kNumQ * count, hipMemcpyDeviceToHost,
                              m->stream),
               "hipMemcpyAsync(history)");
    }
    PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    for (int64_t k = 0; k < count; ++k) {
        pf_status st = pick_quantity(m, which, &h[(size_t)k * kNumQ], &hi[k], &lo[k]);
        if (st != PF_OK) return st;
    }
    return PF_OK;
}

PF_API pf_status pf_sync(pf_model *mm)
{
    Model *m = M(mm);
    if (!m) return fail(PF_ERR_ARG, "model is NULL");
    PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PF_OK;
}

PF_API int64_t pf_steps_done(const pf_model *m)
{
    return m ? reinterpret_cast<const Model *>(m)->steps_done : -1;
}

PF_API pf_status pf_set_steps_done(pf_model *m, int64_t steps)
{
    if (!m || steps < 0) return fail(PF_ERR_ARG, "bad argument");
    M(m)->steps_done = steps;
    return PF_OK;
}

PF_API pf_status pf_stream(pf_model *m, void **s)
{
    if (!m || !s) return fail(PF_ERR_ARG, "NULL argument");
    *s = M(m)->stream;
    return PF_OK;
}

PF_API pf_status pf_set_tile(pf_model *m, int32_t chunk)
{
    if (!m || chunk < 0) return fail(PF_ERR_ARG, "bad argument");
    PF_HIP(hipStreamSynchronize(M(m)->stream), "hipStreamSynchronize");
    return set_chunk(M(m), chunk);
}

PF_API pf_status pf_get_tile(pf_model *m, int32_t *chunk, int32_t *family)
{
    if (!m) return fail(PF_ERR_ARG, "model is NULL");
    if (chunk) *chunk = M(m)->clen;
    if (family) *family = M(m)->family;
    return PF_OK;
}

PF_API pf_status pf_set_time_block(pf_model *m, int32_t tb)
{
    if (!m || (tb != 1 && tb != 2)) return fail(PF_ERR_ARG, "time block must be 1 or 2");
    Model *mm = M(m);
    PF_HIP(hipStreamSynchronize(mm->stream), "hipStreamSynchronize");
    if (tb == 2 && (!time_block_available(mm->L) || mm->desc.flags & PF_FORCE_GENERIC))
        return fail(PF_ERR_UNSUPPORTED, "two-step kernels exist for 2D orders 2 and 4 and 3D order 2");
    mm->tb = tb;
    pf_status st = set_chunk(mm, mm->clen);
    if (st == PF_OK && mm->tb != tb) return fail(PF_ERR_UNSUPPORTED, "two-step kernel not available");
    return st;
}

PF_API int32_t pf_get_time_block(const pf_model *m) { return m ? reinterpret_cast<const Model *>(m)->tb : -1; }

PF_API pf_status pf_set_tile_rows(pf_model *m, int32_t rows)
{
    if (!m || rows < 0 || rows > 4 || rows == 3) return fail(PF_ERR_ARG, "tile rows must be 0, 1, 2 or 4");
    Model *mm = M(m);
    PF_HIP(hipStreamSynchronize(mm->stream), "hipStreamSynchronize");
    if (mm->desc.ndim != 3 || mm->family != 0)
        return fail(PF_ERR_UNSUPPORTED, "tile rows apply to the fused 3D kernels");
    if (rows && !rows_per_wave_available(mm->L, mm->tb, rows))
        return fail(PF_ERR_UNSUPPORTED, "one row per wave is built for FP64 AC (order <= 4) and GS (order 2), "
                                        "four for CH, Model C, GS (order >= 4) and AC (order 8)");
    mm->rpw_req = rows;
    return set_chunk(mm, mm->clen);
}

PF_API int32_t pf_get_tile_rows(const pf_model *m)
{
    if (!m) return -1;
    const Model *mm = reinterpret_cast<const Model *>(m);
    return (mm->desc.ndim == 3 && mm->family == 0) ? mm->rpw : 0;
}

PF_API pf_status pf_set_passes(pf_model *m, int32_t passes)
{
    if (!m || (passes != 1 && passes != 2)) return fail(PF_ERR_ARG, "passes must be 1 or 2");
    Model *mm = M(m);
    PF_HIP(hipStreamSynchronize(mm->stream), "hipStreamSynchronize");
    if (passes == 2 && (mm->desc.flags & (PF_FORCE_GENERIC | PF_SPECTRAL) || !two_pass_available(mm->L)))
        return fail(PF_ERR_UNSUPPORTED, "two passes exist for 3D Cahn-Hilliard (composed form, order <= 6)");
    mm->passes_req = passes;
    if (passes == 2) mm->tb = 1;
    pf_status st = set_chunk(mm, mm->clen);
    if (st == PF_OK && mm->passes == 1 && mm->scratch && mm->family == 0) {
        dev_free(mm, mm->scratch);
        mm->scratch = nullptr;
    }
    if (st == PF_OK && mm->passes != passes) return fail(PF_ERR_UNSUPPORTED, "two-pass kernels not available");
    return st;
}

PF_API int32_t pf_get_passes(const pf_model *m)
{
    if (!m) return -1;
    const Model *mm = reinterpret_cast<const Model *>(m);
    return mm->family == 0 ? mm->passes : 0;
}

PF_API pf_status pf_autotune(pf_model *m, int32_t trials)
{
    if (!m) return fail(PF_ERR_ARG, "model is NULL");
    return autotune(M(m), trials);
}

PF_API pf_status pf_timing_enable(pf_model *mm, int32_t on)
{
    Model *m = M(mm);
    if (!m) return fail(PF_ERR_ARG, "model is NULL");
    PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    m->timing = on != 0;
    m->ev_used = 0;
    m->timed_steps = 0;
    return PF_OK;
}

PF_API pf_status pf_timing_read(pf_model *mm, double *total_ms, int64_t *launches, int64_t *steps)
{
    Model *m = M(mm);
    if (!m) return fail(PF_ERR_ARG, "model is NULL");
    PF_HIP(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    double tot = 0.0;
    for (size_t i = 0; i + 1 < m->ev_used; i += 2) {
        float ms = 0;
        PF_HIP(hipEventElapsedTime(&ms, m->events[i], m->events[i + 1]), "hipEventElapsedTime");
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)(m->ev_used / 2);
    if (steps) *steps = m->timed_steps;
    return PF_OK;
}

PF_API pf_status pf_copy_probe(void *dst, const void *src, uint64_t bytes, void *hip_stream,
                               int32_t reps, double *ms_per_rep)
{
    if (!dst || !src || (bytes & 15) || (reinterpret_cast<uintptr_t>(dst) & 15) ||
        (reinterpret_cast<uintptr_t>(src) & 15))
        return fail(PF_ERR_ARG, "copy probe needs 16-byte aligned pointers and size");
    if (reps < 1) reps = 1;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipEvent_t a, b;
    PF_HIP(hipEventCreate(&a), "hipEventCreate");
    PF_HIP(hipEventCreate(&b), "hipEventCreate");
    hipError_t e = launch_copy(dst, src, bytes, s);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_copy(dst, src, bytes, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "copy probe");
    if (ms_per_rep) *ms_per_rep = ms / reps;
    return PF_OK;
}
