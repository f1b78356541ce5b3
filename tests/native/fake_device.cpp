// Test-only fake executor for the serving scheduler (csrc/serve.cpp) on the
// CPU: the HIP runtime calls the scheduler makes and the runtime/kernel
// functions it links against, implemented on host memory so that the
// scheduler's host logic can run under AddressSanitizer, UndefinedBehavior-
// Sanitizer and ThreadSanitizer with no GPU.
//
// Device model.  One "device thread" executes every enqueued operation in
// global enqueue order (a legal order for any set of streams whose
// cross-stream waits name events recorded earlier), so work really runs
// asynchronously to the host thread that enqueued it.  hipEventSynchronize /
// hipStreamSynchronize wait for the device thread to pass the operation in
// question.  A stream in capture mode records operations instead; a graph
// launch enqueues one operation that runs the graph's recorded operations
// through the executable graph object, each re-reading its arguments from
// memory when it runs, as a replayed kernel does.
//
// Fake kernels.  A batched launch advances each request whose step count in
// the tick exceeds k by min(tb, steps left) steps, adding 1 per step to every
// site of every field (reading buffer parity + k / tb, writing the other), so
// a request initialised to x0 holds exactly x0 + nsteps after its steps: the
// harness checks every result exactly.  Two-step launches exist for the same
// classes as in the library; the tiny class (small grids) runs all of a
// tick's steps in one launch.  Reductions sum field 0 (and field 1) in plain FP64 (the values
// are small integers, so the sums are exact).
//
// Accounting.  Model memory is counted when model_create / the stream-ordered
// release are called (program order = stream order on the scheduler's single
// stream); fake_model_bytes_peak() reports the high-water mark the harness
// compares with the server's budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pfmi.h"
#include "../../paper_2511_10508_amd/csrc/pf_runtime.h"

namespace {

struct Op {
    uint64_t seq;
    std::function<void()> fn;
};

struct Device {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Op> q;
    uint64_t next_seq = 1, done_seq = 0;
    bool stop = false;
    std::thread th;

    Device()
    {
        th = std::thread([this] { run(); });
    }
    ~Device()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
        th.join();
    }
    void run()
    {
        for (;;) {
            Op op;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [this] { return stop || !q.empty(); });
                if (q.empty()) return;
                op = std::move(q.front());
                q.pop_front();
            }
            if (op.fn) op.fn();
            {
                std::lock_guard<std::mutex> lk(mu);
                done_seq = op.seq;
            }
            cv_done.notify_all();
        }
    }
    uint64_t push(std::function<void()> fn)
    {
        uint64_t s;
        {
            std::lock_guard<std::mutex> lk(mu);
            s = next_seq++;
            q.push_back(Op{s, std::move(fn)});
        }
        cv_work.notify_one();
        return s;
    }
    void wait(uint64_t seq)
    {
        std::unique_lock<std::mutex> lk(mu);
        cv_done.wait(lk, [&] { return done_seq >= seq; });
    }
};

Device &dev()
{
    static Device d;
    return d;
}

struct FakeStream {
    std::mutex mu;
    bool capturing = false;
    std::vector<std::function<void()>> rec;
    uint64_t last = 0;  // sequence number of the last operation enqueued
};

struct FakeEvent {
    std::atomic<uint64_t> seq{0};
};

struct FakeGraph {
    std::vector<std::function<void()>> ops;
};

FakeStream g_null_stream;
FakeStream *S(hipStream_t s) { return s ? reinterpret_cast<FakeStream *>(s) : &g_null_stream; }

// Enqueue (or record, under capture) one operation on a stream.
void enqueue(hipStream_t st, std::function<void()> fn)
{
    FakeStream *s = S(st);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->capturing) {
        s->rec.push_back(std::move(fn));
        return;
    }
    s->last = dev().push(std::move(fn));
}

std::atomic<int64_t> g_model_bytes{0}, g_model_peak{0};

void charge(int64_t b)
{
    const int64_t now = g_model_bytes.fetch_add(b) + b;
    int64_t p = g_model_peak.load();
    while (now > p && !g_model_peak.compare_exchange_weak(p, now)) {}
}

}  // namespace

// Failure injection: with every = k > 0, every k-th model creation fails as
// an allocation failure would (PF_ERR_NOMEM, nothing allocated).
static std::atomic<int> g_fail_every{0}, g_creates{0};
extern "C" void fake_fail_creates(int every)
{
    g_fail_every.store(every);
    g_creates.store(0);
}
extern "C" int64_t fake_model_bytes_peak(void) { return g_model_peak.load(); }
extern "C" int64_t fake_model_bytes_live(void) { return g_model_bytes.load(); }
extern "C" void fake_reset_peak(void) { g_model_peak.store(g_model_bytes.load()); }
extern "C" void fake_device_idle(void)
{
    dev().wait(dev().push(nullptr));
}

// ------------------------------------------------------------- HIP runtime
extern "C" {

hipError_t hipSetDevice(int) { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "fake device error"; }
hipError_t hipMemGetInfo(size_t *fr, size_t *tot)
{
    *fr = (size_t)64 << 30;
    *tot = (size_t)64 << 30;
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t n)
{
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p)
{
    // a plain hipFree waits for the device
    fake_device_idle();
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned int)
{
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void *p)
{
    fake_device_idle();
    std::free(p);
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    *s = reinterpret_cast<hipStream_t>(new FakeStream());
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    if (s) {
        (void)hipStreamSynchronize(s);
        delete reinterpret_cast<FakeStream *>(s);
    }
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t st)
{
    FakeStream *s = S(st);
    uint64_t last;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->capturing) return hipErrorStreamCaptureUnsupported;
        last = s->last;
    }
    dev().wait(last);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int)
{
    *e = reinterpret_cast<hipEvent_t>(new FakeEvent());
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = reinterpret_cast<hipEvent_t>(new FakeEvent());
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    // a fixed figure per operation between the events: timing is not modelled
    const uint64_t sa = reinterpret_cast<FakeEvent *>(a)->seq.load();
    const uint64_t sb = reinterpret_cast<FakeEvent *>(b)->seq.load();
    *ms = 0.01f * (float)(sb > sa ? sb - sa : 0);
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete reinterpret_cast<FakeEvent *>(e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t st)
{
    FakeStream *s = S(st);
    FakeEvent *ev = reinterpret_cast<FakeEvent *>(e);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->capturing) return hipErrorStreamCaptureUnsupported;  // the scheduler records outside captures
    s->last = dev().push(nullptr);
    ev->seq.store(s->last);
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    dev().wait(reinterpret_cast<FakeEvent *>(e)->seq.load());
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int)
{
    // one in-order device queue: the event's work precedes everything after it
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t st)
{
    enqueue(st, [=] { std::memcpy(dst, src, n); });
    return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t w,
                            size_t h, hipMemcpyKind, hipStream_t st)
{
    enqueue(st, [=] {
        for (size_t i = 0; i < h; ++i)
            std::memcpy(static_cast<char *>(dst) + i * dpitch,
                        static_cast<const char *>(src) + i * spitch, w);
    });
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode)
{
    FakeStream *s = S(st);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->capturing) return hipErrorIllegalState;
    s->capturing = true;
    s->rec.clear();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t st, hipGraph_t *g)
{
    FakeStream *s = S(st);
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->capturing) return hipErrorIllegalState;
    s->capturing = false;
    FakeGraph *fg = new FakeGraph();
    fg->ops.swap(s->rec);
    *g = reinterpret_cast<hipGraph_t>(fg);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ex, hipGraph_t g, hipGraphNode_t *, char *, size_t)
{
    FakeGraph *c = new FakeGraph(*reinterpret_cast<FakeGraph *>(g));
    *ex = reinterpret_cast<hipGraphExec_t>(c);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g)
{
    delete reinterpret_cast<FakeGraph *>(g);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t g)
{
    delete reinterpret_cast<FakeGraph *>(g);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t g, hipStream_t st)
{
    // the operation runs the executable graph's nodes when the device reaches
    // it, through the graph object itself: a graph destroyed while a launch is
    // in flight is a heap use-after-free that AddressSanitizer reports
    FakeGraph *fg = reinterpret_cast<FakeGraph *>(g);
    enqueue(st, [fg] {
        for (auto &op : fg->ops) op();
    });
    return hipSuccess;
}

}  // extern "C"

// ---------------------------------------------------- library functions
namespace pf {

// the library's roctx ranges: nothing to record on the CPU
void trace_push(const char *) {}
void trace_pop() {}


static thread_local std::string g_err;

pf_status fail(pf_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}
pf_status hip_fail(hipError_t, const char *what)
{
    g_err = what;
    return PF_ERR_DEVICE;
}

pf_status check_desc(const pf_desc *d)
{
    if (!d || d->struct_size != sizeof(pf_desc)) return fail(PF_ERR_ARG, "bad descriptor");
    if (d->kind < 1 || d->kind > 3) return fail(PF_ERR_ARG, "fake: kinds 1..3");
    if (d->ndim < 1 || d->ndim > 3) return fail(PF_ERR_ARG, "bad ndim");
    for (int a = 0; a < 3; ++a)
        if (d->n[a] < 1 || d->n[a] > 4096) return fail(PF_ERR_ARG, "bad extent");
    if (d->nfields != (d->kind == 3 ? 2 : 1)) return fail(PF_ERR_ARG, "bad nfields");
    return PF_OK;
}
double stability_limit(const pf_desc *) { return 1.0; }
double volume(const pf_desc &d)
{
    double v = 1.0;
    for (int a = 0; a < d.ndim; ++a) v *= d.dx;
    return v;
}
int64_t reduce_partial_slots(int64_t) { return 1; }

bool time_block_available(const Launch &L)
{
    return (L.ndim == 2 && (L.r == 1 || L.r == 2)) || (L.ndim == 3 && L.r == 1);
}

// The fake tiny class: grids of at most 200 sites, so the harness's mix has
// both kinds of class.  A launch runs each request's steps of the tick.
bool tiny_available(const Launch &L, int64_t nx, int64_t ny, int64_t nz)
{
    return L.ndim >= 2 && nx * ny * nz <= 200;
}

template <typename T>
static void tiny_step(BatchTable<T> tb)
{
    const int32_t n = *tb.count;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t steps = tb.steps[i];
        if (steps <= 0) continue;
        const StepArgs<T> &a = tb.args[i];
        const int nf = a.buf[1][0] != a.buf[0][0] ? 2 : 1;
        const int64_t N = a.nx * a.ny * a.nz;
        for (int f = 0; f < nf; ++f)
            for (int64_t s = 0; s < N; ++s) a.buf[f][a.parity ^ 1][s] = a.buf[f][a.parity][s] + T(steps);
    }
}

hipError_t launch_tiny(const Launch &L, const void *table, int32_t blocks, hipStream_t s)
{
    if (blocks < 1) return hipErrorInvalidValue;
    if (L.fp32) {
        const BatchTable<float> t = *static_cast<const BatchTable<float> *>(table);
        enqueue(s, [t] { tiny_step<float>(t); });
    } else {
        const BatchTable<double> t = *static_cast<const BatchTable<double> *>(table);
        enqueue(s, [t] { tiny_step<double>(t); });
    }
    return hipSuccess;
}

// Work items of the fake plan: one per `chunk` rows (planes in 3D) per 16
// columns, so that the chunk changes the item count as in the real plans.
static int32_t fake_items(const pf_desc &d, int32_t chunk)
{
    const int64_t march = d.ndim == 2 ? d.n[1] : d.n[2];
    const int64_t chunks = (march + chunk - 1) / chunk;
    return (int32_t)std::max<int64_t>(1, chunks * ((d.n[0] + 15) / 16));
}

pf_status set_chunk(Model *m, int32_t chunk)
{
    m->clen = chunk > 0 ? chunk : 8;
    m->items = fake_items(m->desc, m->clen);
    m->a64.items = m->items;
    m->a32.items = m->items;
    return PF_OK;
}

static int64_t sites(const pf_desc &d) { return d.n[0] * d.n[1] * d.n[2]; }
static int64_t model_bytes(const pf_desc &d)
{
    const int64_t P = d.precision == PF_FP32 ? 4 : 8;
    return 2 * d.nfields * sites(d) * P + 3 * (int64_t)sizeof(double2) * (2 + 256 + 1);
}

Model::~Model() {}

pf_status model_create(const pf_desc *desc, void *stream, void *const *, int32_t, Model **out,
                       bool async_alloc)
{
    pf_status st = check_desc(desc);
    if (st != PF_OK) return st;
    const int every = g_fail_every.load();
    if (every > 0 && (g_creates.fetch_add(1) + 1) % every == 0)
        return fail(PF_ERR_NOMEM, "fake: injected allocation failure");
    Model *m = new Model();
    m->desc = *desc;
    m->nf = desc->nfields;
    m->fp32 = desc->precision == PF_FP32;
    m->L = Launch{desc->kind, desc->ndim, desc->order / 2, m->fp32 ? 1 : 0};
    m->stream = static_cast<hipStream_t>(stream);
    m->async_alloc = async_alloc;
    m->pitch = desc->n[0];
    m->elems = sites(*desc);
    const size_t P = m->fp32 ? 4 : 8;
    for (int f = 0; f < m->nf; ++f)
        for (int p = 0; p < 2; ++p) m->buf[f][p] = std::calloc((size_t)m->elems, P);
    m->part = static_cast<double2 *>(std::calloc(3 * 2, sizeof(double2)));
    m->pstride = 2;
    m->part2 = static_cast<double2 *>(std::calloc(3 * 256, sizeof(double2)));
    m->res = static_cast<double2 *>(std::calloc(3, sizeof(double2)));
    charge(model_bytes(*desc));
    m->family = 0;
    m->tb = async_alloc && time_block_available(m->L) ? 2 : 1;
    m->clen = 8;
    m->items = fake_items(*desc, m->clen);
    auto fill = [&](auto &a) {
        std::memset(&a, 0, sizeof(a));
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(a.buf[0][0])>>;
        for (int f = 0; f < kMaxFields; ++f)
            for (int p = 0; p < 2; ++p) a.buf[f][p] = static_cast<T *>(m->buf[f < m->nf ? f : 0][p]);
        a.nx = desc->n[0];
        a.ny = desc->n[1];
        a.nz = desc->n[2];
        a.pitch = m->pitch;
        a.plane = m->pitch * desc->n[1];
        a.items = m->items;
        a.part = m->part;
        a.pstride = m->pstride;
    };
    if (m->fp32)
        fill(m->a32);
    else
        fill(m->a64);
    *out = m;
    return PF_OK;
}

void model_release_async(Model *m)
{
    if (!m) return;
    charge(-model_bytes(m->desc));
    std::vector<void *> mem;
    for (int f = 0; f < m->nf; ++f)
        for (int p = 0; p < 2; ++p) mem.push_back(m->buf[f][p]);
    mem.push_back(m->part);
    mem.push_back(m->part2);
    mem.push_back(m->res);
    // stream-ordered free: after every operation already enqueued on the stream
    enqueue(m->stream, [mem] {
        for (void *p : mem) std::free(p);
    });
    delete m;
}

void pf_destroy_model(Model *m) { model_release_async(m); }

template <typename T>
static void init_t(Model *m, uint64_t seed)
{
    const T x0 = (T)(seed % 1000);
    T *f0 = static_cast<T *>(m->buf[0][m->parity]);
    T *f1 = m->nf > 1 ? static_cast<T *>(m->buf[1][m->parity]) : nullptr;
    const int64_t n = m->elems;
    enqueue(m->stream, [=] {
        for (int64_t i = 0; i < n; ++i) {
            f0[i] = x0;
            if (f1) f1[i] = x0 + 1;
        }
    });
}

pf_status init_fields(Model *m, int32_t, uint64_t seed, const double *, int32_t)
{
    if (m->fp32)
        init_t<float>(m, seed);
    else
        init_t<double>(m, seed);
    m->steps_done = 0;
    return PF_OK;
}

pf_status do_steps(Model *, int64_t) { return fail(PF_ERR_STATE, "fake: no solo models"); }

template <typename T>
static void batched_step(BatchTable<T> tb, int32_t k, int steps_per_launch)
{
    const int32_t n = *tb.count;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t left = tb.steps[i] - k;
        if (left <= 0) continue;
        const int adv = left < steps_per_launch ? left : steps_per_launch;
        const StepArgs<T> &a = tb.args[i];
        const int par = (a.parity + k / steps_per_launch) & 1;
        const int nf = a.buf[1][0] != a.buf[0][0] ? 2 : 1;
        const int64_t N = a.nx * a.ny * a.nz;
        for (int f = 0; f < nf; ++f) {
            const T *in = a.buf[f][par];
            T *out = a.buf[f][par ^ 1];
            for (int64_t s = 0; s < N; ++s) out[s] = in[s] + T(adv);
        }
    }
}

hipError_t launch_fused2d_batched(const Launch &L, const void *table, int32_t k, int32_t blocks, int tb,
                                  hipStream_t s)
{
    if (blocks < 1 || (tb != 1 && tb != 2) || (tb == 2 && !time_block_available(L)) || k % tb)
        return hipErrorInvalidValue;
    if (L.fp32) {
        const BatchTable<float> t = *static_cast<const BatchTable<float> *>(table);
        enqueue(s, [t, k, tb] { batched_step<float>(t, k, tb); });
    } else {
        const BatchTable<double> t = *static_cast<const BatchTable<double> *>(table);
        enqueue(s, [t, k, tb] { batched_step<double>(t, k, tb); });
    }
    return hipSuccess;
}

hipError_t launch_fused3d_batched(const Launch &L, const void *table, int32_t k, int32_t blocks, int tb,
                                  hipStream_t s)
{
    return launch_fused2d_batched(L, table, k, blocks, tb, s);
}

template <typename T>
static void reduce_t(StepArgs<T> a, int nf)
{
    const int64_t N = a.nx * a.ny * a.nz;
    double s0 = 0, s1 = 0;
    const T *f0 = a.buf[0][a.parity];
    const T *f1 = a.buf[nf - 1][a.parity];
    for (int64_t i = 0; i < N; ++i) {
        s0 += (double)f0[i];
        s1 += nf > 1 ? (double)f1[i] : 0.0;
    }
    a.part[0] = make_double2(s0, 0.0);
    a.part[a.pstride] = make_double2(s1, 0.0);
    a.part[2 * a.pstride] = make_double2(0.0, 0.0);
}

hipError_t launch_reduce_state(const Launch &L, const void *args, hipStream_t s)
{
    const int nf = L.kind == 3 ? 2 : 1;
    if (L.fp32) {
        const StepArgs<float> a = *static_cast<const StepArgs<float> *>(args);
        enqueue(s, [a, nf] { reduce_t<float>(a, nf); });
    } else {
        const StepArgs<double> a = *static_cast<const StepArgs<double> *>(args);
        enqueue(s, [a, nf] { reduce_t<double>(a, nf); });
    }
    return hipSuccess;
}

hipError_t launch_finalize(const double2 *part, int64_t pstride, int64_t, double2 *, double2 *out,
                           hipStream_t s)
{
    enqueue(s, [=] {
        for (int q = 0; q < kNumQ; ++q) out[q] = part[q * pstride];
    });
    return hipSuccess;
}

}  // namespace pf

extern "C" uint64_t pf_footprint_bytes(const pf_desc *d)
{
    if (pf::check_desc(d) != PF_OK) return 0;
    return (uint64_t)pf::model_bytes(*d);
}
extern "C" const char *fake_last_error(void) { return pf::g_err.c_str(); }
