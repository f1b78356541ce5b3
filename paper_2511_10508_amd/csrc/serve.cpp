// Serving engine: continuous batching of independent simulation requests.
//
// A scheduler thread owns one HIP stream.  Every tick it
//   1. admits queued requests in FIFO order while a slot is free and their
//      device footprint fits the HBM budget (allocation and initial
//      conditions are enqueued in stream order, no host synchronisation);
//   2. groups the running requests by kernel class (model, dimension,
//      stencil radius, precision) and uploads one work-item table per class;
//   3. launches, per class and on the class's own stream, a captured HIP
//      graph of the tick's chained persistent batched launches (one per step,
//      or one per two steps where the class has a two-step kernel; captured
//      once per class, table buffer and grid bucket); the class streams fork
//      from and join back into the scheduler stream, so the classes run
//      concurrently;
//   4. enqueues the final reductions of requests that finish in this tick.
// Ticks are pipelined two deep: tick i+1 is enqueued before the host waits
// for tick i, and requests that finished in tick i are retired (results
// visible to pf_server_poll) once its event completes.  Requests submitted
// while ticks run join at the next tick boundary.  The chunk length of each
// request comes from the serving autotuner (tune_served), per kernel class
// and size bucket.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/pfmi.h"
#include "pf_runtime.h"

namespace pf {

namespace {

constexpr int kPersist2D = 2048;  // workgroups of a persistent 2D batched launch
constexpr int kPersist3D = 512;   // workgroups of a persistent 3D batched launch
constexpr int kMaxGraphs = 256;  // cached executable graphs (cleared when full; PFMI_SERVER_MAX_GRAPHS)

enum ReqState { QUEUED = 0, ADMITTING = 1, RUNNING = 2, FINISHED = 3 };

struct Req {
    uint64_t ticket = 0;
    pf_desc desc{};
    int32_t ic = 0;
    uint64_t seed = 0;
    std::vector<double> icp;
    int64_t nsteps = 0, done = 0;
    Model *m = nullptr;
    int state = QUEUED;
    int32_t status = PF_OK;
    bool cancel = false, released = false, reported = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
    uint64_t footprint = 0;
    int64_t finish_tick = -1;
    int cls = -1;            // batched class, -1 = stepped on its own
    double2 *pinned = nullptr;  // final reductions (slot of the server's pinned pool)
    int slot = -1;
    pf_result res{};
};

struct ClassKey {
    int kind, ndim, r, fp32, tiny;
    bool operator<(const ClassKey &o) const
    {
        return std::tie(kind, ndim, r, fp32, tiny) < std::tie(o.kind, o.ndim, o.r, o.fp32, o.tiny);
    }
};

// Steps a tiny-grid request may run per tick, in units of steps_per_tick: its
// launch stays short (a few ms for the largest tiny grid) next to a tick of
// the other classes, and it finishes in a few ticks.
constexpr int kTinyTickFactor = 16;

// Device and pinned host buffers of one class's work-item tables, double
// buffered across pipelined ticks.
struct ClassTables {
    ClassKey key{};
    Launch L{};
    size_t args_bytes = 0;
    void *dev[2] = {nullptr, nullptr};   // [args | count | item_start | steps]
    void *host[2] = {nullptr, nullptr};
    int32_t n[2] = {0, 0};
    int32_t blocks[2] = {1, 1};          // persistent grid of this tick (power of two)
    int tb = 1;                          // steps per batched launch (2: two-step kernels)
    bool tiny = false;                   // whole grid in LDS, one launch per tick
    void *tune_dev = nullptr, *tune_host = nullptr;  // the autotuner's table (same layout)
    hipStream_t stream = nullptr;        // graph branch of this class
    hipEvent_t join = nullptr;
};

}  // namespace

struct Server {
    int device = 0;
    uint64_t budget = 0, used = 0;
    int max_slots = 0;
    int spt = 64;
    int max_graphs = kMaxGraphs;
    bool two_step = true;  // two-step batched kernels where the class has them (PFMI_SERVER_TWO_STEP)
    bool tune = true;      // serving autotuner (PFMI_SERVER_TUNE=off disables it)
    hipStream_t stream = nullptr, copy_stream = nullptr;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::map<uint64_t, Req *> all;
    std::vector<Req *> to_free;
    uint64_t next_ticket = 1;
    int64_t unfinished = 0;
    bool stop = false;
    std::thread worker;

    double2 *pinned_pool = nullptr;  // max_slots x kNumQ result pairs (host-pinned)
    std::vector<int> free_slots;

    std::map<ClassKey, int> class_index;
    std::vector<ClassTables> classes;
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;  // (class, set, steps, grid) -> graph
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr;
    hipEvent_t tev[2] = {nullptr, nullptr};  // autotuner timing
    // serving autotuner: chunk per (class, log2 of each extent)
    std::map<std::tuple<int, int, int, int>, int32_t> tuned;
    // written by the scheduler thread, read by pf_server_stats from any thread
    std::atomic<int64_t> tick{0}, launches{0}, captures{0}, replays{0};
    std::string fatal;  // guarded by mu (set_fatal)

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

// Record a device failure of the scheduler (under the lock, so that submit,
// poll and drain, which read it from other threads, see a whole string) and
// wake drain, which would otherwise wait out its timeout.
static void set_fatal(Server *s, const std::string &msg)
{
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal.empty()) s->fatal = msg;
    s->done_cv.notify_all();
}

static int class_of(Server *s, const Model *m)
{
    const bool tiny = tiny_available(m->L, m->desc.n[0], m->desc.n[1], m->desc.n[2]);
    if (m->family != 0 && !tiny) return -1;
    ClassKey k{m->L.kind, m->L.ndim, m->L.r, m->L.fp32, tiny ? 1 : 0};
    auto it = s->class_index.find(k);
    if (it != s->class_index.end()) return it->second;
    ClassTables t;
    t.key = k;
    t.L = m->L;
    t.tb = m->tb;  // served models are planned for two-step sweeps where the class has them
    t.tiny = tiny;
    const size_t argsz = m->fp32 ? sizeof(StepArgs<float>) : sizeof(StepArgs<double>);
    t.args_bytes = argsz * s->max_slots;
    const size_t total = t.args_bytes + sizeof(int32_t) * (2 * s->max_slots + 2);
    for (int b = 0; b < 2; ++b) {
        if (hipMalloc(&t.dev[b], total) != hipSuccess) return -1;
        if (hipHostMalloc(&t.host[b], total, hipHostMallocDefault) != hipSuccess) return -1;
    }
    if (hipStreamCreateWithFlags(&t.stream, hipStreamNonBlocking) != hipSuccess) return -1;
    if (hipEventCreateWithFlags(&t.join, hipEventDisableTiming) != hipSuccess) return -1;
    const int idx = (int)s->classes.size();
    s->classes.push_back(t);
    s->class_index[k] = idx;
    return idx;
}

static void free_req(Server *s, Req *r)
{
    if (r->m) {
        model_release_async(r->m);
        r->m = nullptr;
    }
    if (r->slot >= 0) {
        s->free_slots.push_back(r->slot);
        r->slot = -1;
        r->pinned = nullptr;
    }
    s->used -= std::min(s->used, r->footprint);
    r->footprint = 0;
}

// Fill the request's result from its pinned reductions.
static void fill_result(Req *r)
{
    pf_result &o = r->res;
    o.ticket = r->ticket;
    o.status = r->status;
    o.t_submit = r->t_submit;
    o.t_admit = r->t_admit;
    o.t_done = r->t_done;
    o.steps_done = r->done;
    if (r->status == PF_OK && r->pinned) {
        const double vol = volume(r->desc);
        const double2 *q = r->pinned;
        o.mass[0] = (q[0].x + q[0].y) * vol;
        if (nfields_kind(r->desc.kind) == 2) {
            o.mass[1] = (q[1].x + q[1].y) * vol;
            o.energy = 0.0;
        } else {
            o.mass[1] = 0.0;
            o.energy = (q[1].x + q[1].y) * vol;
        }
        o.nonfinite = (int64_t)q[2].x;
    }
}

// Steps a request of class t runs in a tick of S steps (at most).
static int64_t tick_steps(const ClassTables &t, int S) { return t.tiny ? (int64_t)kTinyTickFactor * S : S; }

// One batched launch over the table at `dev` (layout [args | count |
// item_start | steps], max_slots entries): step k of the tick.
static hipError_t launch_table(const ClassTables &t, int max_slots, void *dev, int32_t k, int32_t blocks,
                               hipStream_t st)
{
    char *d = static_cast<char *>(dev);
    int32_t *ints = reinterpret_cast<int32_t *>(d + t.args_bytes);
    if (t.tiny) {
        if (t.L.fp32) {
            BatchTable<float> tb{reinterpret_cast<StepArgs<float> *>(d), ints, ints + 1, ints + 1 + max_slots + 1};
            return launch_tiny(t.L, &tb, blocks, st);
        }
        BatchTable<double> tb{reinterpret_cast<StepArgs<double> *>(d), ints, ints + 1, ints + 1 + max_slots + 1};
        return launch_tiny(t.L, &tb, blocks, st);
    }
    if (t.L.fp32) {
        BatchTable<float> tb{reinterpret_cast<StepArgs<float> *>(d), ints, ints + 1, ints + 1 + max_slots + 1};
        return t.L.ndim == 2 ? launch_fused2d_batched(t.L, &tb, k, blocks, t.tb, st)
                             : launch_fused3d_batched(t.L, &tb, k, blocks, t.tb, st);
    }
    BatchTable<double> tb{reinterpret_cast<StepArgs<double> *>(d), ints, ints + 1, ints + 1 + max_slots + 1};
    return t.L.ndim == 2 ? launch_fused2d_batched(t.L, &tb, k, blocks, t.tb, st)
                         : launch_fused3d_batched(t.L, &tb, k, blocks, t.tb, st);
}

// Launch the S batched steps of one class (buffer set `set`) on `st`: one
// launch per step, or per two steps with the class's two-step kernels.
static hipError_t launch_class(Server *s, int c, int set, int S, hipStream_t st)
{
    ClassTables &t = s->classes[c];
    if (t.tiny) {  // one launch runs every step of the tick
        hipError_t e = launch_table(t, s->max_slots, t.dev[set], 0, t.blocks[set], st);
        if (e == hipSuccess) s->launches++;
        return e;
    }
    for (int k = 0; k < S; k += t.tb) {
        hipError_t e = launch_table(t, s->max_slots, t.dev[set], k, t.blocks[set], st);
        if (e != hipSuccess) return e;
        s->launches++;
    }
    return hipSuccess;
}

// Fill a host table (layout of launch_table) with the given models, each
// stepping steps[i] steps from its current parity; returns the work items.
static int32_t fill_table(const ClassTables &t, int max_slots, void *host, const std::vector<Model *> &ms,
                          const std::vector<int32_t> &steps)
{
    char *h = static_cast<char *>(host);
    int32_t *ints = reinterpret_cast<int32_t *>(h + t.args_bytes);
    ints[0] = (int32_t)ms.size();
    int32_t *start = ints + 1;
    int32_t *st = start + max_slots + 1;
    int32_t acc = 0;
    for (size_t i = 0; i < ms.size(); ++i) {
        const Model *m = ms[i];
        if (m->fp32) {
            StepArgs<float> a = m->a32;
            a.parity = m->parity;
            reinterpret_cast<StepArgs<float> *>(host)[i] = a;
        } else {
            StepArgs<double> a = m->a64;
            a.parity = m->parity;
            reinterpret_cast<StepArgs<double> *>(host)[i] = a;
        }
        start[i] = acc;
        acc += m->items;
        st[i] = steps[i];
    }
    start[ms.size()] = acc;
    return acc;
}

// Persistent grid for `items` work items: enough workgroups for every item,
// rounded up to a power of two (so that few distinct graphs are needed).
static int32_t persistent_blocks(const ClassTables &t, int64_t items)
{
    const int64_t need = t.L.ndim == 2 ? (items + kWaves2D - 1) / kWaves2D : items;
    const int32_t cap = t.L.ndim == 2 ? kPersist2D : kPersist3D;
    if (t.tiny) {  // one workgroup per request, at most one per CU
        int32_t b = 1;
        while (b < items && b < 256) b <<= 1;
        return b;
    }
    int32_t b = 1;
    while (b < need && b < cap) b <<= 1;
    return b;
}

// Upload a filled host table of n entries to `dev` on the scheduler stream.
static hipError_t upload_table(Server *s, const ClassTables &t, const void *host, void *dev, size_t n)
{
    const size_t argsz = t.L.fp32 ? sizeof(StepArgs<float>) : sizeof(StepArgs<double>);
    hipError_t e = hipMemcpyAsync(dev, host, argsz * n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(static_cast<char *>(dev) + t.args_bytes, static_cast<const char *>(host) + t.args_bytes,
                           sizeof(int32_t) * (2 * s->max_slots + 2), hipMemcpyHostToDevice, s->stream);
    return e;
}

// Serving autotuner.  The chunk length (rows or planes marched per work item)
// of each kernel class and size bucket (log2 of every extent) is chosen on
// the first request of the bucket: for every candidate chunk the class's
// batched kernel is timed on that request's table entry alone, and the chunk
// with the least time per site and step is kept for the bucket (its later
// requests take it at admission).  The timed launches read the request's
// current buffer and write its other one, which holds no state, so the
// request is unchanged.  A failure leaves the library's default chunk.
// (Timing the request's entry replicated until the grid is full, as a busy
// tick is, chose long chunks whose single work items outlast the rest of a
// tick, and measured slower; PFMI_SERVER_TUNE=off keeps the default chunk.)
static void tune_served(Server *s, Req *r)
{
    Model *m = r->m;
    if (r->cls < 0 || !s->tune) return;
    ClassTables &t = s->classes[r->cls];
    if (t.tiny) return;
    const pf_desc &d = m->desc;
    auto lg = [](int64_t v) { int b = 0; while ((1ll << (b + 1)) <= v) ++b; return b; };
    const auto key = std::make_tuple(r->cls, lg(d.n[0]), lg(d.n[1]), lg(d.n[2]));
    auto it = s->tuned.find(key);
    if (it != s->tuned.end()) {
        if (it->second != m->clen) set_chunk(m, it->second);
        return;
    }
    const int32_t keep = m->clen;
    int32_t best = keep;
    if (!t.tune_dev) {
        const size_t total = t.args_bytes + sizeof(int32_t) * (2 * s->max_slots + 2);
        if (hipMalloc(&t.tune_dev, total) != hipSuccess ||
            hipHostMalloc(&t.tune_host, total, hipHostMallocDefault) != hipSuccess) {
            s->tuned[key] = keep;
            return;
        }
    }
    const int64_t march = d.ndim == 2 ? d.n[1] : d.n[2];
    const int64_t sites = d.n[0] * d.n[1] * d.n[2];
    double best_t = 1e300;
    int32_t prev = -1;
    for (int32_t c : {8, 16, 32, 64, 128, 256, 512}) {
        const int32_t cc = (int32_t)std::min<int64_t>(c, march);
        if (cc == prev) continue;
        prev = cc;
        if (set_chunk(m, cc) != PF_OK || m->family != 0) break;
        std::vector<Model *> ms(1, m);
        std::vector<int32_t> st(1, (int32_t)t.tb);
        const int32_t items = fill_table(t, s->max_slots, t.tune_host, ms, st);
        const int32_t blocks = persistent_blocks(t, items);
        hipError_t e = upload_table(s, t, t.tune_host, t.tune_dev, ms.size());
        if (e == hipSuccess) e = launch_table(t, s->max_slots, t.tune_dev, 0, blocks, s->stream);
        if (e == hipSuccess) e = hipEventRecord(s->tev[0], s->stream);
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
            e = launch_table(t, s->max_slots, t.tune_dev, 0, blocks, s->stream);
        if (e == hipSuccess) e = hipEventRecord(s->tev[1], s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(s->tev[1]);
        float ms_t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms_t, s->tev[0], s->tev[1]);
        if (e != hipSuccess) break;
        s->launches += 4;
        const double per = (double)ms_t / ((double)sites * t.tb);
        if (per < best_t) {
            best_t = per;
            best = cc;
        }
    }
    if (set_chunk(m, best) != PF_OK) (void)set_chunk(m, keep);
    s->tuned[key] = m->clen;
}

// The graph of S chained batched launches of class c for table buffer `set`
// at this tick's grid bucket, captured on the class stream the first time.
static std::vector<int64_t> graph_key(Server *s, int c, int set, int S)
{
    return {c, set, S, s->classes[c].blocks[set]};
}

static hipError_t class_graph(Server *s, int c, int set, int S, hipGraphExec_t *out)
{
    ClassTables &t = s->classes[c];
    const std::vector<int64_t> key = graph_key(s, c, set, S);
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) {
        s->replays++;
        *out = it->second;
        return hipSuccess;
    }
    hipError_t e = hipStreamBeginCapture(t.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t le = launch_class(s, c, set, S, t.stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(t.stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    s->graphs.emplace(key, ex);
    s->captures++;
    *out = ex;
    return hipSuccess;
}

// Runs the classes' graphs concurrently: each class stream waits for the
// scheduler stream (tables uploaded), launches its graph and is joined back.
static hipError_t run_classes(Server *s, const std::vector<int> &cls, int set, int S)
{
    int missing = 0;
    for (int c : cls) missing += s->graphs.count(graph_key(s, c, set, S)) ? 0 : 1;
    if (missing && (int)s->graphs.size() + missing > s->max_graphs) {
        // the cache is full: clear it before this tick takes any graph from it.
        // Graphs of the previous tick may still run (they are joined into the
        // scheduler stream): wait for them before destroying any.
        hipError_t se = hipStreamSynchronize(s->stream);
        if (se != hipSuccess) return se;
        for (auto &g : s->graphs) (void)hipGraphExecDestroy(g.second);
        s->graphs.clear();
    }
    std::vector<hipGraphExec_t> ex(cls.size());
    for (size_t i = 0; i < cls.size(); ++i) {
        hipError_t e = class_graph(s, cls[i], set, S, &ex[i]);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(s->fork, s->stream);
    for (size_t i = 0; i < cls.size() && e == hipSuccess; ++i) {
        ClassTables &t = s->classes[cls[i]];
        e = hipStreamWaitEvent(t.stream, s->fork, 0);
        if (e == hipSuccess) e = hipGraphLaunch(ex[i], t.stream);
        if (e == hipSuccess) e = hipEventRecord(t.join, t.stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, t.join, 0);
    }
    return e;
}

// Enqueue one tick.  Returns false on a device error (recorded in fatal).
static bool enqueue_tick(Server *s, std::vector<Req *> &run, int set)
{
    const int S = s->spt;
    std::vector<std::vector<Req *>> by_class(s->classes.size());
    std::vector<Req *> solo;
    for (Req *r : run) {
        if (r->cls >= 0)
            by_class[r->cls].push_back(r);
        else
            solo.push_back(r);
    }
    std::vector<int> cls;
    for (size_t c = 0; c < by_class.size(); ++c) {
        ClassTables &t = s->classes[c];
        auto &v = by_class[c];
        t.n[set] = (int32_t)v.size();
        if (v.empty()) continue;
        cls.push_back((int)c);
        std::vector<Model *> ms;
        std::vector<int32_t> steps;
        for (Req *r : v) {
            ms.push_back(r->m);
            steps.push_back((int32_t)std::min<int64_t>(tick_steps(t, S), r->nsteps - r->done));
        }
        const int32_t items = fill_table(t, s->max_slots, t.host[set], ms, steps);
        t.blocks[set] = persistent_blocks(t, t.tiny ? (int64_t)ms.size() : items);
        hipError_t e = upload_table(s, t, t.host[set], t.dev[set], ms.size());
        if (e != hipSuccess) {
            set_fatal(s, std::string("table upload: ") + hipGetErrorString(e));
            return false;
        }
    }
    if (!cls.empty()) {
        hipError_t e = run_classes(s, cls, set, S);
        if (e != hipSuccess) {
            set_fatal(s, std::string("batched launch: ") + hipGetErrorString(e));
            return false;
        }
    }
    for (Req *r : solo) {
        const int64_t n = std::min<int64_t>(S, r->nsteps - r->done);
        if (do_steps(r->m, n) != PF_OK) {
            r->status = PF_ERR_DEVICE;
            r->nsteps = r->done;  // stop it
            continue;
        }
        r->done += n;  // do_steps advanced the model's parity and step count
    }
    for (size_t c = 0; c < by_class.size(); ++c)
        for (Req *r : by_class[c]) {
            // every launch that advanced the request flipped its buffers once
            const ClassTables &t = s->classes[c];
            const int64_t n = std::min<int64_t>(tick_steps(t, S), r->nsteps - r->done);
            const int64_t flips = t.tiny ? (n > 0 ? 1 : 0) : (n + t.tb - 1) / t.tb;
            r->m->parity ^= (int)(flips & 1);
            r->m->steps_done += n;
            r->done += n;
        }
    // final reductions of requests that finish in this tick
    for (Req *r : run) {
        if (r->done < r->nsteps) continue;
        Model *m = r->m;
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
        hipError_t e = launch_reduce_state(m->L, ap, s->stream);
        if (e == hipSuccess)
            e = launch_finalize(m->part, m->pstride, reduce_partial_slots(N), m->part2, m->res, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->pinned, m->res, sizeof(double2) * kNumQ, hipMemcpyDeviceToHost, s->stream);
        if (e != hipSuccess) r->status = PF_ERR_DEVICE;
        r->finish_tick = s->tick;
    }
    return true;
}

static void retire(Server *s, int64_t tick)
{
    std::lock_guard<std::mutex> lk(s->mu);
    const double t = s->now();
    std::vector<Req *> keep;
    for (Req *r : s->active) {
        if (r->finish_tick >= 0 && r->finish_tick <= tick) {
            r->state = FINISHED;
            r->t_done = t;
            fill_result(r);
            s->unfinished--;
        } else {
            keep.push_back(r);
        }
    }
    s->active.swap(keep);
    s->done_cv.notify_all();
}

static void worker_main(Server *s)
{
    (void)hipSetDevice(s->device);
    bool pending[2] = {false, false};
    while (true) {
        std::vector<Req *> admitted;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (Req *r : s->to_free) {
                free_req(s, r);
                delete r;
            }
            s->to_free.clear();
            if (s->stop) break;
            // FIFO admission by footprint and slots
            // (finished requests hold their result slot until released)
            while (!s->queue.empty() && (int)s->active.size() + (int)admitted.size() < s->max_slots &&
                   !s->free_slots.empty()) {
                Req *r = s->queue.front();
                if (s->used + r->footprint > s->budget) break;
                s->queue.pop_front();
                s->used += r->footprint;
                r->slot = s->free_slots.back();
                s->free_slots.pop_back();
                r->pinned = s->pinned_pool + (size_t)r->slot * kNumQ;
                r->state = ADMITTING;  // no longer cancellable as queued
                admitted.push_back(r);
            }
            if (admitted.empty() && s->active.empty() && !pending[0] && !pending[1]) {
                s->cv.wait_for(lk, std::chrono::milliseconds(50));
                continue;
            }
        }
        for (Req *r : admitted) {
            Model *m = nullptr;
            pf_status st = model_create(&r->desc, s->stream, nullptr, 0, &m, true);
            if (st == PF_OK)
                st = init_fields(m, r->ic, r->seed, r->icp.data(), (int32_t)r->icp.size());
            std::lock_guard<std::mutex> lk(s->mu);
            r->m = m;
            r->t_admit = s->now();
            if (st != PF_OK) {
                r->status = st;
                r->state = FINISHED;
                r->t_done = r->t_admit;
                fill_result(r);
                s->unfinished--;
                s->done_cv.notify_all();
                continue;
            }
            if (!s->two_step && m->tb == 2) {
                m->tb = 1;
                (void)set_chunk(m, m->clen);
            }
            r->cls = class_of(s, m);
            r->state = RUNNING;
            s->active.push_back(r);  // a cancel during admission takes effect at the next tick
        }
        // tile of each newly admitted request (the scheduler thread owns its model)
        for (Req *r : admitted) {
            if (r->m && r->state == RUNNING) tune_served(s, r);
        }
        std::vector<Req *> run;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (Req *r : s->active) {
                if (r->finish_tick >= 0) continue;  // finished, waiting for retirement
                if (r->cancel) {
                    r->status = PF_ERR_STATE;
                    r->finish_tick = s->tick;
                    continue;
                }
                run.push_back(r);
            }
        }
        const int set = (int)(s->tick & 1);
        if (!run.empty()) {
            TraceRange range("pf_server tick");
            if (!enqueue_tick(s, run, set)) break;
        }
        (void)hipEventRecord(s->ev[set], s->stream);
        pending[set] = true;
        // wait for the previous tick, retire what finished in it
        const int prev = set ^ 1;
        if (pending[prev]) {
            (void)hipEventSynchronize(s->ev[prev]);
            pending[prev] = false;
            retire(s, s->tick - 1);
        }
        if (run.empty()) {
            (void)hipEventSynchronize(s->ev[set]);
            pending[set] = false;
            retire(s, s->tick);
        }
        s->tick++;
    }
    (void)hipStreamSynchronize(s->stream);
}

}  // namespace pf

using namespace pf;
#define PF_API extern "C" __attribute__((visibility("default")))

static Server *SV(pf_server *s) { return reinterpret_cast<Server *>(s); }

PF_API pf_status pf_server_create(int32_t device, uint64_t hbm_budget, int32_t max_slots,
                                  int32_t steps_per_tick, pf_server **out)
{
    if (!out) return fail(PF_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 4096) return fail(PF_ERR_ARG, "max_slots must be 1..4096");
    if (steps_per_tick < 0 || steps_per_tick > 4096) return fail(PF_ERR_ARG, "steps_per_tick must be 0..4096");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    Server *s = new Server();
    s->device = device;
    s->max_slots = max_slots;
    s->spt = steps_per_tick ? steps_per_tick : 64;
    if (const char *g = std::getenv("PFMI_SERVER_MAX_GRAPHS")) s->max_graphs = std::max(1, std::atoi(g));
    if (const char *g = std::getenv("PFMI_SERVER_TWO_STEP")) s->two_step = std::atoi(g) != 0;
    if (const char *g = std::getenv("PFMI_SERVER_TUNE")) s->tune = std::string(g) != "off";
    s->t0 = std::chrono::steady_clock::now();
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        e = hipMemGetInfo(&fr, &tot);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e, "hipMemGetInfo");
        }
        hbm_budget = (uint64_t)(0.9 * (double)fr);
    }
    s->budget = hbm_budget;
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev[1], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&s->tev[0]);
    if (e == hipSuccess) e = hipEventCreate(&s->tev[1]);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&s->pinned_pool, sizeof(double2) * kNumQ * (size_t)max_slots,
                          hipHostMallocDefault);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "server stream/event/pinned pool");
    }
    for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->worker = std::thread(worker_main, s);
    *out = reinterpret_cast<pf_server *>(s);
    return PF_OK;
}

PF_API pf_status pf_server_submit(pf_server *ss, const pf_desc *desc, int32_t ic, uint64_t seed,
                                  const double *ic_params, int32_t n_ic_params, int64_t nsteps,
                                  uint64_t *ticket)
{
    Server *s = SV(ss);
    if (!s || !ticket) return fail(PF_ERR_ARG, "NULL argument");
    pf_status st = check_desc(desc);
    if (st != PF_OK) return st;
    if (nsteps < 0) return fail(PF_ERR_ARG, "nsteps must be >= 0");
    if (!(desc->flags & PF_ALLOW_UNSTABLE) && desc->dt > stability_limit(desc))
        return fail(PF_ERR_UNSTABLE, "dt exceeds the explicit-stability limit");
    if (desc->flags & (PF_USE_GRAPH | PF_REDUCE_EACH_STEP))
        return fail(PF_ERR_ARG, "served requests take no PF_USE_GRAPH / PF_REDUCE_EACH_STEP");
    if (desc->ndim == 1 || desc->kind == PF_MH || (desc->flags & (PF_BIHARMONIC_DIRECT | PF_SPECTRAL)))
        return fail(PF_ERR_UNSUPPORTED, "the server batches 2D and 3D finite-difference grids "
                                        "with the composed biharmonic only");
    if (n_ic_params < 0 || n_ic_params > 8 || (n_ic_params && !ic_params))
        return fail(PF_ERR_ARG, "bad initial-condition parameters");
    const uint64_t fp = pf_footprint_bytes(desc);
    if (fp > s->budget) return fail(PF_ERR_NOMEM, "request footprint exceeds the server's HBM budget");
    Req *r = new Req();
    r->desc = *desc;
    r->ic = ic;
    r->seed = seed;
    r->icp.assign(ic_params, ic_params + n_ic_params);
    r->nsteps = nsteps;
    r->footprint = fp;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->fatal.empty()) return fail(PF_ERR_DEVICE, s->fatal);
    r->ticket = s->next_ticket++;
    r->t_submit = s->now();
    s->queue.push_back(r);
    s->all[r->ticket] = r;
    s->unfinished++;
    *ticket = r->ticket;
    s->cv.notify_all();
    return PF_OK;
}

PF_API pf_status pf_server_poll(pf_server *ss, pf_result *out, int32_t max, int32_t *n)
{
    Server *s = SV(ss);
    if (!s || !n || (max > 0 && !out)) return fail(PF_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t k = 0;
    for (auto &kv : s->all) {
        if (k >= max) break;
        Req *r = kv.second;
        if (r->state == FINISHED && !r->reported) {
            out[k++] = r->res;
            r->reported = true;
        }
    }
    *n = k;
    if (!s->fatal.empty()) return fail(PF_ERR_DEVICE, s->fatal);
    return PF_OK;
}

PF_API pf_status pf_server_fetch(pf_server *ss, uint64_t ticket, int32_t field, double *host,
                                 int64_t count)
{
    Server *s = SV(ss);
    if (!s || !host) return fail(PF_ERR_ARG, "NULL argument");
    Model *m;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return fail(PF_ERR_NOTFOUND, "unknown ticket");
        Req *r = it->second;
        if (r->state != FINISHED || r->released || !r->m) return fail(PF_ERR_STATE, "request not finished or released");
        m = r->m;
    }
    if (field < 0 || field >= m->nf) return fail(PF_ERR_ARG, "field index out of range");
    const pf_desc &d = m->desc;
    const int64_t N = d.n[0] * d.n[1] * d.n[2];
    if (count != N) return fail(PF_ERR_ARG, "count must equal the number of sites");
    const size_t ts = m->fp32 ? 4 : 8;
    std::vector<unsigned char> stage(ts * (size_t)N);
    hipError_t e = hipMemcpy2DAsync(stage.data(), ts * d.n[0], m->buf[field][m->parity], ts * m->pitch,
                                    ts * d.n[0], d.n[1] * d.n[2], hipMemcpyDeviceToHost, s->copy_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->copy_stream);
    if (e != hipSuccess) return hip_fail(e, "fetch");
    for (int64_t i = 0; i < N; ++i)
        host[i] = m->fp32 ? (double)reinterpret_cast<float *>(stage.data())[i]
                          : reinterpret_cast<double *>(stage.data())[i];
    return PF_OK;
}

PF_API pf_status pf_server_release(pf_server *ss, uint64_t ticket)
{
    Server *s = SV(ss);
    if (!s) return fail(PF_ERR_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(PF_ERR_NOTFOUND, "unknown ticket");
    Req *r = it->second;
    if (r->state != FINISHED) return fail(PF_ERR_STATE, "request not finished");
    s->all.erase(it);
    r->released = true;
    s->to_free.push_back(r);  // freed by the scheduler, in stream order
    s->cv.notify_all();
    return PF_OK;
}

PF_API pf_status pf_server_cancel(pf_server *ss, uint64_t ticket)
{
    Server *s = SV(ss);
    if (!s) return fail(PF_ERR_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(PF_ERR_NOTFOUND, "unknown ticket");
    Req *r = it->second;
    if (r->state == QUEUED) {
        s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), r), s->queue.end());
        r->footprint = 0;  // never admitted: nothing was charged to the budget
        r->status = PF_ERR_STATE;
        r->state = FINISHED;
        r->t_done = r->t_admit = s->now();
        fill_result(r);
        s->unfinished--;
        s->done_cv.notify_all();
    } else if (r->state == RUNNING || r->state == ADMITTING) {
        r->cancel = true;
    }
    return PF_OK;
}

PF_API pf_status pf_server_drain(pf_server *ss, double timeout_s)
{
    Server *s = SV(ss);
    if (!s) return fail(PF_ERR_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::microseconds((int64_t)(timeout_s * 1e6));
    while (s->unfinished > 0 && s->fatal.empty()) {
        if (s->done_cv.wait_until(lk, until) == std::cv_status::timeout && s->unfinished > 0)
            return fail(PF_ERR_BUSY, "drain timed out");
    }
    if (!s->fatal.empty()) return fail(PF_ERR_DEVICE, s->fatal);
    return PF_OK;
}

PF_API pf_status pf_server_stats(pf_server *ss, int64_t *ticks, int64_t *launches,
                                 int64_t *captures, int64_t *replays)
{
    Server *s = SV(ss);
    if (!s) return fail(PF_ERR_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticks) *ticks = s->tick.load();
    if (launches) *launches = s->launches.load();
    if (captures) *captures = s->captures.load();
    if (replays) *replays = s->replays.load();
    return PF_OK;
}

PF_API void pf_server_destroy(pf_server *ss)
{
    Server *s = SV(ss);
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    // every request is in `all` (queued, running or finished) until released,
    // then in to_free: each is freed and deleted exactly once
    s->queue.clear();
    s->active.clear();
    for (auto &kv : s->all) free_req(s, kv.second), delete kv.second;
    s->all.clear();
    for (Req *r : s->to_free) free_req(s, r), delete r;
    s->to_free.clear();
    (void)hipStreamSynchronize(s->stream);
    for (auto &g : s->graphs) (void)hipGraphExecDestroy(g.second);
    for (auto &t : s->classes) {
        for (int b = 0; b < 2; ++b) {
            (void)hipFree(t.dev[b]);
            (void)hipHostFree(t.host[b]);
        }
        if (t.tune_dev) (void)hipFree(t.tune_dev);
        if (t.tune_host) (void)hipHostFree(t.tune_host);
        (void)hipStreamDestroy(t.stream);
        (void)hipEventDestroy(t.join);
    }
    (void)hipHostFree(s->pinned_pool);
    (void)hipEventDestroy(s->fork);
    (void)hipEventDestroy(s->tev[0]);
    (void)hipEventDestroy(s->tev[1]);
    (void)hipEventDestroy(s->ev[0]);
    (void)hipEventDestroy(s->ev[1]);
    (void)hipStreamDestroy(s->stream);
    (void)hipStreamDestroy(s->copy_stream);
    delete s;
}
