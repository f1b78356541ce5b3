// Host-side model object shared by the runtime and the serving engine.
#pragma once

#include <string>
#include <vector>

#include "../../include/pfmi.h"
#include "pf_internal.h"

namespace pf {

constexpr int kGraphSteps = 32;  // steps per captured graph (pf_step with PF_USE_GRAPH)
constexpr int64_t kDefaultPitchPadBytes = 0;  // row padding for rows >= 4 KiB

struct Model {
    pf_desc desc{};
    int nf = 1;
    bool fp32 = false;
    Launch L{};
    int64_t pitch = 0, elems = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false, own_bufs = true;
    bool async_alloc = false;     // stream-ordered allocations, no host syncs (server models)
    void *buf[kMaxFields][2] = {};   // [field][parity]
    int parity = 0;
    int64_t steps_done = 0;

    // decomposition of the fused family (family 0), per-site (family 1) or
    // spectral (family 2)
    int family = 1;
    int tb = 1;                   // time steps fused per launch (2D, r <= 2)
    int rpw_req = 0, rpw = 2;     // 3D tile rows per wave: requested (0: default), in use
    // 3D CH: mu in registers (1) or through `scratch` (2); requested (0: the
    // library's choice), in use
    int passes_req = 0, passes = 1;
    // small Allen-Cahn grids of the fused family: step calls without per-step
    // reductions or kernel timing run every step in one workgroup's LDS
    bool lds_steps = false;
    int32_t clen = 0, strips = 0, ow = 0, ytiles = 1, chunks = 0, items = 0, blocks = 0,
            threads = 0;
    int64_t fused_slots = 0;
    StepArgs<double> a64{};
    StepArgs<float> a32{};

    double2 *part = nullptr;     // partial sums [kNumQ][pstride]
    int64_t pstride = 0;
    double2 *part2 = nullptr;    // second-level partials [kNumQ][kFinSlots]
    double2 *res = nullptr;      // finalised reductions [kNumQ]
    double2 *hist = nullptr;     // per-step reductions [hist_cap][kNumQ]
    int64_t hist_cap = 0, hist_len = 0;
    double2 *stage = nullptr;    // graph staging rows [kGraphSteps][kNumQ]
    void *scratch = nullptr;     // CH mu buffer(s) of the per-site family or of a two-pass plan
    void *spec = nullptr;        // spectral scheme state (family 2): plans and half spectra

    struct Graph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        int par = 0, steps = 0, launches = 0;
        bool red = false;
    };
    std::vector<Graph> graphs;
    bool graphs_valid = false;
    int64_t captures = 0, replays = 0, launches = 0, timed_steps = 0;

    bool timing = false;
    std::vector<hipEvent_t> events;
    size_t ev_used = 0;

    ~Model();
};

pf_status fail(pf_status s, const std::string &msg);
pf_status hip_fail(hipError_t e, const char *what);
pf_status check_desc(const pf_desc *d);
double stability_limit(const pf_desc *d);
int nfields_of(int kind);
int64_t pitch_of(const pf_desc *d);
int64_t buffer_elems(const pf_desc *d);
int elem_bytes(const pf_desc *d);
double volume(const pf_desc &d);

pf_status model_create(const pf_desc *desc, void *stream, void *const *bufs, int32_t nbufs,
                       Model **out, bool async_alloc = false);
void model_release_async(Model *m);  // free a server model's memory in stream order
void pf_destroy_model(Model *m);
pf_status init_fields(Model *m, int32_t ic, uint64_t seed, const double *p, int32_t np);
pf_status set_chunk(Model *m, int32_t chunk);
pf_status do_steps(Model *m, int64_t nsteps);
pf_status reduce_now(Model *m, double2 *host_out);
pf_status pick_quantity(const Model *m, int32_t which, const double2 *q, double *hi, double *lo);
int32_t default_chunk(const pf_desc *d);

// pf_step_noalloc (noalloc.hip): plan a borrowed model (all checks, no device
// call, no allocation), then run it on the given reduction scratch.
pf_status borrow_plan(Model *m, const pf_desc *d, void *stream, void *const *bufs, int32_t nbufs,
                      int32_t parity, int64_t nsteps, const void *hist, int64_t *pairs_need);
pf_status borrow_run(Model *m, double2 *scratch, int64_t nsteps, double2 *hist);

// roctx ranges (trace.cpp): TraceRange opens one for its lifetime.
void trace_push(const char *msg);
void trace_pop();
struct TraceRange {
    explicit TraceRange(const char *msg) { trace_push(msg); }
    ~TraceRange() { trace_pop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// Model H on 2D grids (r <= 2) in one y-marching pass, bitwise equal to the
// two passes of the per-site kernels (which run it with PF_FORCE_GENERIC);
// kernels_mh2d.hip.
bool mh2d_available(const Launch &L);
hipError_t launch_mh2d(const Launch &L, const void *args, hipStream_t s);
// Model H on 3D grids (r <= 2) in one z-marching pass, bitwise equal to the
// per-site kernels' two passes; kernels_mh3d.hip.
bool mh3d_available(const Launch &L);
hipError_t launch_mh3d(const Launch &L, const void *args, hipStream_t s);

// Semi-implicit Fourier spectral scheme (spectral.cpp).
pf_status spectral_setup(Model *m);
pf_status spectral_step(Model *m, int par, const void *step_args);
void spectral_release(Model *m);
// The kept spectrum no longer matches the state (set from outside).
void spectral_invalidate(Model *m);
uint64_t spectral_bytes(const pf_desc *d);

}  // namespace pf
