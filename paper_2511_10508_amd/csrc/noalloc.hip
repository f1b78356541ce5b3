// pf_step_noalloc: the fused step on caller-owned buffers with no allocation.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid it).  The only scratch
// the fused kernels use is the reduction partials of PF_REDUCE_EACH_STEP; here
// they live in one file-scope device array, `scratch`, of kNoAllocPairs
// double2 pairs (16 MiB), which every GPU the library runs on holds until
// the process ends.  Host code never passes the array's name to a kernel (in
// host code it is a stand-in, not a device address): on the first call on
// each device, with that device current, hipGetSymbolAddress gives that
// device's copy, and that pointer is kept per device and passed to the
// kernels.  Calls on one device share its array; calls that overlap on one
// device race (see include/pfmi.h).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pfmi.h"
#include "pf_runtime.h"

namespace pf {

constexpr int64_t kNoAllocPairs = int64_t(1) << 20;  // 16 MiB
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) double2 scratch[kNoAllocPairs];

static std::mutex g_scratch_mu;
static double2 *g_scratch_dev[kNoAllocMaxDevices];  // per device: its copy of `scratch`

// Device address of the current device's `scratch`, looked up once per device.
static pf_status scratch_of_current_device(double2 **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(PF_ERR_DEVICE, "device ordinal beyond the allocation-free path's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(PF_ERR_DEVICE, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_dev[dev] = static_cast<double2 *>(p);
    }
    *out = g_scratch_dev[dev];
    return PF_OK;
}

}  // namespace pf

using namespace pf;

extern "C" __attribute__((visibility("default"))) pf_status
pf_step_noalloc(const pf_desc *desc, void *hip_stream, void *const *dev_bufs, int32_t nbufs,
                int32_t parity, int64_t nsteps, double *dev_history)
{
    Model m;  // on the stack: its containers stay empty and allocate nothing
    int64_t need = 0;
    pf_status st = borrow_plan(&m, desc, hip_stream, dev_bufs, nbufs, parity, nsteps, dev_history,
                               &need);
    if (st != PF_OK) return st;
    if (need > kNoAllocPairs)
        return fail(PF_ERR_ARG, "this grid needs more reduction scratch than the 16 MiB the "
                                "allocation-free path holds; use pf_create_on and pf_step");
    double2 *s = nullptr;
    if (need > 0) {
        st = scratch_of_current_device(&s);
        if (st != PF_OK) return st;
    }
    return borrow_run(&m, s, nsteps, reinterpret_cast<double2 *>(dev_history));
}
