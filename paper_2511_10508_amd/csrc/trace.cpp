// roctx ranges around the library's step batches, tuning and serving ticks,
// so that a rocprofv3 --marker-trace run shows them beside the kernels.
// Without a profiler attached a range costs a call into the roctx library.
#include <rocprofiler-sdk-roctx/roctx.h>

#include "pf_runtime.h"

namespace pf {

void trace_push(const char *msg) { (void)roctxRangePushA(msg); }
void trace_pop() { (void)roctxRangePop(); }

}  // namespace pf
