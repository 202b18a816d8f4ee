// Named host ranges for profilers (rocprofv3 --marker-trace shows them beside
// the kernels they enqueue): every public call that steps, initialises or
// reads back a lattice opens one for its duration on the calling thread.
// With no profiler attached a range is two calls into the roctx library that
// return at once.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace lbm {

class TraceRange {
  public:
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

} // namespace lbm
