// Named host ranges for profilers (roctx): each stage of the hot path opens
// a range while it enqueues its kernels, so `rocprofv3 --marker-trace
// --kernel-trace` shows which call and which stage each dispatch came from.
// Without a profiler attached a range costs a few tens of nanoseconds.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace pi {

struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace pi
