// roctx ranges around the library's C entry points: a profiler that traces
// markers (rocprofv3 --marker-trace) shows each kgs_* call as a named range
// on the host timeline, beside the kernels it launched.  Without such a
// profiler attached the calls cost a few nanoseconds.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace kgs {

class TraceRange {
public:
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace kgs

#define KGS_TRACE(name) const kgs::TraceRange kgs_trace_range_(name)
