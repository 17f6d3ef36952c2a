// Host-side trace ranges (roctx): each entry point and solver phase pushes a
// named range, visible with rocprofv3 --marker-trace; without a profiler
// attached a push or pop is a call through an empty dispatch table.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace hm {
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};
}  // namespace hm
