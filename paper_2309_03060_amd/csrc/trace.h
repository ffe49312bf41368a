// Host-side ranges of the library's calls for rocprofv3 --marker-trace (roctx).  Off unless
// cola_trace_enable(1) was called; a disabled range costs one relaxed atomic load.
#pragma once
#include <atomic>

namespace cola {

extern std::atomic<int> g_trace_on;

struct TraceRange {
    bool on;
    explicit TraceRange(const char* name);
    ~TraceRange();
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace cola
