// Host-side instrumentation of the library.
//
// * roctx ranges around the entry points (GDGS_TRACE): rocprofv3
//   --marker-trace shows them beside the kernels.  A range spans the host's
//   enqueue of a call (argument checks, graph launches), not the GPU's
//   execution of it, which the kernel trace gives.
// * A log level from the environment variable GDGS_LOG, read once:
//   0 (default) silent; 1 every error message the library records (the text
//   gdgs_last_error returns); 2 also graph captures and server events
//   (creation, capacity re-runs, teardown); 3 also every entry-point call and
//   multigrid plan.  Lines go to stderr with the prefix "gdgs[<level>] ".
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace gdgs {

int log_level();
void log_msg(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

struct TraceRange {
    explicit TraceRange(const char* name) {
        roctxRangePushA(name);
        if (log_level() >= 3) log_msg(3, "call %s", name);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace gdgs

#define GDGS_LOG(level, ...)                                                   \
    do {                                                                       \
        if (::gdgs::log_level() >= (level)) ::gdgs::log_msg((level), __VA_ARGS__); \
    } while (0)
#define GDGS_TRACE(name) ::gdgs::TraceRange gdgs_trace_range_(name)
