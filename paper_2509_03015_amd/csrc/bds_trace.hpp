// Optional per-kernel timing: when enabled through bds_trace_enable, every
// kernel launch of the library is bracketed by two HIP events recorded on the
// launch stream, and bds_trace_read sums the elapsed times per kernel name.
// Disabled (the default), a scope costs one branch on a global flag.
#pragma once

#include <hip/hip_runtime.h>

namespace bds {

extern bool g_trace_on;

// Records the opening event; returns the slot to close, or -1.
int trace_open(const char* name, hipStream_t st);
void trace_close(int slot, hipStream_t st);

struct TraceScope {
    int slot = -1;
    hipStream_t st;
    TraceScope(const char* name, hipStream_t s) : st(s)
    {
        if (g_trace_on) slot = trace_open(name, s);
    }
    ~TraceScope()
    {
        if (slot >= 0) trace_close(slot, st);
    }
};

}  // namespace bds

// Launch statement `...` under a timing scope named `name` on stream `st`.
#define BDS_TIMED(name, st, ...)            \
    do {                                    \
        ::bds::TraceScope bds_ts_(name, st); \
        __VA_ARGS__;                        \
    } while (0)
