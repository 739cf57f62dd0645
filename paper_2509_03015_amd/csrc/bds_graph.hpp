// Launch sequences replayed as HIP graphs.
//
// A factorisation or an FP64 solve is a fixed sequence of kernel launches
// (a few per reduction level) whose arguments depend only on the call's
// descriptor and pointers.  The first call with a given argument set records
// the sequence into a graph on a library-owned capture stream; later calls
// with the same arguments launch the instantiated graph on the caller's
// stream, which replaces the per-level launches by one graph launch.
// Sequences are launched directly instead when kernel timing is on, when the
// caller's stream is itself being captured, or when the environment sets
// BDS_GRAPH=0.  Only sequences without host synchronisation go through here.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>

#include "../../include/bds.h"

namespace bds {

struct GraphKey {
    int kind = 0;              // entry point
    int device = 0;
    int64_t count = 0;         // systems (batched) or 1
    uint64_t args[24] = {};    // descriptor fields, pointers and sizes
    int nargs = 0;
    void add(uint64_t v)
    {
        if (nargs < 24) args[nargs++] = v;
    }
    void add(const void* p) { add((uint64_t)(uintptr_t)p); }
    void add_desc(const bds_desc& d);
    uint64_t digest = 0;       // hash of variable-length content (batched descriptors and pointers)
    bool operator==(const GraphKey& o) const;
};

// Runs launch(stream) through a cached graph (or directly, see above) and
// returns its status; the launches end up ordered on `st`.
int run_graph(GraphKey key, hipStream_t st, const std::function<int(hipStream_t)>& launch);

// FNV-1a over a byte range, for GraphKey::digest.
uint64_t hash_bytes(uint64_t h, const void* p, size_t n);

}  // namespace bds
