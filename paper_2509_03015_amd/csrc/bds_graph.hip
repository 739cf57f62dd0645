// Graph cache for the launch sequences (see bds_graph.hpp).
#include "bds_graph.hpp"

#include <cstdlib>
#include <cstring>
#include <list>
#include <mutex>

#include "bds_trace.hpp"

namespace bds {

namespace {

constexpr size_t kMaxGraphs = 32;

struct Entry {
    GraphKey key;
    hipGraphExec_t exec;
};

std::mutex g_mu;
std::list<Entry> g_cache;  // most recently used first
hipStream_t g_capture[64] = {};

bool graphs_enabled()
{
    static const bool on = [] {
        const char* e = std::getenv("BDS_GRAPH");
        return !(e && e[0] == '0');
    }();
    return on;
}

}  // namespace

void GraphKey::add_desc(const bds_desc& d)
{
    add((uint64_t)d.N);
    add((uint64_t)d.n);
    add((uint64_t)d.d);
    add((uint64_t)(uint32_t)d.prec | ((uint64_t)(uint32_t)d.nstar << 32));
    add((uint64_t)(uint32_t)d.tiles);
}

bool GraphKey::operator==(const GraphKey& o) const
{
    return kind == o.kind && device == o.device && count == o.count && nargs == o.nargs && digest == o.digest &&
           std::memcmp(args, o.args, sizeof(uint64_t) * nargs) == 0;
}

uint64_t hash_bytes(uint64_t h, const void* p, size_t n)
{
    const unsigned char* c = static_cast<const unsigned char*>(p);
    if (h == 0) h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

int run_graph(GraphKey key, hipStream_t st, const std::function<int(hipStream_t)>& launch)
{
    if (!graphs_enabled() || g_trace_on) return launch(st);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return BDS_EHIP;
    if (cs != hipStreamCaptureStatusNone) return launch(st);  // the caller is recording a graph
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return BDS_EHIP;
    key.device = dev;

    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
        if (it->key == key) {
            g_cache.splice(g_cache.begin(), g_cache, it);
            return hipGraphLaunch(g_cache.front().exec, st) == hipSuccess ? BDS_OK : BDS_EHIP;
        }
    }
    if (!g_capture[dev] && hipStreamCreateWithFlags(&g_capture[dev], hipStreamNonBlocking) != hipSuccess) {
        g_capture[dev] = nullptr;
        return BDS_EHIP;
    }
    hipStream_t cap = g_capture[dev];
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return BDS_EHIP;
    const int rc = launch(cap);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cap, &graph);
    if (rc != BDS_OK || ec != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc != BDS_OK ? rc : BDS_EHIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess || !exec) return BDS_EHIP;
    if (g_cache.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(g_cache.back().exec);
        g_cache.pop_back();
    }
    g_cache.push_front(Entry{key, exec});
    return hipGraphLaunch(exec, st) == hipSuccess ? BDS_OK : BDS_EHIP;
}

}  // namespace bds
