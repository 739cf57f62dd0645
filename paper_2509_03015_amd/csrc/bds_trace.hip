// Per-kernel timing with HIP events (diagnostics; see bds_trace.hpp).
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/bds.h"
#include "bds_trace.hpp"

namespace bds {

bool g_trace_on = false;

namespace {

std::mutex g_mu;
std::vector<hipEvent_t> g_pool;      // 2 events per slot
std::vector<const char*> g_names;    // kernel name per used slot
int g_used = 0;
int64_t g_dropped = 0;

void free_pool()
{
    for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
    g_pool.clear();
    g_names.clear();
    g_used = 0;
    g_dropped = 0;
}

}  // namespace

int trace_open(const char* name, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (2 * (size_t)(g_used + 1) > g_pool.size()) {
        ++g_dropped;
        return -1;
    }
    const int s = g_used++;
    g_names[s] = name;
    if (hipEventRecord(g_pool[2 * s], st) != hipSuccess) {
        --g_used;
        ++g_dropped;
        return -1;
    }
    return s;
}

void trace_close(int slot, hipStream_t st) { (void)hipEventRecord(g_pool[2 * slot + 1], st); }

}  // namespace bds

using namespace bds;

extern "C" {

int bds_trace_enable(int64_t max_launches)
{
    if (max_launches < 0 || max_launches > (int64_t(1) << 20)) return BDS_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_trace_on = false;
    free_pool();
    if (max_launches == 0) return BDS_OK;
    g_pool.resize(2 * (size_t)max_launches);
    for (size_t i = 0; i < g_pool.size(); ++i)
        if (hipEventCreate(&g_pool[i]) != hipSuccess) {
            g_pool.resize(i);
            free_pool();
            return BDS_EHIP;
        }
    g_names.assign((size_t)max_launches, nullptr);
    g_trace_on = true;
    return BDS_OK;
}

int bds_trace_read(int64_t max_kernels, char* names, int64_t* launches, double* total_ms, int64_t* n_kernels,
                   int64_t* dropped)
{
    if (max_kernels < 0 || (max_kernels > 0 && (!names || !launches || !total_ms)) || !n_kernels) return BDS_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<const char*> seen;
    std::vector<int64_t> cnt;
    std::vector<double> tot;
    int rc = BDS_OK;
    for (int s = 0; s < g_used; ++s) {
        float ms = 0.f;
        if (hipEventSynchronize(g_pool[2 * s + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, g_pool[2 * s], g_pool[2 * s + 1]) != hipSuccess) {
            rc = BDS_EHIP;
            continue;
        }
        size_t k = 0;
        while (k < seen.size() && std::strcmp(seen[k], g_names[s]) != 0) ++k;
        if (k == seen.size()) {
            seen.push_back(g_names[s]);
            cnt.push_back(0);
            tot.push_back(0.0);
        }
        cnt[k] += 1;
        tot[k] += (double)ms;
    }
    *n_kernels = (int64_t)seen.size();
    if (dropped) *dropped = g_dropped;
    for (size_t k = 0; k < seen.size() && (int64_t)k < max_kernels; ++k) {
        std::memset(names + 64 * k, 0, 64);
        std::strncpy(names + 64 * k, seen[k], 63);
        launches[k] = cnt[k];
        total_ms[k] = tot[k];
    }
    g_used = 0;
    g_dropped = 0;
    return rc;
}

}  // extern "C"
