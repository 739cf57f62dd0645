// Autotuner: coordinate search over the recursion's crossover nstar and the
// tile shapes of the per-level kernels, timing whole factor + solve runs of
// the caller's problem on the caller's stream (see bds.h).
//
// The searched quantities do not change the result beyond rounding: nstar
// moves the point where the recursion hands over to the sequential coarse
// factorisation (the paper's N_star of Alg. 4), and the tile fields choose
// how each level's products are cut into work-groups.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <vector>

#include "../../include/bds.h"
#include "bds_host.hpp"
#include "bds_kernels.hpp"

namespace bds {

int check_desc(const bds_desc* d);

namespace {

constexpr int kNstarCandidates[] = {1, 2, 4, 8, 16, 32, 64};

int field(int32_t tiles, int f) { return (tiles >> (4 * f)) & 15; }
int32_t with_field(int32_t tiles, int f, int code) { return (tiles & ~(15 << (4 * f))) | (code << (4 * f)); }

// Explicit codes for every field (the rule's choice where tiles has a zero).
int32_t explicit_tiles(const bds_desc& d)
{
    Tiling t;
    resolve_tiling((int)round_up(d.n, 16), d.prec, d.tiles, t);
    return BDS_TILES(t.couple, t.schur, t.sol);
}

std::vector<int> nstar_candidates(const bds_desc& d)
{
    std::vector<int> v;
    if (d.nstar > 0) {
        v.push_back(d.nstar);
        return v;
    }
    for (int c : kNstarCandidates)
        if (c == 1 || c <= d.N) v.push_back(c);
    return v;
}

// One untimed run, then `reps` timed runs; ms receives the time per run.
// Returns the first failing status (and ms = -1); *status receives info.status
// after the untimed run (copied to the host).
int time_runs(hipStream_t st, int reps, const std::function<int()>& run, const bds_info* info, int ninfo,
              float& ms, int& status)
{
    ms = -1.0f;
    status = BDS_OK;
    int rc = run();
    if (rc != BDS_OK) return rc;
    std::vector<bds_info> h((size_t)ninfo);
    if (hipMemcpyAsync(h.data(), info, sizeof(bds_info) * (size_t)ninfo, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return BDS_EHIP;
    for (const bds_info& x : h)
        if (x.status != BDS_OK) {
            status = x.status;
            return BDS_OK;
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return BDS_EHIP;
    }
    rc = hipEventRecord(e0, st) == hipSuccess ? BDS_OK : BDS_EHIP;
    for (int r = 0; r < reps && rc == BDS_OK; ++r) rc = run();
    if (rc == BDS_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = BDS_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == BDS_OK) ms /= (float)reps;
    return rc;
}

}  // namespace
}  // namespace bds

using namespace bds;

extern "C" {

int bds_tune_workspace_size(const bds_desc* desc, size_t* factor_bytes, size_t* solve_bytes)
{
    const int rc = check_desc(desc);
    if (rc != BDS_OK) return rc;
    size_t f = 0, s = 0;
    for (int ns : nstar_candidates(*desc)) {
        bds_desc d = *desc;
        d.nstar = ns;
        size_t fb = 0, sb = 0;
        const int r = bds_workspace_size(&d, &fb, &sb);
        if (r != BDS_OK) return r;
        f = std::max(f, fb);
        s = std::max(s, sb);
    }
    if (factor_bytes) *factor_bytes = f;
    if (solve_bytes) *solve_bytes = s;
    return BDS_OK;
}

int bds_tune(const bds_desc* desc, const double* Ad, const double* As, const double* B, double* X,
             void* factor_ws, size_t factor_bytes, void* solve_ws, size_t solve_bytes, bds_info* info, int reps,
             void* stream, bds_desc* best)
{
    int rc = check_desc(desc);
    if (rc != BDS_OK) return rc;
    if (!best || !Ad || (desc->N > 1 && !As) || !B || !X || !factor_ws || !solve_ws || !info) return BDS_EINVAL;
    size_t need_f = 0, need_s = 0;
    rc = bds_tune_workspace_size(desc, &need_f, &need_s);
    if (rc != BDS_OK) return rc;
    if (factor_bytes < need_f || solve_bytes < need_s) return BDS_EWORKSPACE;
    if (reps <= 0) reps = 3;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int np = (int)round_up(desc->n, 16);

    // tile fields start at the caller's value: a zero (library choice, which may
    // differ per level) competes with the explicit codes and is kept if it wins
    bds_desc cur = *desc;
    cur.nstar = nstar_candidates(*desc)[0];
    auto run_one = [&](const bds_desc& d) {
        return std::function<int()>([&, d] {
            int r = bds_factor(&d, Ad, As, factor_ws, factor_bytes, info, st);
            if (r != BDS_OK) return r;
            return bds_solve(&d, factor_ws, factor_bytes, Ad, As, B, X, solve_ws, solve_bytes, info, st);
        });
    };
    float best_ms = -1.0f;
    int status = BDS_OK;
    rc = time_runs(st, reps, run_one(cur), info, 1, best_ms, status);
    if (rc != BDS_OK) return rc;
    bds_desc winner = cur;
    // a failing system ends the search: its status stays in info
    bool stop = status != BDS_OK;
    auto consider = [&](const bds_desc& cand) -> int {
        float ms = -1.0f;
        int stt = BDS_OK;
        const int r = time_runs(st, reps, run_one(cand), info, 1, ms, stt);
        if (r != BDS_OK) return r;
        if (stt != BDS_OK) {
            stop = true;
            return BDS_OK;
        }
        if (ms < best_ms) {
            best_ms = ms;
            winner = cand;
        }
        return BDS_OK;
    };
    // 1. crossover N_star
    for (int ns : nstar_candidates(*desc)) {
        if (stop) break;
        if (ns == cur.nstar) continue;
        bds_desc c = cur;
        c.nstar = ns;
        rc = consider(c);
        if (rc != BDS_OK) return rc;
    }
    // 2. each tile field the caller left to the library, one at a time
    for (int f = 0; f < 3 && !stop; ++f) {
        if (field(desc->tiles, f) != 0) continue;
        cur = winner;
        for (int code : tile_choices(np, f == 2)) {
            if (stop) break;
            bds_desc c = cur;
            c.tiles = with_field(cur.tiles, f, code);
            rc = consider(c);
            if (rc != BDS_OK) return rc;
        }
    }
    // leave the winner's factor and solution in the caller's buffers
    rc = run_one(winner)();
    if (rc != BDS_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return BDS_EHIP;
    *best = winner;
    return BDS_OK;
}

int bds_tune_batched(int64_t K, const bds_desc* descs, const double* const* Ad, const double* const* As,
                     const double* const* B, double* const* X, void* factor_ws, size_t factor_bytes,
                     void* solve_ws, size_t solve_bytes, bds_info* info, int reps, void* stream,
                     bds_desc* best)
{
    size_t fb = 0, sb = 0;
    int rc = bds_batched_workspace_size(K, descs, &fb, &sb);
    if (rc != BDS_OK) return rc;
    if (!best || !Ad || !As || !B || !X || !factor_ws || !solve_ws || !info) return BDS_EINVAL;
    if (reps <= 0) reps = 3;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<bds_desc> cur(descs, descs + K);
    std::vector<int> nps;
    for (auto& d : cur) {
        d.tiles = explicit_tiles(d);
        nps.push_back((int)round_up(d.n, 16));
    }
    std::vector<int> groups(nps);
    std::sort(groups.begin(), groups.end());
    groups.erase(std::unique(groups.begin(), groups.end()), groups.end());
    auto fits = [&](const std::vector<bds_desc>& c) {
        size_t f2 = 0, s2 = 0;
        return bds_batched_workspace_size(K, c.data(), &f2, &s2) == BDS_OK && f2 <= factor_bytes &&
               s2 <= solve_bytes;
    };
    if (!fits(cur)) return BDS_EWORKSPACE;
    auto run_one = [&](const std::vector<bds_desc>& c) {
        return std::function<int()>([&, c] {
            int r = bds_factor_batched(K, c.data(), Ad, As, factor_ws, factor_bytes, info, st);
            if (r != BDS_OK) return r;
            return bds_solve_batched(K, c.data(), factor_ws, factor_bytes, Ad, As, B, X, solve_ws, solve_bytes,
                                     info, st);
        });
    };
    float best_ms = -1.0f;
    int status = BDS_OK;
    rc = time_runs(st, reps, run_one(cur), info, (int)K, best_ms, status);
    if (rc != BDS_OK) return rc;
    std::vector<bds_desc> winner = cur;
    bool stop = status != BDS_OK;
    for (int np : groups) {
        for (int f = 0; f < 3 && !stop; ++f) {
            // searched only if every system of the group left the field to the library
            bool free_field = true;
            for (int64_t k = 0; k < K; ++k)
                if (nps[k] == np && field(descs[k].tiles, f) != 0) free_field = false;
            if (!free_field) continue;
            cur = winner;
            int now = 0;
            for (int64_t k = 0; k < K; ++k)
                if (nps[k] == np) now = field(cur[k].tiles, f);
            for (int code : tile_choices(np, f == 2)) {
                if (stop) break;
                if (code == now) continue;
                std::vector<bds_desc> c = cur;
                for (int64_t k = 0; k < K; ++k)
                    if (nps[k] == np) c[k].tiles = with_field(c[k].tiles, f, code);
                if (!fits(c)) continue;
                float ms = -1.0f;
                int stt = BDS_OK;
                rc = time_runs(st, reps, run_one(c), info, (int)K, ms, stt);
                if (rc != BDS_OK) return rc;
                if (stt != BDS_OK) {
                    stop = true;
                    break;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    winner = c;
                }
            }
        }
    }
    rc = run_one(winner)();
    if (rc != BDS_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return BDS_EHIP;
    std::copy(winner.begin(), winner.end(), best);
    return BDS_OK;
}

}  // extern "C"
