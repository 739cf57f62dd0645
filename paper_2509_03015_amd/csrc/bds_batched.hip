// Batched form: K independent systems of uneven (N, n, d) (the paper's batch
// notation {A^(k)} of Sec. 3.2).  Every reduction level of every system runs
// in one launch per kernel and level over the whole batch: the host builds a
// table of per-system records with exclusive prefix sums of their work units,
// uploads it into the workspace, and each work-group finds its record by
// binary search.  Systems whose recursion is shorter simply drop out of the
// deeper levels' tables.
//
// Workspace layout: the systems' own factor (solve) regions one after the
// other, each laid out by make_plan, followed by a table region.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <type_traits>
#include <vector>

#include "../../include/bds.h"
#include "bds_graph.hpp"
#include "bds_host.hpp"
#include "bds_kernels.hpp"
#include "bds_plan.hpp"

namespace bds {

int check_desc(const bds_desc* d);

namespace {

constexpr int kMaxBatch = 1 << 20;

struct BatchPlan {
    int64_t K = 0;
    int prec = BDS_F64;
    int nlev = 0;                 // deepest recursion over the batch
    std::vector<SysPlan> sys;     // offsets relative to the workspace start
    // systems are grouped by padded block size np and tile shapes (one launch per
    // kernel, level and group, so that each group runs its own tiling): the
    // distinct groups in increasing order, and the number of systems of each
    // group that reach each level
    struct Group {
        int np;
        Tiling tl;
        bool operator<(const Group& o) const { return np != o.np ? np < o.np : tl < o.tl; }
        bool operator==(const Group& o) const { return np == o.np && tl == o.tl; }
    };
    std::vector<Group> groups;
    std::vector<std::vector<int64_t>> lvcnt;   // [level][group]
    int group(const SysPlan& p) const
    {
        const Group key{(int)p.np, p.tl};
        return (int)(std::lower_bound(groups.begin(), groups.end(), key) - groups.begin());
    }
    bool in_group(const SysPlan& p, const Group& g) const { return (int)p.np == g.np && p.tl == g.tl; }
    size_t ftab = 0, ftab_bytes = 0;   // factor table region
    size_t stab = 0, stab_bytes = 0;   // solve table region (solve core)
    size_t rtab = 0, rtab_bytes = 0;   // refinement / packing table region
    size_t nrm = 0;               // 2K doubles: per-system (sum C^2, sum X^2)
    size_t ic = 0;                // 2K ints: per-system (iterations, converged)
    size_t factor_bytes = 0, solve_bytes = 0;
};

size_t tab_bytes(size_t nrec, size_t rec_size, int nprefix)
{
    return align_up(nrec * rec_size) + (size_t)nprefix * align_up((nrec + 1) * sizeof(int64_t));
}

int make_batch_plan(int64_t K, const bds_desc* descs, BatchPlan& bp)
{
    if (K < 1 || K > kMaxBatch || !descs) return BDS_EINVAL;
    for (int64_t k = 0; k < K; ++k) {
        if (check_desc(&descs[k]) != BDS_OK) return BDS_EINVAL;
        if (descs[k].prec != descs[0].prec || descs[k].nstar != descs[0].nstar ||
            descs[k].max_refine != descs[0].max_refine || descs[k].refine_tol != descs[0].refine_tol)
            return BDS_EINVAL;
    }
    bp.K = K;
    bp.prec = descs[0].prec;
    bp.sys.reserve((size_t)K);
    size_t f = 0, s = 0;
    for (int64_t k = 0; k < K; ++k) {
        SysPlan p = make_plan(descs[k], f, s);
        f += p.factor_bytes;
        s += p.solve_bytes;
        bp.nlev = std::max<int>(bp.nlev, (int)p.lv.size());
        bp.groups.push_back(BatchPlan::Group{(int)p.np, p.tl});
        bp.sys.push_back(std::move(p));
    }
    std::sort(bp.groups.begin(), bp.groups.end());
    bp.groups.erase(std::unique(bp.groups.begin(), bp.groups.end()), bp.groups.end());
    const size_t G = bp.groups.size();
    bp.lvcnt.assign((size_t)bp.nlev, std::vector<int64_t>(G, 0));
    std::vector<int64_t> gcnt(G, 0);
    for (const SysPlan& p : bp.sys) {
        const int g = bp.group(p);
        gcnt[g] += 1;
        for (size_t l = 0; l < p.lv.size(); ++l) bp.lvcnt[l][g] += 1;
    }
    const size_t Kz = (size_t)K;
    // factor tables: per level and group records + 3 prefix arrays, coarse records (two kinds), packing
    size_t ft = 0;
    for (int l = 0; l < bp.nlev; ++l)
        for (size_t g = 0; g < G; ++g)
            if (bp.lvcnt[l][g] > 0) ft += tab_bytes((size_t)bp.lvcnt[l][g], sizeof(FacLv<double, double>), 3);
    ft += 2 * tab_bytes(Kz, sizeof(CoarseFac<double>), 0);
    ft += tab_bytes(2 * Kz, sizeof(PackRec), 1);
    bp.ftab = f;
    bp.ftab_bytes = align_up(ft);
    bp.factor_bytes = f + bp.ftab_bytes;
    // solve-core tables: per level and group records + 3 prefix arrays, coarse records + prefix
    size_t st = 0;
    for (int l = 0; l < bp.nlev; ++l)
        for (size_t g = 0; g < G; ++g)
            if (bp.lvcnt[l][g] > 0) st += tab_bytes((size_t)bp.lvcnt[l][g], sizeof(SolLv<double>), 3);
    st += tab_bytes(Kz, sizeof(CoarseSol), 1);
    bp.stab = s;
    bp.stab_bytes = align_up(st);
    s += bp.stab_bytes;
    // refinement (residual records per group) and packing tables
    size_t rt = tab_bytes(Kz, sizeof(AxpyArgs), 1) + tab_bytes(Kz, sizeof(PackRec), 1);
    for (size_t g = 0; g < G; ++g) rt += tab_bytes((size_t)gcnt[g], sizeof(ResidArgs), 1);
    bp.rtab = s;
    bp.rtab_bytes = align_up(rt);
    s += bp.rtab_bytes;
    bp.nrm = s;
    s = align_up(s + 2 * Kz * sizeof(double));
    bp.ic = s;
    s = align_up(s + 2 * Kz * sizeof(int));
    bp.solve_bytes = s;
    return BDS_OK;
}

// Host image of a device table region, uploaded with one copy.
class Table {
public:
    Table(void* ws, size_t off, size_t cap) : dev_(static_cast<char*>(ws) + off), cap_(cap), h_(new char[cap]) {}
    // Reserve `count` records; returns the host slot and sets *dev to the device address.
    template <typename R> R* take(size_t count, const R** dev)
    {
        const size_t o = align_up(used_);
        used_ = o + std::max<size_t>(count, 1) * sizeof(R);
        if (used_ > cap_) return nullptr;
        *dev = reinterpret_cast<const R*>(dev_ + o);
        return reinterpret_cast<R*>(h_.get() + o);
    }
    hipError_t upload(hipStream_t st)
    {
        if (used_ == 0) return hipSuccess;
        // ordered on the stream and complete on return, so the host image may be freed after it
        return hipMemcpyWithStream(dev_, h_.get(), used_, hipMemcpyHostToDevice, st);
    }
    bool overflow() const { return used_ > cap_; }

private:
    char* dev_;
    size_t cap_;
    size_t used_ = 0;
    std::unique_ptr<char[]> h_;
};

// Prefix table for `recs` records with unit counts from `units(i)`.
template <typename F>
int64_t* fill_prefix(Table& t, size_t nrec, const int64_t** dev, F units, int64_t& total)
{
    int64_t* pre = t.take<int64_t>(nrec + 1, dev);
    if (!pre) return nullptr;
    pre[0] = 0;
    for (size_t i = 0; i < nrec; ++i) pre[i + 1] = pre[i] + units(i);
    total = pre[nrec];
    return pre;
}

template <typename C>
int factor_batched_impl(const BatchPlan& bp, const double* const* Ad, const double* const* As, void* fws,
                        bds_info* info, hipStream_t st)
{
    using T = typename Stor<C>::type;
    const int K = (int)bp.K;
    Table tab(fws, bp.ftab, bp.ftab_bytes);
    // packing of systems whose n is not a multiple of 16
    std::vector<PackRec> packs;
    std::vector<int64_t> pack_units;
    for (int k = 0; k < K; ++k) {
        const SysPlan& p = bp.sys[k];
        if (!p.packed) continue;
        packs.push_back(PackRec{Ad[k], at<double>(fws, p.Ad0), (int)p.n, (int)p.np, 0, PACK_DIAG});
        pack_units.push_back(p.N);
        if (p.N > 1) {
            packs.push_back(PackRec{As[k], at<double>(fws, p.As0), (int)p.n, (int)p.np, 0, PACK_OFFDIAG});
            pack_units.push_back(p.N - 1);
        }
    }
    const PackRec* pack_dev = nullptr;
    const int64_t* pack_start = nullptr;
    int64_t pack_tot = 0;
    if (!packs.empty()) {
        PackRec* h = tab.take<PackRec>(packs.size(), &pack_dev);
        if (!h) return BDS_EWORKSPACE;
        std::copy(packs.begin(), packs.end(), h);
        if (!fill_prefix(tab, packs.size(), &pack_start, [&](size_t i) { return pack_units[i]; }, pack_tot))
            return BDS_EWORKSPACE;
    }
    struct LevelTab {
        int level, np;
        Tiling tl;
        const void* recs;
        const int64_t *sd, *sc, *ss;
        int64_t td, tc, ts;
        int cnt;
    };
    std::vector<LevelTab> lt;
    for (int l = 0; l < bp.nlev; ++l) {
        for (const auto& grp : bp.groups) {
            std::vector<int> members;
            for (int k = 0; k < K; ++k)
                if ((int)bp.sys[k].lv.size() > l && bp.in_group(bp.sys[k], grp)) members.push_back(k);
            if (members.empty()) continue;
            const int np = grp.np;
            lt.push_back(LevelTab{});
            LevelTab& L = lt.back();
            L.level = l;
            L.np = np;
            L.tl = grp.tl;
            L.cnt = (int)members.size();
            const size_t m = members.size();
            // level 0 reads the FP64 inputs (or their padded copies), deeper levels the
            // previous level's Schur complement in the factor precision T
            auto fill = [&](auto* h, auto read_ad, auto read_as) {
                using Rec = std::remove_pointer_t<decltype(h)>;
                for (size_t i = 0; i < m; ++i) {
                    const int k = members[i];
                    const SysPlan& p = bp.sys[k];
                    const LevelPlan& V = p.lv[l];
                    h[i] = Rec{read_ad(k), read_as(k), at<T>(fws, V.Li), at<T>(fws, V.Wt), at<T>(fws, V.Pr),
                               at<T>(fws, V.Adn), at<T>(fws, V.Asn), (int)V.M, (int)p.np, l, 0, info + k};
                }
            };
            if (l == 0) {
                const FacLv<T, double>* dev = nullptr;
                FacLv<T, double>* h = tab.take<FacLv<T, double>>(m, &dev);
                if (!h) return BDS_EWORKSPACE;
                fill(h, [&](int k) { return level0_matrices(bp.sys[k], Ad[k], As[k], fws).Ad; },
                     [&](int k) { return level0_matrices(bp.sys[k], Ad[k], As[k], fws).As; });
                L.recs = dev;
            } else {
                const FacLv<T, T>* dev = nullptr;
                FacLv<T, T>* h = tab.take<FacLv<T, T>>(m, &dev);
                if (!h) return BDS_EWORKSPACE;
                fill(h, [&](int k) { return (const T*)at<T>(fws, bp.sys[k].lv[l - 1].Adn); },
                     [&](int k) { return (const T*)at<T>(fws, bp.sys[k].lv[l - 1].Asn); });
                L.recs = dev;
            }
            auto M_of = [&](size_t i) { return (int)bp.sys[members[i]].lv[l].M; };
            const Tiling tl = grp.tl;
            if (!fill_prefix(tab, m, &L.sd, [&](size_t i) { return units_fac_diag(M_of(i)); }, L.td) ||
                !fill_prefix(tab, m, &L.sc, [&](size_t i) { return units_fac_couple(M_of(i), np, tl.couple); }, L.tc) ||
                !fill_prefix(tab, m, &L.ss, [&](size_t i) { return units_fac_schur(M_of(i), np, tl.schur); }, L.ts))
                return BDS_EWORKSPACE;
        }
    }
    // coarse systems: those with no reduction level read FP64 inputs, the others level blocks of type T
    std::vector<CoarseFac<double>> c0;
    std::vector<CoarseFac<T>> c1;
    for (int k = 0; k < K; ++k) {
        const SysPlan& p = bp.sys[k];
        const int Lv = (int)p.lv.size();
        if (Lv == 0) {
            const Level0 a0 = level0_matrices(p, Ad[k], As[k], fws);
            c0.push_back(CoarseFac<double>{a0.Ad, a0.As, at<double>(fws, p.Lc), at<double>(fws, p.Lsc),
                                           at<double>(fws, p.Cw), (int)p.Mc, (int)p.np, 0, 0, info + k});
        } else {
            const LevelPlan& P = p.lv.back();
            c1.push_back(CoarseFac<T>{at<T>(fws, P.Adn), at<T>(fws, P.Asn), at<double>(fws, p.Lc),
                                      at<double>(fws, p.Lsc), at<double>(fws, p.Cw), (int)p.Mc, (int)p.np, Lv, 0,
                                      info + k});
        }
    }
    const CoarseFac<double>* c0_dev = nullptr;
    const CoarseFac<T>* c1_dev = nullptr;
    if (!c0.empty()) {
        CoarseFac<double>* h = tab.take<CoarseFac<double>>(c0.size(), &c0_dev);
        if (!h) return BDS_EWORKSPACE;
        std::copy(c0.begin(), c0.end(), h);
    }
    if (!c1.empty()) {
        CoarseFac<T>* h = tab.take<CoarseFac<T>>(c1.size(), &c1_dev);
        if (!h) return BDS_EWORKSPACE;
        std::copy(c1.begin(), c1.end(), h);
    }
    BDS_TRY(tab.upload(st));
    int np0 = 16, np1 = 16;
    for (const auto& c : c0) np0 = std::max(np0, c.np);
    for (const auto& c : c1) np1 = std::max(np1, c.np);

    // The launch sequence reads every per-system argument from the tables just
    // uploaded, so it depends only on the table addresses and the unit counts:
    // it is recorded once per such signature and replayed as a graph.
    std::vector<int64_t> sig = {(int64_t)(uintptr_t)pack_dev, (int64_t)(uintptr_t)pack_start,
                                (int64_t)packs.size(), pack_tot, (int64_t)(uintptr_t)c0_dev, (int64_t)c0.size(), np0,
                                (int64_t)(uintptr_t)c1_dev, (int64_t)c1.size(), np1};
    for (const LevelTab& L : lt) {
        const int64_t v[] = {L.level, L.np, L.tl.couple, L.tl.schur, L.tl.sol, (int64_t)(uintptr_t)L.recs,
                             (int64_t)(uintptr_t)L.sd, (int64_t)(uintptr_t)L.sc, (int64_t)(uintptr_t)L.ss, L.cnt,
                             L.td, L.tc, L.ts};
        sig.insert(sig.end(), v, v + sizeof(v) / sizeof(v[0]));
    }
    GraphKey key;
    key.kind = 3;
    key.count = K;
    key.add((uint64_t)PrecOf<C>::value);
    key.add(fws);
    key.add(info);
    key.digest = hash_bytes(0, sig.data(), sig.size() * sizeof(int64_t));
    return run_graph(key, st, [&](hipStream_t s) -> int {
        BDS_TRY(launch_clear_info(info, K, s));
        BDS_TRY(launch_pack_tab(pack_dev, pack_start, (int)packs.size(), pack_tot, s));
        // levels in order; the groups of one level are independent of each other
        for (const LevelTab& L : lt) {
            if (L.level == 0) {
                BDS_TRY(launch_factor_level<C, double>(FacLv<T, double>{},
                                                       static_cast<const FacLv<T, double>*>(L.recs), L.sd, L.sc,
                                                       L.ss, L.cnt, L.td, L.tc, L.ts, L.np, L.tl, s));
            } else {
                BDS_TRY(launch_factor_level<C, T>(FacLv<T, T>{}, static_cast<const FacLv<T, T>*>(L.recs), L.sd,
                                                  L.sc, L.ss, L.cnt, L.td, L.tc, L.ts, L.np, L.tl, s));
            }
        }
        BDS_TRY(launch_coarse_factor<double>(CoarseFac<double>{}, c0_dev, (int)c0.size(), np0, s));
        BDS_TRY(launch_coarse_factor<T>(CoarseFac<T>{}, c1_dev, (int)c1.size(), np1, s));
        return BDS_OK;
    });
}

// One solve through the stored hierarchies of the systems in `act`: B0[k] -> X0[k] (padded).
template <typename T>
int solve_core_batched(const BatchPlan& bp, const std::vector<int>& act, const void* fws, void* sws,
                       const std::vector<const double*>& B0, const std::vector<double*>& X0, hipStream_t st)
{
    Table tab(sws, bp.stab, bp.stab_bytes);
    struct LevelTab {
        int level, np;
        Tiling tl;
        const SolLv<T>* recs;
        const int64_t *si, *ss, *sb;
        int64_t ti, ts, tb;
        int cnt;
    };
    std::vector<LevelTab> lt;
    for (int l = 0; l < bp.nlev; ++l) {
        for (const auto& grp : bp.groups) {
            std::vector<int> members;
            for (int k : act)
                if ((int)bp.sys[k].lv.size() > l && bp.in_group(bp.sys[k], grp)) members.push_back(k);
            if (members.empty()) continue;
            const int np = grp.np;
            lt.push_back(LevelTab{});
            LevelTab& L = lt.back();
            L.level = l;
            L.np = np;
            L.tl = grp.tl;
            L.cnt = (int)members.size();
            const size_t m = members.size();
            SolLv<T>* h = tab.take<SolLv<T>>(m, &L.recs);
            if (!h) return BDS_EWORKSPACE;
            for (size_t i = 0; i < m; ++i) {
                const int k = members[i];
                const SysPlan& p = bp.sys[k];
                const LevelPlan& V = p.lv[l];
                const double* B = l == 0 ? B0[k] : at<double>(sws, p.lv[l - 1].Bn);
                double* X = l == 0 ? X0[k] : at<double>(sws, p.lv[l - 1].Xn);
                h[i] = SolLv<T>{at<T>(fws, V.Li), at<T>(fws, V.Wt), at<T>(fws, V.Pr), B, at<double>(sws, V.Y),
                                at<double>(sws, V.Bn), at<double>(sws, V.Xn), X, (int)V.M, (int)p.np, (int)p.d, 0};
            }
            auto M_of = [&](size_t i) { return (int)bp.sys[members[i]].lv[l].M; };
            auto d_of = [&](size_t i) { return (int)bp.sys[members[i]].d; };
            if (!fill_prefix(tab, m, &L.si, [&](size_t i) { return units_sol_fwd_int(M_of(i), np, d_of(i), L.tl.sol); }, L.ti) ||
                !fill_prefix(tab, m, &L.ss, [&](size_t i) { return units_sol_fwd_sep(M_of(i), np, d_of(i), L.tl.sol); }, L.ts) ||
                !fill_prefix(tab, m, &L.sb, [&](size_t i) { return units_sol_bwd(M_of(i), d_of(i)); }, L.tb))
                return BDS_EWORKSPACE;
        }
    }
    const size_t m = act.size();
    const CoarseSol* cdev = nullptr;
    CoarseSol* ch = tab.take<CoarseSol>(m, &cdev);
    if (!ch) return BDS_EWORKSPACE;
    for (size_t i = 0; i < m; ++i) {
        const int k = act[i];
        const SysPlan& p = bp.sys[k];
        const int Lv = (int)p.lv.size();
        ch[i] = CoarseSol{at<double>(fws, p.Lc), at<double>(fws, p.Lsc),
                          Lv == 0 ? B0[k] : at<double>(sws, p.lv.back().Bn), at<double>(sws, p.Yc),
                          Lv == 0 ? X0[k] : at<double>(sws, p.lv.back().Xn), (int)p.Mc, (int)p.np, (int)p.d, 0};
    }
    const int64_t* cstart = nullptr;
    int64_t ctot = 0;
    if (!fill_prefix(tab, m, &cstart, [&](size_t i) { return (bp.sys[act[i]].d + 15) / 16; }, ctot))
        return BDS_EWORKSPACE;
    BDS_TRY(tab.upload(st));
    for (const LevelTab& L : lt)
        BDS_TRY(launch_solve_fwd<T>(SolLv<T>{}, L.recs, L.si, L.ss, L.cnt, L.ti, L.ts, L.np, L.tl, st));
    BDS_TRY(launch_coarse_solve(CoarseSol{}, cdev, cstart, (int)m, ctot, st));
    for (auto it = lt.rbegin(); it != lt.rend(); ++it)
        BDS_TRY(launch_solve_bwd<T>(SolLv<T>{}, it->recs, it->sb, it->cnt, it->tb, it->np, it->tl, st));
    return BDS_OK;
}

// Batched packing/unpacking of right-hand sides; nblk[i] blocks per record.
int pack_batched(const BatchPlan& bp, void* sws, const std::vector<PackRec>& recs, const std::vector<int64_t>& nblk,
                 hipStream_t st)
{
    if (recs.empty()) return BDS_OK;
    Table tab(sws, bp.rtab, bp.rtab_bytes);
    const PackRec* dev = nullptr;
    PackRec* h = tab.take<PackRec>(recs.size(), &dev);
    if (!h) return BDS_EWORKSPACE;
    std::copy(recs.begin(), recs.end(), h);
    const int64_t* start = nullptr;
    int64_t tot = 0;
    if (!fill_prefix(tab, recs.size(), &start, [&](size_t i) { return nblk[i]; }, tot)) return BDS_EWORKSPACE;
    BDS_TRY(tab.upload(st));
    BDS_TRY(launch_pack_tab(dev, start, (int)recs.size(), tot, st));
    return BDS_OK;
}

// X0[k] = A_k^-1 B0[k] for every system, refined in FP64 when prec != F64.
// All systems iterate together; a system leaves the iteration once its own
// stopping rule fires.  Synchronises the stream once per iteration.
template <typename T>
int refined_solve_batched(const BatchPlan& bp, const void* fws, const std::vector<Level0>& a0, void* sws,
                          const std::vector<const double*>& B0, const std::vector<double*>& X0, bds_info* info,
                          hipStream_t st)
{
    const int K = (int)bp.K;
    std::vector<int> act(K);
    for (int k = 0; k < K; ++k) act[k] = k;
    int rc = solve_core_batched<T>(bp, act, fws, sws, B0, X0, st);
    if (rc != BDS_OK) return rc;
    const SysPlan& p0 = bp.sys[0];
    std::vector<int> ic(2 * (size_t)K, 0);
    std::vector<double> prev((size_t)K, HUGE_VAL), h(2 * (size_t)K, 0.0);
    std::vector<double*> Rp(K), Cp(K);
    for (int k = 0; k < K; ++k) {
        Rp[k] = at<double>(sws, bp.sys[k].R);
        Cp[k] = at<double>(sws, bp.sys[k].Cr);
    }
    double* nrm = at<double>(sws, bp.nrm);
    for (int it = 1; it <= p0.max_refine && !act.empty(); ++it) {
        Table tab(sws, bp.rtab, bp.rtab_bytes);
        const size_t m = act.size();
        const AxpyArgs* xdev = nullptr;
        AxpyArgs* xh = tab.take<AxpyArgs>(m, &xdev);
        if (!xh) return BDS_EWORKSPACE;
        for (size_t i = 0; i < m; ++i) {
            const int k = act[i];
            const SysPlan& p = bp.sys[k];
            xh[i] = AxpyArgs{X0[k], Cp[k], at<double>(sws, p.Nrm), nrm + 2 * k, (int)p.N, (int)p.np, (int)p.d, 0};
        }
        const int64_t* xs = nullptr;
        int64_t xt = 0;
        if (!fill_prefix(tab, m, &xs, [&](size_t i) { return bp.sys[act[i]].N; }, xt)) return BDS_EWORKSPACE;
        // residuals, one launch per block-size group
        struct ResTab {
            const ResidArgs* recs;
            const int64_t* start;
            int64_t tot;
            int cnt, np;
        };
        std::vector<ResTab> rts;
        for (const auto& grp : bp.groups) {
            const int np = grp.np;
            std::vector<int> members;
            for (int k : act)
                if (bp.in_group(bp.sys[k], grp)) members.push_back(k);
            if (members.empty()) continue;
            ResTab r{nullptr, nullptr, 0, (int)members.size(), np};
            ResidArgs* rh = tab.take<ResidArgs>(members.size(), &r.recs);
            if (!rh) return BDS_EWORKSPACE;
            for (size_t i = 0; i < members.size(); ++i) {
                const int k = members[i];
                const SysPlan& p = bp.sys[k];
                rh[i] = ResidArgs{a0[k].Ad, a0[k].As, B0[k], X0[k], Rp[k], (int)p.N, (int)p.np, (int)p.d, 0};
            }
            if (!fill_prefix(tab, members.size(), &r.start,
                             [&](size_t i) {
                                 const SysPlan& p = bp.sys[members[i]];
                                 return units_resid((int)p.N, np, (int)p.d);
                             },
                             r.tot))
                return BDS_EWORKSPACE;
            rts.push_back(r);
        }
        BDS_TRY(tab.upload(st));
        for (const ResTab& r : rts) BDS_TRY(launch_residual(ResidArgs{}, r.recs, r.start, r.cnt, r.tot, r.np, st));
        rc = solve_core_batched<T>(bp, act, fws, sws, std::vector<const double*>(Rp.begin(), Rp.end()), Cp, st);
        if (rc != BDS_OK) return rc;
        BDS_TRY(launch_axpy_norm(AxpyArgs{}, xdev, xs, (int)m, xt, st));
        BDS_TRY(hipMemcpyAsync(h.data(), nrm, 2 * (size_t)K * sizeof(double), hipMemcpyDeviceToHost, st));
        BDS_TRY(hipStreamSynchronize(st));
        std::vector<int> still;
        for (int k : act) {
            ic[2 * k] = it;
            int conv = 0;
            if (refine_stop(std::sqrt(h[2 * k]), std::sqrt(h[2 * k + 1]), prev[k], p0.refine_tol, conv))
                ic[2 * k + 1] = conv;
            else
                still.push_back(k);
        }
        act.swap(still);
    }
    int* icd = at<int>(sws, bp.ic);
    BDS_TRY(hipMemcpyAsync(icd, ic.data(), ic.size() * sizeof(int), hipMemcpyHostToDevice, st));
    BDS_TRY(launch_set_refine_info_tab(info, icd, K, st));
    // the copy source must outlive the copy: wait for it before `ic` goes out of scope
    BDS_TRY(hipStreamSynchronize(st));
    return BDS_OK;
}

template <typename T>
int solve_batched_impl(const BatchPlan& bp, const void* fws, const double* const* Ad, const double* const* As,
                       const double* const* B, double* const* X, void* sws, bds_info* info, hipStream_t st)
{
    const int K = (int)bp.K;
    std::vector<const double*> B0(K);
    std::vector<double*> X0(K);
    std::vector<PackRec> packs;
    std::vector<int64_t> nblk;
    for (int k = 0; k < K; ++k) {
        const SysPlan& p = bp.sys[k];
        if (p.packed) {
            packs.push_back(PackRec{B[k], at<double>(sws, p.B0), (int)p.n, (int)p.np, (int)p.d, PACK_RHS});
            nblk.push_back(p.N);
            B0[k] = at<double>(sws, p.B0);
            X0[k] = at<double>(sws, p.X0);
        } else {
            B0[k] = B[k];
            X0[k] = X[k];
        }
    }
    int rc = pack_batched(bp, sws, packs, nblk, st);
    if (rc != BDS_OK) return rc;
    if (bp.prec == BDS_F64) {
        std::vector<int> act(K);
        for (int k = 0; k < K; ++k) act[k] = k;
        rc = solve_core_batched<T>(bp, act, fws, sws, B0, X0, st);
    } else {
        std::vector<Level0> a0(K);
        for (int k = 0; k < K; ++k) a0[k] = level0_matrices(bp.sys[k], Ad[k], As[k], fws);
        rc = refined_solve_batched<T>(bp, fws, a0, sws, B0, X0, info, st);
    }
    if (rc != BDS_OK) return rc;
    packs.clear();
    nblk.clear();
    for (int k = 0; k < K; ++k) {
        const SysPlan& p = bp.sys[k];
        if (!p.packed) continue;
        packs.push_back(PackRec{X0[k], X[k], (int)p.n, (int)p.np, (int)p.d, PACK_UNPACK_RHS});
        nblk.push_back(p.N);
    }
    return pack_batched(bp, sws, packs, nblk, st);
}

}  // namespace
}  // namespace bds

using namespace bds;

extern "C" {

int bds_batched_workspace_size(int64_t K, const bds_desc* descs, size_t* factor_bytes, size_t* solve_bytes)
{
    BatchPlan bp;
    const int rc = make_batch_plan(K, descs, bp);
    if (rc != BDS_OK) return rc;
    if (factor_bytes) *factor_bytes = bp.factor_bytes;
    if (solve_bytes) *solve_bytes = bp.solve_bytes;
    return BDS_OK;
}

int bds_factor_batched(int64_t K, const bds_desc* descs, const double* const* Ad, const double* const* As,
                       void* factor_ws, size_t factor_bytes, bds_info* info, void* stream)
{
    BatchPlan bp;
    const int rc = make_batch_plan(K, descs, bp);
    if (rc != BDS_OK) return rc;
    if (!Ad || !As || !factor_ws || !info) return BDS_EINVAL;
    for (int64_t k = 0; k < K; ++k)
        if (!Ad[k] || (descs[k].N > 1 && !As[k])) return BDS_EINVAL;
    if (factor_bytes < bp.factor_bytes) return BDS_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (bp.prec == BDS_F64) return factor_batched_impl<double>(bp, Ad, As, factor_ws, info, st);
    if (bp.prec == BDS_BF16) return factor_batched_impl<bf16x>(bp, Ad, As, factor_ws, info, st);
    return factor_batched_impl<float>(bp, Ad, As, factor_ws, info, st);
}

int bds_solve_batched(int64_t K, const bds_desc* descs, const void* factor_ws, size_t factor_bytes,
                      const double* const* Ad, const double* const* As, const double* const* B, double* const* X,
                      void* solve_ws, size_t solve_bytes, bds_info* info, void* stream)
{
    BatchPlan bp;
    const int rc = make_batch_plan(K, descs, bp);
    if (rc != BDS_OK) return rc;
    if (!factor_ws || !B || !X || !solve_ws || !info) return BDS_EINVAL;
    const bool refine = bp.prec != BDS_F64;
    if (refine && (!Ad || !As)) return BDS_EINVAL;
    for (int64_t k = 0; k < K; ++k) {
        if (!B[k] || !X[k] || B[k] == X[k]) return BDS_EINVAL;
        if (refine && (!Ad[k] || (descs[k].N > 1 && !As[k]))) return BDS_EINVAL;
    }
    if (factor_bytes < bp.factor_bytes || solve_bytes < bp.solve_bytes) return BDS_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (bp.prec == BDS_F64) return solve_batched_impl<double>(bp, factor_ws, Ad, As, B, X, solve_ws, info, st);
    return solve_batched_impl<float>(bp, factor_ws, Ad, As, B, X, solve_ws, info, st);
}

}  // extern "C"
