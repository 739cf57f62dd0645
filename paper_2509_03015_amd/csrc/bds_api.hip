// C ABI of libbds: argument checks, level plans, and the launch sequences of
// the recursive factorisation (Alg. 4), the recursive solve (Alg. 5-7), the
// mixed-precision refinement and the adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/bds.h"
#include "bds_graph.hpp"
#include "bds_host.hpp"
#include "bds_kernels.hpp"
#include "bds_plan.hpp"

namespace bds {

int check_desc(const bds_desc* d)
{
    if (!d) return BDS_EINVAL;
    if (d->N < 1 || d->N > (int64_t(1) << 30)) return BDS_EINVAL;
    if (d->n < 1 || d->n > kMaxN) return BDS_EINVAL;
    if (d->d < 1 || d->d > 65536) return BDS_EINVAL;
    if (d->prec != BDS_F64 && d->prec != BDS_F32 && d->prec != BDS_BF16) return BDS_EINVAL;
    if (d->nstar < 0 || d->max_refine < 0 || !(d->refine_tol >= 0)) return BDS_EINVAL;
    Tiling t;
    if (!resolve_tiling((int)round_up(d->n, 16), d->prec, d->tiles, t)) return BDS_EINVAL;
    return BDS_OK;
}

SysPlan make_plan(const bds_desc& d, size_t base_f, size_t base_s)
{
    SysPlan p;
    p.N = d.N;
    p.n = d.n;
    p.np = round_up(d.n, 16);
    p.d = d.d;
    p.prec = d.prec;
    p.nstar = d.nstar > 0 ? d.nstar : kDefaultNstar;
    p.max_refine = d.max_refine > 0 ? d.max_refine : kDefaultMaxRefine;
    p.refine_tol = d.refine_tol > 0 ? d.refine_tol : kDefaultRefineTol;
    p.esize = matrix_elem_bytes(d.prec);
    p.packed = p.np != p.n;
    resolve_tiling((int)p.np, p.prec, d.tiles, p.tl);  // checked by check_desc
    p.tiles_req = d.tiles;
    size_t f = base_f, s = base_s;
    auto take = [](size_t& off, size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t blk = (size_t)(p.np * p.np);
    const size_t bv = (size_t)(p.np * p.d) * sizeof(double);
    if (p.packed) {
        p.Ad0 = take(f, (size_t)p.N * blk * 8);
        p.As0 = take(f, (size_t)std::max<int64_t>(p.N - 1, 0) * blk * 8);
    }
    int64_t M = p.N;
    while (M > p.nstar) {
        LevelPlan L;
        L.M = M;
        L.E = M / 2;
        L.Mn = (M + 1) / 2;
        L.Li = take(f, (size_t)L.E * blk * p.esize);
        L.Wt = take(f, (size_t)L.E * blk * p.esize);
        L.Pr = take(f, (size_t)L.E * blk * p.esize);
        L.Adn = take(f, (size_t)L.Mn * blk * p.esize);
        L.Asn = take(f, (size_t)std::max<int64_t>(L.Mn - 1, 0) * blk * p.esize);
        L.Y = take(s, (size_t)L.E * bv);
        L.Bn = take(s, (size_t)L.Mn * bv);
        L.Xn = take(s, (size_t)L.Mn * bv);
        p.lv.push_back(L);
        M = L.Mn;
    }
    p.Mc = M;
    p.Lc = take(f, (size_t)p.Mc * blk * 8);
    p.Lsc = take(f, (size_t)std::max<int64_t>(p.Mc - 1, 0) * blk * 8);
    p.Cw = take(f, blk * 8);
    p.Yc = take(s, (size_t)p.Mc * bv);
    if (p.packed) {
        p.B0 = take(s, (size_t)p.N * bv);
        p.X0 = take(s, (size_t)p.N * bv);
    }
    p.G = take(s, (size_t)p.N * bv);
    if (p.prec != BDS_F64) {
        p.R = take(s, (size_t)p.N * bv);
        p.Cr = take(s, (size_t)p.N * bv);
        p.Nrm = take(s, (size_t)(2 * p.N + 2) * sizeof(double));
    }
    p.factor_bytes = f - base_f;
    p.solve_bytes = s - base_s;
    return p;
}

Level0 level0_matrices(const SysPlan& p, const double* Ad, const double* As, const void* fws)
{
    if (p.packed) return {at<double>(fws, p.Ad0), at<double>(fws, p.As0)};
    return {Ad, As};
}

namespace {

template <typename C>
int factor_impl(const SysPlan& p, const double* Ad, const double* As, void* fws, bds_info* info, hipStream_t st)
{
    using T = typename Stor<C>::type;
    BDS_TRY(launch_clear_info(info, 1, st));
    if (p.packed) {
        BDS_TRY(launch_pack_blocks(Ad, at<double>(fws, p.Ad0), p.N, (int)p.n, (int)p.np, true, st));
        BDS_TRY(launch_pack_blocks(As, at<double>(fws, p.As0), p.N - 1, (int)p.n, (int)p.np, false, st));
    }
    const Level0 a0 = level0_matrices(p, Ad, As, fws);
    const int np = (int)p.np;
    for (size_t l = 0; l < p.lv.size(); ++l) {
        const LevelPlan& L = p.lv[l];
        const int M = (int)L.M;
        const Tiling lt = level_tiling(p.tl, p.tiles_req, M, np);
        if (l == 0) {
            FacLv<T, double> r{a0.Ad, a0.As, at<T>(fws, L.Li), at<T>(fws, L.Wt), at<T>(fws, L.Pr),
                               at<T>(fws, L.Adn), at<T>(fws, L.Asn), M, np, 0, 0, info};
            BDS_TRY(launch_factor_level<C, double>(r, nullptr, nullptr, nullptr, nullptr, 1, units_fac_diag(M),
                                                   units_fac_couple(M, np, lt.couple),
                                                   units_fac_schur(M, np, lt.schur), np, lt, st));
        } else {
            const LevelPlan& P = p.lv[l - 1];
            FacLv<T, T> r{at<T>(fws, P.Adn), at<T>(fws, P.Asn), at<T>(fws, L.Li), at<T>(fws, L.Wt),
                          at<T>(fws, L.Pr), at<T>(fws, L.Adn), at<T>(fws, L.Asn), M, np, (int)l, 0, info};
            BDS_TRY(launch_factor_level<C, T>(r, nullptr, nullptr, nullptr, nullptr, 1, units_fac_diag(M),
                                              units_fac_couple(M, np, lt.couple),
                                              units_fac_schur(M, np, lt.schur), np, lt, st));
        }
    }
    const int Lv = (int)p.lv.size();
    if (Lv == 0) {
        CoarseFac<double> c{a0.Ad, a0.As, at<double>(fws, p.Lc), at<double>(fws, p.Lsc), at<double>(fws, p.Cw),
                            (int)p.Mc, np, 0, 0, info};
        BDS_TRY(launch_coarse_factor<double>(c, nullptr, 1, np, st));
    } else {
        const LevelPlan& P = p.lv.back();
        CoarseFac<T> c{at<T>(fws, P.Adn), at<T>(fws, P.Asn), at<double>(fws, p.Lc), at<double>(fws, p.Lsc),
                       at<double>(fws, p.Cw), (int)p.Mc, np, Lv, 0, info};
        BDS_TRY(launch_coarse_factor<T>(c, nullptr, 1, np, st));
    }
    return BDS_OK;
}

// One solve through the stored hierarchy: B0 -> X0, both padded (N, np, d).
template <typename T>
int solve_core(const SysPlan& p, const void* fws, void* sws, const double* B0, double* X0, hipStream_t st)
{
    const int np = (int)p.np, d = (int)p.d;
    const int Lv = (int)p.lv.size();
    std::vector<SolLv<T>> recs(Lv);
    for (int l = 0; l < Lv; ++l) {
        const LevelPlan& L = p.lv[l];
        const double* B = l == 0 ? B0 : at<double>(sws, p.lv[l - 1].Bn);
        double* X = l == 0 ? X0 : at<double>(sws, p.lv[l - 1].Xn);
        recs[l] = SolLv<T>{at<T>(fws, L.Li), at<T>(fws, L.Wt), at<T>(fws, L.Pr), B, at<double>(sws, L.Y),
                           at<double>(sws, L.Bn), at<double>(sws, L.Xn), X, (int)L.M, np, d, 0};
        BDS_TRY(launch_solve_fwd<T>(recs[l], nullptr, nullptr, nullptr, 1, units_sol_fwd_int((int)L.M, np, d, p.tl.sol),
                                    units_sol_fwd_sep((int)L.M, np, d, p.tl.sol), np, p.tl, st));
    }
    CoarseSol c{at<double>(fws, p.Lc), at<double>(fws, p.Lsc),
                Lv == 0 ? B0 : at<double>(sws, p.lv.back().Bn), at<double>(sws, p.Yc),
                Lv == 0 ? X0 : at<double>(sws, p.lv.back().Xn), (int)p.Mc, np, d, 0};
    BDS_TRY(launch_coarse_solve(c, nullptr, nullptr, 1, (d + 15) / 16, st));
    for (int l = Lv - 1; l >= 0; --l)
        BDS_TRY(launch_solve_bwd<T>(recs[l], nullptr, nullptr, 1, units_sol_bwd((int)p.lv[l].M, d), np, p.tl, st));
    return BDS_OK;
}

// X0 = A^-1 B0 with iterative refinement in FP64 around the low-precision
// hierarchy (prec != F64).  Synchronises the stream once per iteration.
template <typename T>
int refined_solve(const SysPlan& p, const void* fws, const Level0& a0, void* sws, const double* B0, double* X0,
                  bds_info* info, hipStream_t st)
{
    int rc = solve_core<T>(p, fws, sws, B0, X0, st);
    if (rc != BDS_OK) return rc;
    const int np = (int)p.np, d = (int)p.d, N = (int)p.N;
    double* R = at<double>(sws, p.R);
    double* C = at<double>(sws, p.Cr);
    double* nrm = at<double>(sws, p.Nrm);
    ResidArgs ra{a0.Ad, a0.As, B0, X0, R, N, np, d, 0};
    AxpyArgs xa{X0, C, nrm, nrm + 2 * N, N, np, d, 0};
    int iters = 0, converged = 0;
    double prev = HUGE_VAL;
    for (int it = 1; it <= p.max_refine; ++it) {
        BDS_TRY(launch_residual(ra, nullptr, nullptr, 1, units_resid(N, np, d), np, st));
        rc = solve_core<T>(p, fws, sws, R, C, st);
        if (rc != BDS_OK) return rc;
        BDS_TRY(launch_axpy_norm(xa, nullptr, nullptr, 1, N, st));
        double h[2] = {0, 0};
        BDS_TRY(hipMemcpyAsync(h, nrm + 2 * N, sizeof(h), hipMemcpyDeviceToHost, st));
        BDS_TRY(hipStreamSynchronize(st));
        iters = it;
        if (refine_stop(std::sqrt(h[0]), std::sqrt(h[1]), prev, p.refine_tol, converged)) break;
    }
    BDS_TRY(launch_set_refine_info(info, iters, converged, st));
    return BDS_OK;
}

template <typename T>
int solve_impl(const SysPlan& p, const void* fws, const double* Ad, const double* As, const double* B, double* X,
               void* sws, bds_info* info, hipStream_t st)
{
    const int np = (int)p.np, n = (int)p.n, d = (int)p.d;
    const double* B0 = B;
    double* X0 = X;
    if (p.packed) {
        BDS_TRY(launch_pack_rhs(B, at<double>(sws, p.B0), p.N, n, np, d, st));
        B0 = at<double>(sws, p.B0);
        X0 = at<double>(sws, p.X0);
    }
    int rc;
    if (p.prec == BDS_F64) {
        rc = solve_core<T>(p, fws, sws, B0, X0, st);
    } else {
        const Level0 a0 = level0_matrices(p, Ad, As, fws);
        rc = refined_solve<T>(p, fws, a0, sws, B0, X0, info, st);
    }
    if (rc != BDS_OK) return rc;
    if (p.packed) BDS_TRY(launch_unpack_rhs(X0, X, p.N, n, np, d, st));
    return BDS_OK;
}

template <typename T>
int backward_impl(const SysPlan& p, const void* fws, const double* Ad, const double* As, const double* X,
                  const double* dX, double* dAd, double* dAs, double* dB, void* sws, bds_info* info,
                  hipStream_t st)
{
    const int np = (int)p.np, n = (int)p.n, d = (int)p.d;
    // G = A^-1 dX in padded layout
    const double* W0 = dX;
    const double* Xp = X;
    double* G = at<double>(sws, p.G);
    if (p.packed) {
        BDS_TRY(launch_pack_rhs(dX, at<double>(sws, p.B0), p.N, n, np, d, st));
        BDS_TRY(launch_pack_rhs(X, at<double>(sws, p.X0), p.N, n, np, d, st));
        W0 = at<double>(sws, p.B0);
        Xp = at<double>(sws, p.X0);
    }
    int rc;
    if (p.prec == BDS_F64) {
        rc = solve_core<T>(p, fws, sws, W0, G, st);
    } else {
        const Level0 a0 = level0_matrices(p, Ad, As, fws);
        rc = refined_solve<T>(p, fws, a0, sws, W0, G, info, st);
    }
    if (rc != BDS_OK) return rc;
    if (p.packed)
        BDS_TRY(launch_unpack_rhs(G, dB, p.N, n, np, d, st));
    else
        BDS_TRY(hipMemcpyAsync(dB, G, (size_t)(p.N * np * d) * sizeof(double), hipMemcpyDeviceToDevice, st));
    AdjArgs aa{G, Xp, dAd, dAs, (int)p.N, n, np, d};
    BDS_TRY(launch_adjoint(aa, st));
    return BDS_OK;
}

}  // namespace
}  // namespace bds

using namespace bds;

extern "C" {

int bds_workspace_size(const bds_desc* desc, size_t* factor_bytes, size_t* solve_bytes)
{
    const int rc = check_desc(desc);
    if (rc != BDS_OK) return rc;
    const SysPlan p = make_plan(*desc);
    if (factor_bytes) *factor_bytes = p.factor_bytes;
    if (solve_bytes) *solve_bytes = p.solve_bytes;
    return BDS_OK;
}

int bds_factor(const bds_desc* desc, const double* Ad, const double* As, void* factor_ws, size_t factor_bytes,
               bds_info* info, void* stream)
{
    const int rc = check_desc(desc);
    if (rc != BDS_OK) return rc;
    if (!Ad || (desc->N > 1 && !As) || !factor_ws || !info) return BDS_EINVAL;
    const SysPlan p = make_plan(*desc);
    if (factor_bytes < p.factor_bytes) return BDS_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    GraphKey key;
    key.kind = 1;
    key.add_desc(*desc);
    key.add(Ad);
    key.add(As);
    key.add(factor_ws);
    key.add(info);
    return run_graph(key, st, [&](hipStream_t s) {
        if (p.prec == BDS_F64) return factor_impl<double>(p, Ad, As, factor_ws, info, s);
        if (p.prec == BDS_BF16) return factor_impl<bf16x>(p, Ad, As, factor_ws, info, s);
        return factor_impl<float>(p, Ad, As, factor_ws, info, s);
    });
}

int bds_solve(const bds_desc* desc, const void* factor_ws, size_t factor_bytes, const double* Ad, const double* As,
              const double* B, double* X, void* solve_ws, size_t solve_bytes, bds_info* info, void* stream)
{
    const int rc = check_desc(desc);
    if (rc != BDS_OK) return rc;
    if (!factor_ws || !B || !X || !solve_ws || !info || B == X) return BDS_EINVAL;
    if (desc->prec != BDS_F64 && (!Ad || (desc->N > 1 && !As))) return BDS_EINVAL;
    const SysPlan p = make_plan(*desc);
    if (factor_bytes < p.factor_bytes || solve_bytes < p.solve_bytes) return BDS_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p.prec == BDS_F64) {
        // a fixed launch sequence: replayed as a graph
        GraphKey key;
        key.kind = 2;
        key.add_desc(*desc);
        key.add(factor_ws);
        key.add(B);
        key.add(X);
        key.add(solve_ws);
        key.add(info);
        return run_graph(key, st, [&](hipStream_t s) {
            return solve_impl<double>(p, factor_ws, Ad, As, B, X, solve_ws, info, s);
        });
    }
    // refinement synchronises once per iteration to test its stopping rule
    return solve_impl<float>(p, factor_ws, Ad, As, B, X, solve_ws, info, st);
}

int bds_backward(const bds_desc* desc, const void* factor_ws, size_t factor_bytes, const double* Ad,
                 const double* As, const double* X, const double* dX, double* dAd, double* dAs, double* dB,
                 void* solve_ws, size_t solve_bytes, bds_info* info, void* stream)
{
    const int rc = check_desc(desc);
    if (rc != BDS_OK) return rc;
    if (!factor_ws || !X || !dX || !dAd || (desc->N > 1 && !dAs) || !dB || !solve_ws || !info) return BDS_EINVAL;
    if (desc->prec != BDS_F64 && (!Ad || (desc->N > 1 && !As))) return BDS_EINVAL;
    const SysPlan p = make_plan(*desc);
    if (factor_bytes < p.factor_bytes || solve_bytes < p.solve_bytes) return BDS_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p.prec == BDS_F64) return backward_impl<double>(p, factor_ws, Ad, As, X, dX, dAd, dAs, dB, solve_ws, info, st);
    return backward_impl<float>(p, factor_ws, Ad, As, X, dX, dAd, dAs, dB, solve_ws, info, st);
}

const char* bds_version(void) { return "libbds 0.1 gfx950"; }

}  // extern "C"
