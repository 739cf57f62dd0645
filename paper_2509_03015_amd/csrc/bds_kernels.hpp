// Kernel argument records and launch entry points of libbds (host-visible).
//
// Every kernel reads its per-system arguments through a "table": either one
// record passed by value (single system) or a device array of records with
// an exclusive prefix sum of work units per record (batched systems, one
// launch per level across the whole batch).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/bds.h"
#include "bds_device.hpp"

namespace bds {

// One reduction level of one system (factorisation).
template <typename T, typename In> struct FacLv {
    const In* Ad;   // M diagonal blocks of this level (np x np, lower triangle read)
    const In* As;   // M-1 sub-diagonal blocks
    T* Li;          // E interiors: inverse Cholesky factor
    T* Wt;          // E interiors: A[i-1,i] * Li^T  (= (Li A[i,i-1])^T)
    T* Pr;          // E interiors: A[i+1,i] * Li^T
    T* Adn;         // Mn next-level diagonal blocks
    T* Asn;         // Mn-1 next-level sub-diagonal blocks
    int M, np, level, pad;
    bds_info* info;
};

// Coarse system of one system (sequential block Cholesky, FP64).
template <typename In> struct CoarseFac {
    const In* Ad;
    const In* As;
    double* Lc;     // Mc: inverse Cholesky factors of the pivots
    double* Lsc;    // Mc-1: A[i+1,i] Lc[i]^T
    double* Cw;     // 1 block scratch
    int Mc, np, level, pad;
    bds_info* info;
};

// One reduction level of one system (solve); vectors FP64, np x d blocks, ld d.
template <typename T> struct SolLv {
    const T* Li;
    const T* Wt;
    const T* Pr;
    const double* B;   // M blocks: right-hand side of this level
    double* Y;         // E blocks
    double* Bn;        // Mn blocks
    const double* Xn;  // Mn blocks
    double* X;         // M blocks: solution of this level
    int M, np, d, pad;
};

struct CoarseSol {
    const double* Lc;
    const double* Lsc;
    const double* B;
    double* Y;
    double* X;
    int Mc, np, d, pad;
};

// Refinement helpers: residual R = B - A X over the whole (padded) system.
struct ResidArgs {
    const double* Ad;  // N blocks np x np (ld np), lower triangle read
    const double* As;  // N-1 blocks
    const double* B;   // N blocks np x d
    const double* X;
    double* R;
    int N, np, d, pad;
};

struct AxpyArgs {
    double* X;          // N blocks np x d: X += C
    const double* C;
    double* part;       // 2 * N partial sums (sum C^2, sum X^2 per block)
    double* out;        // 2 final sums
    int N, np, d, pad;
};

struct AdjArgs {
    const double* G;    // N blocks np x d (padded)
    const double* X;    // N blocks np x d (padded)
    double* dAd;        // N blocks n x n (ld n)
    double* dAs;        // N-1 blocks n x n
    int N, n, np, d;
};

// Batched packing between the user's n-row blocks and the padded np-row blocks.
enum { PACK_RHS = 0, PACK_DIAG = 1, PACK_OFFDIAG = 2, PACK_UNPACK_RHS = 3 };
struct PackRec {
    const double* src;
    double* dst;
    int n, np, cols, mode;  // cols: d for right-hand sides (unused for matrix blocks)
};

// Tile shapes of one system's reduction levels (BDS_TILE_* codes of bds.h),
// resolved from bds_desc::tiles with the library's rule for the zero fields.
struct Tiling {
    int couple = BDS_TILE_W16;  // coupling products
    int schur = BDS_TILE_W16;   // Schur updates
    int sol = BDS_TILE_W16;     // solve sweeps (wave tiles)
    bool operator==(const Tiling& o) const { return couple == o.couple && schur == o.schur && sol == o.sol; }
    bool operator<(const Tiling& o) const
    {
        return couple != o.couple ? couple < o.couple : schur != o.schur ? schur < o.schur : sol < o.sol;
    }
};
// false if a field is not a known code or does not fit the padded block size np.
bool resolve_tiling(int np, int prec, int32_t tiles, Tiling& out);
// Tile codes that fit np for one field (couple/schur: all; solve: wave tiles).
std::vector<int> tile_choices(int np, bool solve);
// Tiling of one reduction level of M blocks: tl, except that the coupling and
// Schur fields the caller left to the library (zero in req) take per-wave
// 16 x 16 tiles on levels where the work-group tiles would launch no more
// work-groups than the device has CUs.
Tiling level_tiling(const Tiling& tl, int32_t req, int M, int np);

// Work-unit counts per record (waves for wave kernels, work-groups otherwise).
// tile_r(np) is the wave tile factor (a wave computes (16R) x (16R) outputs)
// of the kernels that are not tuned (residual, coarse system).  A table
// passed to a launcher holds records of one np and one Tiling.
int tile_r(int np);
int64_t units_fac_diag(int M);
int64_t units_fac_couple(int M, int np, int code);
int64_t units_fac_schur(int M, int np, int code);
int64_t units_sol_fwd_int(int M, int np, int d, int code);
int64_t units_sol_fwd_sep(int M, int np, int d, int code);
int64_t units_sol_bwd(int M, int d);
int64_t units_resid(int N, int np, int d);

// Launchers.  tab_dev/start_dev == nullptr: single record passed by value.
// Otherwise K records at tab_dev with exclusive prefix sums start_dev (K+1).
// C: compute tag (double, float, or bf16x = FP32 storage with bfloat16 MFMA operands).
template <typename C, typename In>
hipError_t launch_factor_level(const FacLv<typename Stor<C>::type, In>& one,
                               const FacLv<typename Stor<C>::type, In>* tab_dev,
                               const int64_t* start_diag, const int64_t* start_couple,
                               const int64_t* start_schur, int K, int64_t tot_diag,
                               int64_t tot_couple, int64_t tot_schur, int np, const Tiling& tl, hipStream_t st);

template <typename In>
hipError_t launch_coarse_factor(const CoarseFac<In>& one, const CoarseFac<In>* tab_dev, int K, int np_max,
                                hipStream_t st);

template <typename T>
hipError_t launch_solve_fwd(const SolLv<T>& one, const SolLv<T>* tab_dev, const int64_t* start_int,
                            const int64_t* start_sep, int K, int64_t tot_int, int64_t tot_sep,
                            int np, const Tiling& tl, hipStream_t st);

template <typename T>
hipError_t launch_solve_bwd(const SolLv<T>& one, const SolLv<T>* tab_dev, const int64_t* start,
                            int K, int64_t tot, int np, const Tiling& tl, hipStream_t st);

hipError_t launch_coarse_solve(const CoarseSol& one, const CoarseSol* tab_dev, const int64_t* start,
                               int K, int64_t tot, hipStream_t st);

hipError_t launch_residual(const ResidArgs& one, const ResidArgs* tab_dev, const int64_t* start, int K,
                           int64_t tot, int np, hipStream_t st);

hipError_t launch_axpy_norm(const AxpyArgs& one, const AxpyArgs* tab_dev, const int64_t* start, int K,
                            int64_t tot, hipStream_t st);

hipError_t launch_adjoint(const AdjArgs& a, hipStream_t st);

hipError_t launch_pack_blocks(const double* src, double* dst, int64_t nblk, int n, int np, bool diag,
                              hipStream_t st);
hipError_t launch_pack_rhs(const double* src, double* dst, int64_t nblk, int n, int np, int d,
                           hipStream_t st);
hipError_t launch_unpack_rhs(const double* src, double* dst, int64_t nblk, int n, int np, int d,
                             hipStream_t st);
hipError_t launch_pack_tab(const PackRec* tab, const int64_t* start, int K, int64_t tot, hipStream_t st);
hipError_t launch_set_refine_info_tab(bds_info* info, const int* ic, int K, hipStream_t st);
hipError_t launch_clear_info(bds_info* info, int K, hipStream_t st);
hipError_t launch_set_refine_info(bds_info* info, int iters, int converged, hipStream_t st);

}  // namespace bds
