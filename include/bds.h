/*
 * bds.h -- C ABI of libbds, an MI355X (gfx950) solver for symmetric positive
 * definite block-tridiagonal systems A X = B by recursive Schur-complement
 * (block cyclic) reduction.
 *
 * The system (eq. (1) of the paper): A has N diagonal blocks A_ii and N-1
 * coupling blocks, each n x n; X and B have N row blocks of n rows and d
 * columns.  The factorisation follows the paper's recursive factorisation
 * (Sec. 3.3, Alg. 4): at each level the odd-numbered blocks (0-based) are the
 * interiors and the even-numbered ones the separators (segment length 1, the
 * odd-even form of the symmetric permutation of eqs. (2)-(4)); the interior
 * blocks are factorised (potrf), their coupling blocks solved against the
 * factor (trsm), and the separator Schur complement S of eq. (5) is formed
 * (Alg. 3) and reduced again, until at most `nstar` blocks remain, which are
 * factorised by sequential block Cholesky (Alg. 1 with one chain).  The solve
 * follows the recursive solve (Sec. 3.4, Alg. 5-7).
 *
 * Memory and layout.  Every array argument named as a device pointer lives in
 * GPU memory of the current HIP device; all are row-major (C order):
 *   Ad  (N, n, n)    diagonal blocks A_ii, FP64.  Only the lower triangle
 *                    (including the diagonal) is read; the block is taken to
 *                    be its symmetric completion.
 *   As  (N-1, n, n)  sub-diagonal blocks As[i] = A_{i+1,i}, FP64; the block
 *                    above the diagonal is As[i]^T.  May be NULL when N == 1.
 *   B, X (N, n, d)   right-hand sides and solution, FP64.
 * The caller owns every buffer, including the workspaces, whose sizes come
 * from bds_workspace_size / bds_batched_workspace_size.  The library never
 * allocates device memory inside these calls.  All calls are asynchronous on
 * the given stream (a hipStream_t passed as void*; NULL is the null stream),
 * except where a function says it synchronises.
 *
 * Lifetime.  A factor workspace, together with the unchanged Ad and As it was
 * built from, must stay alive while any solve or backward call that reads it
 * is in flight.  Calls that share a workspace must not overlap.
 *
 * Errors.  The return value reports what the host can see: BDS_EINVAL for a
 * bad argument (nothing launched), BDS_EWORKSPACE for a workspace smaller than
 * required (nothing launched), BDS_EHIP for a failed launch or HIP call.
 * Numerical outcomes are written to the device-side bds_info record(s):
 * status BDS_ENOTSPD when a pivot of a block factorisation is not positive or
 * is NaN (then the factor must not be used), BDS_ENOCONV when mixed-precision
 * refinement did not reach its tolerance within its iteration cap.  The info
 * record is cleared by bds_factor; solves add their own status without
 * clearing an earlier failure.
 */
#ifndef BDS_H
#define BDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return and info status codes. */
enum {
    BDS_OK = 0,
    BDS_EINVAL = 1,
    BDS_ENOTSPD = 2,
    BDS_ENOCONV = 3,
    BDS_EWORKSPACE = 4,
    BDS_EHIP = 5
};

/*
 * Factor precision.  The paper computes in FP64 and mentions single-precision
 * support (Sec. 1).  BDS_F32 and BDS_BF16 factor the reduction levels in low
 * precision (BF16: operands rounded to bfloat16, products accumulated in FP32)
 * while the coarsest system is factorised in FP64; bds_solve then recovers
 * FP64 accuracy by iterative refinement with an FP64 residual B - A X and an
 * FP64 update of X.
 */
enum { BDS_F64 = 0, BDS_F32 = 1, BDS_BF16 = 2 };

/* Problem description (host struct). */
typedef struct bds_desc {
    int64_t N;          /* number of diagonal blocks, >= 1 */
    int64_t n;          /* block size, 1 <= n <= 256 */
    int64_t d;          /* right-hand sides, >= 1 */
    int32_t prec;       /* BDS_F64, BDS_F32 or BDS_BF16 */
    int32_t nstar;      /* recursion stops once a level has <= nstar blocks
                           (the paper's crossover N_star); 0 = library choice */
    int32_t max_refine; /* refinement iteration cap for prec != BDS_F64; 0 = default (30) */
    int32_t tiles;      /* tile shapes, BDS_TILES(couple, schur, solve); 0 = library rule */
    double refine_tol;  /* stop when the estimated remaining error is <= refine_tol * ||X||_F:
                           ||dX||_F itself, or rho * ||dX||_F once the contraction rho of
                           successive corrections is known; 0 = default (1e-14) */
} bds_desc;

/*
 * Tile shapes (bds_desc.tiles).  Each field selects how one step of a
 * reduction level is cut into work for the GPU; BDS_TILE_RULE leaves it to
 * the library's rule (a function of the padded block size np and the
 * precision; for the coupling and Schur fields of bds_factor also of the
 * level: levels whose work-group tiles would launch no more work-groups than
 * the device has CUs take W16), which is also what bds_tune starts from.
 *   couple: the coupling products of Alg. 4 (trsm as products with the
 *           stored inverse factor);
 *   schur:  the Schur updates of Alg. 3;
 *   solve:  the forward and backward sweeps of Alg. 5-7 (wave tiles only).
 * BDS_TILE_W16 / W32: one wavefront per 16 x 16 / 32 x 32 output tile, operands
 * read directly (W32 needs np % 32 == 0).  BDS_TILE_G64 / G128: a work-group
 * of four wavefronts per 64 x 64 / 128 x 128 output tile, operands staged
 * through LDS (need np % 64 == 0 / np % 128 == 0).  np = n rounded up to a
 * multiple of 16.  A choice that does not fit np is rejected with BDS_EINVAL.
 * Every choice computes the same result up to rounding.
 */
enum { BDS_TILE_RULE = 0, BDS_TILE_W16 = 1, BDS_TILE_W32 = 2, BDS_TILE_G64 = 3, BDS_TILE_G128 = 4 };
#define BDS_TILES(couple, schur, solve) ((int32_t)((couple) | ((schur) << 4) | ((solve) << 8)))

/* Device-side outcome record, written by the kernels (8 x int32). */
typedef struct bds_info {
    int32_t status;     /* BDS_OK, BDS_ENOTSPD or BDS_ENOCONV */
    int32_t level;      /* reduction level of a failed pivot (-1 = coarse system) */
    int32_t position;   /* block position within that level */
    int32_t orig_block; /* index of that block in the original ordering */
    int32_t column;     /* column of the failed pivot within the block */
    int32_t iters;      /* refinement iterations taken by the last solve */
    int32_t converged;  /* 1 if the last refined solve met its tolerance */
    int32_t reserved;
} bds_info;

/*
 * Workspace sizes in bytes for one system described by *desc (host only, no
 * GPU work).  factor_bytes: the factor hierarchy (per-level factors, coupling
 * solves and Schur complements of Alg. 4, plus the coarse factor).
 * solve_bytes: per-level right-hand sides and solutions of Alg. 7 for desc->d
 * columns, plus refinement buffers when desc->prec != BDS_F64.
 */
int bds_workspace_size(const bds_desc* desc, size_t* factor_bytes, size_t* solve_bytes);

/*
 * Factorise A (Alg. 4).  Ad, As: device pointers (layout above).  factor_ws:
 * device buffer of factor_bytes.  info: device pointer to one bds_info, which
 * is cleared and then receives BDS_ENOTSPD with the failing pivot's level,
 * position, original block and column if A is not numerically SPD.
 */
int bds_factor(const bds_desc* desc, const double* Ad, const double* As, void* factor_ws,
               size_t factor_bytes, bds_info* info, void* stream);

/*
 * Solve A X = B with a factor from bds_factor (Alg. 7).  B, X: device
 * pointers (N, n, d); X may not alias B.  For desc->prec == BDS_F64, Ad and
 * As are not read and may be NULL.  Otherwise they must be the arrays the
 * factor was built from: the call runs refinement, X_0 = solve(B), then
 * R = B - A X (FP64), C = solve(R), X += C (FP64) until the tolerance or the
 * cap, and it synchronises the stream once per iteration to test the
 * stopping rule; info receives iters, converged and, on failure, BDS_ENOCONV.
 */
int bds_solve(const bds_desc* desc, const void* factor_ws, size_t factor_bytes, const double* Ad,
              const double* As, const double* B, double* X, void* solve_ws, size_t solve_bytes,
              bds_info* info, void* stream);

/*
 * Adjoint of X = A^{-1} B for a scalar loss with gradient dX = dL/dX (the
 * paper does not differentiate; this follows from dX = -A^{-1} dA X).
 * With G = A^{-1} dX (one more solve with the stored factor):
 *   dB     = G                                          (N, n, d)
 *   dAd[i] = -(G_i X_i^T + X_i G_i^T) / 2               (N, n, n), symmetric
 *   dAs[i] = -(G_{i+1} X_i^T + X_{i+1} G_i^T)           (N-1, n, n)
 * All pointers are device pointers; X is the solution of the forward solve.
 * dAd and dAs are the gradients with respect to symmetric diagonal blocks and
 * to the coupling blocks A_{i+1,i}.  Ad/As are read only when desc->prec !=
 * BDS_F64 (the solve for G is then refined like bds_solve).
 */
int bds_backward(const bds_desc* desc, const void* factor_ws, size_t factor_bytes,
                 const double* Ad, const double* As, const double* X, const double* dX,
                 double* dAd, double* dAs, double* dB, void* solve_ws, size_t solve_bytes,
                 bds_info* info, void* stream);

/*
 * Batched form: K independent systems, each with its own (N, n, d) and the
 * shared precision and nstar of descs[0] (the paper's batch notation
 * {A^(k)}, Sec. 3.2).  Every level of every system is processed by one launch
 * per kernel and level across the whole batch.  descs: host array of K.
 */
int bds_batched_workspace_size(int64_t K, const bds_desc* descs, size_t* factor_bytes,
                               size_t* solve_bytes);

/*
 * Ad, As: host arrays of K device pointers (As[k] may be NULL when N_k == 1).
 * info: device array of K bds_info.  The factor workspace also stores the
 * batch's task tables, so solves must pass the same descs.
 */
int bds_factor_batched(int64_t K, const bds_desc* descs, const double* const* Ad,
                       const double* const* As, void* factor_ws, size_t factor_bytes,
                       bds_info* info, void* stream);

/*
 * B, X: host arrays of K device pointers.  Ad/As as for bds_factor_batched
 * (read only for refinement, may be NULL for BDS_F64).  Refinement runs all
 * systems together and stops when every system has met its tolerance or the
 * cap is reached; each system's info gets its own iters/converged.
 */
int bds_solve_batched(int64_t K, const bds_desc* descs, const void* factor_ws,
                      size_t factor_bytes, const double* const* Ad, const double* const* As,
                      const double* const* B, double* const* X, void* solve_ws,
                      size_t solve_bytes, bds_info* info, void* stream);

/*
 * Autotuner.  Times factor + solve of the caller's system for a sequence of
 * configurations and writes the fastest descriptor to *best (nstar and tiles
 * chosen; every other field copied from *desc).  Coordinate search from the
 * library's choices: nstar over {1, 2, 4, ..., 64} (up to N), then each tile
 * field the caller left at zero over the shapes that fit np, against zero
 * itself (the library's choice, which for the coupling and Schur fields of a
 * single system takes per-wave tiles on levels too small for work-group
 * tiles); a field of *best stays zero where that wins.  Each candidate is run once untimed and
 * timed over `reps` runs (reps <= 0: 3) with HIP events on `stream`.  The
 * search excludes workspace sizing and is meant to run once per problem
 * shape, before the timed work (the paper's Init phase).
 * Arguments as for bds_factor + bds_solve; the workspaces must have the sizes
 * given by bds_tune_workspace_size (the largest over the candidates).  On
 * return factor_ws holds the factor of *best and X its solution.  The stream
 * is synchronised.  Returns BDS_OK or the first error of a candidate run;
 * a candidate that reports a numerical failure in info ends the search with
 * that status left in info.
 */
int bds_tune_workspace_size(const bds_desc* desc, size_t* factor_bytes, size_t* solve_bytes);
int bds_tune(const bds_desc* desc, const double* Ad, const double* As, const double* B, double* X,
             void* factor_ws, size_t factor_bytes, void* solve_ws, size_t solve_bytes, bds_info* info,
             int reps, void* stream, bds_desc* best);

/*
 * Batched autotuner: the tile fields are chosen per padded block size np (all
 * systems of one np share them), by coordinate search over each group's
 * fields in turn, timing factor + solve of the whole batch.  nstar is kept.
 * Workspaces as given by bds_batched_workspace_size for descs (tile choices
 * do not change them).  best: host array of K descriptors.
 */
int bds_tune_batched(int64_t K, const bds_desc* descs, const double* const* Ad, const double* const* As,
                     const double* const* B, double* const* X, void* factor_ws, size_t factor_bytes,
                     void* solve_ws, size_t solve_bytes, bds_info* info, int reps, void* stream,
                     bds_desc* best);

/*
 * Kernel timing, for diagnostics and benchmarking; it does not change any
 * result.  bds_trace_enable(max_launches > 0) creates 2 * max_launches HIP
 * events on the current device and from then on brackets every kernel launch
 * of the library with two of them, recorded on the launch stream.  Launches
 * beyond the pool are not timed and are counted as dropped.
 * bds_trace_enable(0) stops timing and destroys the events.  Returns BDS_OK,
 * BDS_EINVAL (max_launches < 0 or > 2^20) or BDS_EHIP.
 */
int bds_trace_enable(int64_t max_launches);

/*
 * Waits for every timed launch, then reports per-kernel totals and clears the
 * record.  For up to max_kernels distinct kernel names k: names + 64 * k
 * receives the NUL-terminated name (host buffer of 64 * max_kernels chars),
 * launches[k] the number of timed launches and total_ms[k] their summed
 * event-to-event time in milliseconds (host arrays).  *n_kernels receives the
 * number of distinct names (which may exceed max_kernels) and *dropped, if
 * not NULL, the launches that were not timed.  Returns BDS_OK, BDS_EINVAL or
 * BDS_EHIP (an event could not be read; the other totals are still written).
 */
int bds_trace_read(int64_t max_kernels, char* names, int64_t* launches, double* total_ms, int64_t* n_kernels,
                   int64_t* dropped);

/* Library version string and the gfx target it was built for. */
const char* bds_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BDS_H */
