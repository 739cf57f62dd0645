// Level plan and workspace layout of the recursive Schur-complement solver.
//
// Odd-even reduction (segment length 1 in the paper's partition of Sec. 3.1):
// a level with M blocks eliminates the E = floor(M/2) blocks at odd positions
// (the interiors) and keeps the ceil(M/2) blocks at even positions (the
// separators), which form the next level's block-tridiagonal Schur complement
// (eq. (5)).  Reduction stops once a level has at most nstar blocks (the
// paper's crossover N_star, Alg. 4); that coarse system is factorised by
// sequential block Cholesky in FP64.  A block at position p of level l is
// block p * 2^l of the original system.
//
// Every n x n block is stored padded to np = round_up(n, 16) (row-major,
// leading dimension np).  The padding of a diagonal block is the identity and
// that of a coupling block is zero, so the padded system is the original one
// plus decoupled identity rows: every derived quantity keeps zero/identity
// padding and the kernels work on whole 16 x 16 tiles.  When n is not a
// multiple of 16 the user's arrays are first copied into padded buffers.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/bds.h"
#include "bds_kernels.hpp"

namespace bds {

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxN = 256;
constexpr int kDefaultNstar = 1;
constexpr int kDefaultMaxRefine = 30;
constexpr double kDefaultRefineTol = 1e-14;

// Bytes per stored factor element: FP64, or FP32 for both low-precision modes (BF16 rounds
// MFMA operands, it does not change the storage).
inline size_t matrix_elem_bytes(int prec) { return prec == BDS_F64 ? 8 : 4; }

struct LevelPlan {
    int64_t M = 0;   // blocks entering the level
    int64_t E = 0;   // interiors eliminated here: M / 2
    int64_t Mn = 0;  // blocks of the next level: (M + 1) / 2
    // factor workspace byte offsets; matrix precision, np x np blocks
    size_t Li = 0;   // E blocks: inverse of the Cholesky factor of each interior
    size_t Wt = 0;   // E blocks: A[i-1, i] * Li^T (left coupling, solved and stored transposed)
    size_t Pr = 0;   // E blocks: A[i+1, i] * Li^T (right coupling, solved, transposed)
    size_t Adn = 0;  // Mn blocks: next level diagonal blocks (Schur complement)
    size_t Asn = 0;  // Mn - 1 blocks: next level sub-diagonal blocks
    // solve workspace byte offsets; FP64, np x d blocks
    size_t Y = 0;    // E blocks: Li * B_i of the interiors
    size_t Bn = 0;   // Mn blocks: next level right-hand side
    size_t Xn = 0;   // Mn blocks: next level solution
};

struct SysPlan {
    int64_t N = 0, n = 0, np = 0, d = 0;
    int prec = BDS_F64;
    int nstar = kDefaultNstar;
    int max_refine = kDefaultMaxRefine;
    double refine_tol = kDefaultRefineTol;
    size_t esize = 8;
    Tiling tl;            // tile shapes of the reduction levels
    int32_t tiles_req = 0;  // the caller's tile field (0 in a field: left to the library)
    bool packed = false;  // n % 16 != 0: user arrays are copied into padded buffers
    std::vector<LevelPlan> lv;
    int64_t Mc = 0;       // blocks of the coarse system
    // factor workspace
    size_t Ad0 = 0, As0 = 0;  // padded FP64 copies of Ad, As (packed only)
    size_t Lc = 0;        // Mc blocks FP64: inverse Cholesky factors of the coarse pivots
    size_t Lsc = 0;       // Mc - 1 blocks FP64: A[i+1,i] Lc[i]^T of the coarse chain
    size_t Cw = 0;        // 1 block FP64: coarse pivot scratch
    size_t factor_bytes = 0;
    // solve workspace (FP64, np x d blocks)
    size_t B0 = 0, X0 = 0;    // padded copies of B and X (packed only)
    size_t G = 0;         // N blocks: adjoint solve A^-1 dX
    size_t Yc = 0;        // Mc blocks: coarse forward result
    size_t R = 0;         // N blocks: refinement residual
    size_t Cr = 0;        // N blocks: refinement correction
    size_t Nrm = 0;       // norm partial sums
    size_t solve_bytes = 0;
};

// Validates a descriptor; returns BDS_OK or BDS_EINVAL.
int check_desc(const bds_desc* d);

// Plan of one system; offsets are relative to the start of its factor and
// solve workspaces, starting at base_f / base_s.
SysPlan make_plan(const bds_desc& d, size_t base_f = 0, size_t base_s = 0);

// Number of norm partial slots used by the refinement of one system.
inline int64_t norm_slots(const SysPlan& p) { return p.N; }

}  // namespace bds
