/*
 * Test infrastructure only: the CPU oracle for the block-tridiagonal SPD solver.
 * Nothing in the product path may include, link or call this code; only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * This file is the body of the oracle, written once and instantiated twice by
 * bds_oracle.c: with REAL = double (suffix _d) and REAL = long double (suffix
 * _ld).  Every loop is plain; there is no blocking, no BLAS and no reordering
 * beyond what the definitions below state.
 *
 * What it computes.  The system of eq. (1) of the paper: A is symmetric
 * positive definite and block tridiagonal with N diagonal n x n blocks A_ii
 * and N-1 coupling blocks; X and B have N row blocks of n rows and d columns.
 * The oracle solves A X = B the plain way, by the sequential block-Cholesky
 * factorisation and block forward/backward substitution that the paper gives
 * as its serial base case (Alg. 1 and Alg. 2 with a single chain, K = 1,
 * which Alg. 4 and Alg. 7 call SerialFactorize and SerialSolve).
 *
 * Storage (all host arrays, row-major, C order):
 *   Ad  (N, n, n)   diagonal blocks A_ii; only the lower triangle is read and
 *                   the block is taken as its symmetric completion.
 *   As  (N-1, n, n) sub-diagonal blocks, As[i] = A_{i+1,i}; the block above
 *                   the diagonal is As[i]^T.  (The paper's text names the
 *                   coupling blocks A_{i,i+1} but its displayed matrix puts
 *                   A_{i+1,i} below the diagonal; this storage follows the
 *                   displayed matrix.)
 *   B, X (N, n, d)
 *   Ld  (N, n, n)   lower Cholesky factor of each pivot block (upper part 0).
 *   Ls  (N-1, n, n) Ls[i] = A_{i+1,i} Ld[i]^{-T}, the sub-diagonal blocks of
 *                   the block Cholesky factor.  Together Ld and Ls are exactly
 *                   the (banded) Cholesky factor of A.
 */

#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)
#define FN(name) CAT(name, SUFFIX)

/* Symmetric completion of a diagonal block: element (r, c) from the lower triangle. */
static REAL FN(sym_at)(const double* blk, int64_t n, int64_t r, int64_t c)
{
    return (REAL)(r >= c ? blk[r * n + c] : blk[c * n + r]);
}

/*
 * Dense Cholesky-Banachiewicz of the n x n symmetric matrix C (full storage,
 * symmetric), written into the lower triangle of Lo (upper set to zero).
 * Returns 0, or 1 + the first column whose pivot is not positive (or NaN).
 */
static int64_t FN(chol_dense)(const REAL* C, int64_t n, REAL* Lo)
{
    for (int64_t i = 0; i < n * n; ++i) Lo[i] = 0;
    for (int64_t j = 0; j < n; ++j) {
        REAL s = C[j * n + j];
        for (int64_t k = 0; k < j; ++k) s -= Lo[j * n + k] * Lo[j * n + k];
        if (!(s > 0)) return j + 1;
        REAL ljj = SQRT(s);
        Lo[j * n + j] = ljj;
        for (int64_t r = j + 1; r < n; ++r) {
            REAL t = C[r * n + j];
            for (int64_t k = 0; k < j; ++k) t -= Lo[r * n + k] * Lo[j * n + k];
            Lo[r * n + j] = t / ljj;
        }
    }
    return 0;
}

/*
 * Block Cholesky factorisation in natural order (Alg. 1 with K = 1):
 *   C_0 = A_00
 *   C_i = A_ii - Ls[i-1] Ls[i-1]^T                (rank-n update)
 *   Ld[i] = chol(C_i)                              (potrf)
 *   Ls[i] = A_{i+1,i} Ld[i]^{-T}                   (trsm, from the right)
 * Ld, Ls are REAL work arrays.  Returns 0, or 1 + the global row index
 * (i * n + column) of the first pivot that is not positive.
 */
static int64_t FN(factor_work)(int64_t N, int64_t n, const double* Ad, const double* As,
                               REAL* Ld, REAL* Ls)
{
    REAL* C = (REAL*)malloc(sizeof(REAL) * (size_t)(n * n));
    if (!C) return -1;
    for (int64_t i = 0; i < N; ++i) {
        const double* a = Ad + i * n * n;
        for (int64_t r = 0; r < n; ++r)
            for (int64_t c = 0; c < n; ++c) C[r * n + c] = FN(sym_at)(a, n, r, c);
        if (i > 0) {
            const REAL* P = Ls + (i - 1) * n * n;
            for (int64_t r = 0; r < n; ++r)
                for (int64_t c = 0; c < n; ++c) {
                    REAL t = 0;
                    for (int64_t k = 0; k < n; ++k) t += P[r * n + k] * P[c * n + k];
                    C[r * n + c] -= t;
                }
        }
        REAL* Li = Ld + i * n * n;
        int64_t bad = FN(chol_dense)(C, n, Li);
        if (bad) { free(C); return i * n + bad; }
        if (i + 1 < N) {
            /* Row r of Ls[i] solves Li x = (row r of A_{i+1,i})^T by forward substitution. */
            const double* s = As + i * n * n;
            REAL* P = Ls + i * n * n;
            for (int64_t r = 0; r < n; ++r)
                for (int64_t c = 0; c < n; ++c) {
                    REAL t = (REAL)s[r * n + c];
                    for (int64_t k = 0; k < c; ++k) t -= P[r * n + k] * Li[c * n + k];
                    P[r * n + c] = t / Li[c * n + c];
                }
        }
    }
    free(C);
    return 0;
}

/*
 * Block forward and backward substitution (Alg. 2 with K = 1):
 *   Y_0 = Ld[0]^{-1} B_0,  Y_i = Ld[i]^{-1} (B_i - Ls[i-1] Y_{i-1})
 *   X_{N-1} = Ld[N-1]^{-T} Y_{N-1},  X_i = Ld[i]^{-T} (Y_i - Ls[i]^T X_{i+1})
 * Y and X may alias (X is written in place over Y).
 */
static void FN(solve_work)(int64_t N, int64_t n, int64_t d, const REAL* Ld, const REAL* Ls,
                           const REAL* B, REAL* X)
{
    for (int64_t i = 0; i < N; ++i) {
        const REAL* Li = Ld + i * n * n;
        REAL* y = X + i * n * d;
        for (int64_t r = 0; r < n; ++r)
            for (int64_t c = 0; c < d; ++c) {
                REAL t = B[i * n * d + r * d + c];
                if (i > 0) {
                    const REAL* P = Ls + (i - 1) * n * n;
                    const REAL* yp = X + (i - 1) * n * d;
                    for (int64_t k = 0; k < n; ++k) t -= P[r * n + k] * yp[k * d + c];
                }
                for (int64_t k = 0; k < r; ++k) t -= Li[r * n + k] * y[k * d + c];
                y[r * d + c] = t / Li[r * n + r];
            }
    }
    for (int64_t i = N - 1; i >= 0; --i) {
        const REAL* Li = Ld + i * n * n;
        REAL* x = X + i * n * d;
        for (int64_t r = n - 1; r >= 0; --r)
            for (int64_t c = 0; c < d; ++c) {
                REAL t = x[r * d + c];
                if (i + 1 < N) {
                    const REAL* P = Ls + i * n * n;
                    const REAL* xn = X + (i + 1) * n * d;
                    for (int64_t k = 0; k < n; ++k) t -= P[k * n + r] * xn[k * d + c];
                }
                for (int64_t k = r + 1; k < n; ++k) t -= Li[k * n + r] * x[k * d + c];
                x[r * d + c] = t / Li[r * n + r];
            }
    }
}
