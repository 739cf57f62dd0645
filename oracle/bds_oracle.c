/*
 * Test infrastructure only: the CPU oracle of the block-tridiagonal SPD
 * solver.  It is written from the paper's definitions and shares no code,
 * header, table or helper with the GPU library.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.
 *
 * Build: gcc -O2 -fPIC -shared -fopenmp bds_oracle.c -o liboracle.so -lm
 *
 * Entry points (host arrays, row-major; shapes as described in oracle_impl.h):
 *
 *   oracle_factor      FP64 block Cholesky (Alg. 1, K = 1)        -> Ld, Ls
 *   oracle_solve       FP64 block substitution (Alg. 2, K = 1)    -> X
 *   oracle_matvec      Y = A X for the block-tridiagonal A of eq. (1)
 *   oracle_logdet      log det A = 2 sum log diag(Ld)
 *   oracle_backward    adjoint of X = A^{-1} B for the loss <W, X>  (the paper
 *                      is silent on differentiation; the formulas follow from
 *                      dX = -A^{-1} dA X, see below)
 *   oracle_solve_ld    factor + solve in long double, X rounded to double
 *   oracle_loss_ld     <W, A^{-1} B> in long double, returned as hi + lo
 *   oracle_solve_batched  FP64 factor + solve of K independent systems
 *                      (the batch notation of the paper's Sec. 3.2), OpenMP
 *                      across systems.
 *
 * Return codes: 0 on success; for factorisations, 1 + (block * n + column)
 * of the first pivot that is not positive, counted in natural block order;
 * -1 if a scratch allocation failed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REAL double
#define SUFFIX _d
#define SQRT sqrt
#include "oracle_impl.h"
#undef REAL
#undef SUFFIX
#undef SQRT

#define REAL long double
#define SUFFIX _ld
#define SQRT sqrtl
#include "oracle_impl.h"
#undef REAL
#undef SUFFIX
#undef SQRT

int64_t oracle_factor(int64_t N, int64_t n, const double* Ad, const double* As, double* Ld,
                      double* Ls)
{
    return factor_work_d(N, n, Ad, As, Ld, Ls);
}

void oracle_solve(int64_t N, int64_t n, int64_t d, const double* Ld, const double* Ls,
                  const double* B, double* X)
{
    solve_work_d(N, n, d, Ld, Ls, B, X);
}

/* Y = A X with A of eq. (1): Y_i = A_ii X_i + A_{i,i-1} X_{i-1} + A_{i+1,i}^T X_{i+1}. */
void oracle_matvec(int64_t N, int64_t n, int64_t d, const double* Ad, const double* As,
                   const double* X, double* Y)
{
    for (int64_t i = 0; i < N; ++i)
        for (int64_t r = 0; r < n; ++r)
            for (int64_t c = 0; c < d; ++c) {
                double t = 0;
                const double* a = Ad + i * n * n;
                for (int64_t k = 0; k < n; ++k) t += sym_at_d(a, n, r, k) * X[(i * n + k) * d + c];
                if (i > 0) {
                    const double* s = As + (i - 1) * n * n; /* A_{i,i-1} */
                    for (int64_t k = 0; k < n; ++k) t += s[r * n + k] * X[((i - 1) * n + k) * d + c];
                }
                if (i + 1 < N) {
                    const double* s = As + i * n * n; /* A_{i+1,i}, used transposed */
                    for (int64_t k = 0; k < n; ++k) t += s[k * n + r] * X[((i + 1) * n + k) * d + c];
                }
                Y[(i * n + r) * d + c] = t;
            }
}

double oracle_logdet(int64_t N, int64_t n, const double* Ld)
{
    double s = 0;
    for (int64_t i = 0; i < N; ++i)
        for (int64_t r = 0; r < n; ++r) s += log(Ld[(i * n + r) * n + r]);
    return 2.0 * s;
}

/*
 * Adjoint of X = A^{-1} B for the scalar loss l = sum(W .* X).
 *   G = A^{-1} W  (one more solve with the stored factor; A is symmetric)
 *   dB = G
 *   dl/dA (dense) = -G X^T; restricted to the parameters of A:
 *   dAd[i] = -(G_i X_i^T + X_i G_i^T) / 2       (symmetric diagonal block)
 *   dAs[i] = -(G_{i+1} X_i^T + X_{i+1} G_i^T)   (A_{i+1,i} enters at (i+1, i)
 *                                               and, transposed, at (i, i+1))
 * Ld, Ls: the factor from oracle_factor; X the solution; W = dl/dX.
 */
void oracle_backward(int64_t N, int64_t n, int64_t d, const double* Ld, const double* Ls,
                     const double* X, const double* W, double* dAd, double* dAs, double* dB)
{
    solve_work_d(N, n, d, Ld, Ls, W, dB);
    const double* G = dB;
    for (int64_t i = 0; i < N; ++i)
        for (int64_t r = 0; r < n; ++r)
            for (int64_t c = 0; c < n; ++c) {
                double t = 0;
                for (int64_t k = 0; k < d; ++k)
                    t += G[(i * n + r) * d + k] * X[(i * n + c) * d + k] +
                         X[(i * n + r) * d + k] * G[(i * n + c) * d + k];
                dAd[(i * n + r) * n + c] = -0.5 * t;
            }
    for (int64_t i = 0; i + 1 < N; ++i)
        for (int64_t r = 0; r < n; ++r)
            for (int64_t c = 0; c < n; ++c) {
                double t = 0;
                for (int64_t k = 0; k < d; ++k)
                    t += G[((i + 1) * n + r) * d + k] * X[(i * n + c) * d + k] +
                         X[((i + 1) * n + r) * d + k] * G[(i * n + c) * d + k];
                dAs[(i * n + r) * n + c] = -t;
            }
}

/* Factor and solve in long double; X is rounded to double at the end. */
int64_t oracle_solve_ld(int64_t N, int64_t n, int64_t d, const double* Ad, const double* As,
                        const double* B, double* X)
{
    size_t nn = (size_t)(n * n), nd = (size_t)(N * n * d);
    long double* Ld = (long double*)malloc(sizeof(long double) * nn * (size_t)N);
    long double* Ls = (long double*)malloc(sizeof(long double) * nn * (size_t)(N > 1 ? N - 1 : 1));
    long double* Y = (long double*)malloc(sizeof(long double) * nd);
    if (!Ld || !Ls || !Y) { free(Ld); free(Ls); free(Y); return -1; }
    int64_t info = factor_work_ld(N, n, Ad, As, Ld, Ls);
    if (info == 0) {
        for (size_t i = 0; i < nd; ++i) Y[i] = (long double)B[i];
        solve_work_ld(N, n, d, Ld, Ls, Y, Y);
        for (size_t i = 0; i < nd; ++i) X[i] = (double)Y[i];
    }
    free(Ld); free(Ls); free(Y);
    return info;
}

/* l = sum(W .* A^{-1} B) in long double; out[0] = (double)l, out[1] = (double)(l - out[0]). */
int64_t oracle_loss_ld(int64_t N, int64_t n, int64_t d, const double* Ad, const double* As,
                       const double* B, const double* W, double* out)
{
    size_t nn = (size_t)(n * n), nd = (size_t)(N * n * d);
    long double* Ld = (long double*)malloc(sizeof(long double) * nn * (size_t)N);
    long double* Ls = (long double*)malloc(sizeof(long double) * nn * (size_t)(N > 1 ? N - 1 : 1));
    long double* Y = (long double*)malloc(sizeof(long double) * nd);
    if (!Ld || !Ls || !Y) { free(Ld); free(Ls); free(Y); return -1; }
    int64_t info = factor_work_ld(N, n, Ad, As, Ld, Ls);
    if (info == 0) {
        for (size_t i = 0; i < nd; ++i) Y[i] = (long double)B[i];
        solve_work_ld(N, n, d, Ld, Ls, Y, Y);
        long double l = 0;
        for (size_t i = 0; i < nd; ++i) l += (long double)W[i] * Y[i];
        out[0] = (double)l;
        out[1] = (double)(l - (long double)out[0]);
    }
    free(Ld); free(Ls); free(Y);
    return info;
}

/*
 * K independent systems, system k with sizes (Ns[k], ns[k], ds[k]) at element
 * offsets offAd[k], offAs[k], offB[k] into the packed arrays.  X uses the same
 * offsets as B.  info[k] receives each system's factorisation code.  Threads:
 * OpenMP across systems (OMP_NUM_THREADS); returns the number of threads used.
 */
int oracle_solve_batched(int64_t K, const int64_t* Ns, const int64_t* ns, const int64_t* ds,
                         const int64_t* offAd, const int64_t* offAs, const int64_t* offB,
                         const double* Ad, const double* As, const double* B, double* X,
                         int64_t* info)
{
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            used = omp_get_num_threads();
#endif
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < K; ++k) {
            int64_t N = Ns[k], n = ns[k], d = ds[k];
            double* Ld = (double*)malloc(sizeof(double) * (size_t)(N * n * n));
            double* Ls = (double*)malloc(sizeof(double) * (size_t)((N > 1 ? N - 1 : 1) * n * n));
            if (!Ld || !Ls) { info[k] = -1; free(Ld); free(Ls); continue; }
            info[k] = factor_work_d(N, n, Ad + offAd[k], As + offAs[k], Ld, Ls);
            if (info[k] == 0) solve_work_d(N, n, d, Ld, Ls, B + offB[k], X + offB[k]);
            free(Ld); free(Ls);
        }
    }
    return used;
}
