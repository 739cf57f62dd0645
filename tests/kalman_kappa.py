"""Condition number of the Kalman-smoother Hessian from ``inputs.gen_kalman``.

Used to calibrate ``inputs.KALMAN_RHO`` (rho = q/r for kappa targets 1e2, 1e4,
1e6 on the high-rho branch).  lambda_max comes from Lanczos on A, lambda_min
from Lanczos on A^-1 applied with the CPU oracle's factorisation.

Run as a script:  python tests/kalman_kappa.py N n rho [rho ...]
"""
import os
import sys

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from paper_2509_03015_amd import inputs  # noqa: E402


def sparse_matrix(Ad, As):
    N, n, _ = Ad.shape
    rows, cols, vals = [], [], []
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for i in range(N):
        rows.append(i * n + ii.ravel()); cols.append(i * n + jj.ravel()); vals.append(Ad[i].ravel())
    for i in range(N - 1):
        rows.append((i + 1) * n + ii.ravel()); cols.append(i * n + jj.ravel()); vals.append(As[i].ravel())
        rows.append(i * n + jj.ravel()); cols.append((i + 1) * n + ii.ravel()); vals.append(As[i].ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N * n, N * n))


def kappa(Ad, As):
    N, n, _ = Ad.shape
    A = sparse_matrix(Ad, As)
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0]
    Ld, Ls = oracle.factor(Ad, As)
    inv = spla.LinearOperator((N * n, N * n), dtype=np.float64,
                              matvec=lambda v: oracle.solve_factored(Ld, Ls, v.reshape(N, n, 1)).ravel())
    mu = spla.eigsh(inv, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0]
    return float(lmax * mu), float(lmax), float(1.0 / mu)


if __name__ == "__main__":
    N, n = int(sys.argv[1]), int(sys.argv[2])
    for rho in map(float, sys.argv[3:]):
        Ad, As, _, _ = inputs.gen_kalman(N, n, 1, rho, seed=0)
        k, lmax, lmin = kappa(Ad, As)
        print(f"N={N} n={n} rho={rho:g}: kappa={k:.3e} lmax={lmax:.3e} lmin={lmin:.3e}", flush=True)
