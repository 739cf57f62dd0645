"""Dense helpers for the tests: assemble the full matrix of eq. (1) from its blocks.

Independent of both the oracle and the GPU library (plain NumPy indexing).
"""
import numpy as np


def sym_lower(Ad):
    """Symmetric completion of each diagonal block from its lower triangle."""
    return np.tril(Ad) + np.transpose(np.tril(Ad, -1), (0, 2, 1))


def dense(Ad, As):
    N, n, _ = Ad.shape
    A = np.zeros((N * n, N * n))
    S = sym_lower(Ad)
    for i in range(N):
        A[i * n:(i + 1) * n, i * n:(i + 1) * n] = S[i]
    for i in range(N - 1):
        A[(i + 1) * n:(i + 2) * n, i * n:(i + 1) * n] = As[i]
        A[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] = As[i].T
    return A


def flat(X):
    N, n, d = X.shape
    return X.reshape(N * n, d)


def blocks(x, N, n):
    return x.reshape(N, n, -1)


def relerr(X, Y):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    den = np.linalg.norm(Y.ravel())
    return float(np.linalg.norm((X - Y).ravel()) / (den if den > 0 else 1.0))
