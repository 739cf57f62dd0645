"""Test infrastructure only: the CPU oracle of the block-tridiagonal SPD solver.

This package is a plain, slow, obviously correct reference.  It exists so that
the tests, the smoke check and the benchmark's CPU-baseline leg can check the
GPU library against the paper's definitions.  The product path never imports
it, and it imports nothing from the product package.

The arithmetic lives in ``bds_oracle.c`` / ``oracle_impl.h`` (plain C loops,
FP64 and long double):

* ``factor``   -- sequential block Cholesky (the paper's Alg. 1 with K = 1,
  the SerialFactorize base case of Alg. 4);
* ``solve``    -- block forward/backward substitution (Alg. 2 with K = 1, the
  SerialSolve base case of Alg. 7);
* ``matvec``   -- ``A @ X`` for the block-tridiagonal ``A`` of eq. (1);
* ``logdet``   -- ``2 * sum(log(diag(L)))``;
* ``backward`` -- adjoint of ``X = A^{-1} B`` for the loss ``sum(W * X)``
  (differentiation is not in the paper; the formulas follow from
  ``dX = -A^{-1} dA X``);
* ``solve_ld`` / ``loss_ld`` -- the same in long double (80-bit x87), used as
  the reference where FP64 rounding (about 1.6e-17 * kappa) is too coarse;
* ``solve_batched`` -- K independent systems, OpenMP over systems.

Layout: ``Ad`` (N, n, n) with only the lower triangle read, ``As`` (N-1, n, n)
with ``As[i] = A[i+1, i]`` (the block below the diagonal in the paper's
displayed matrix), ``B`` and ``X`` (N, n, d); all float64, C order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = [os.path.join(_HERE, "bds_oracle.c"), os.path.join(_HERE, "oracle_impl.h")]
_lib = None


class OracleError(RuntimeError):
    """The oracle's factorisation met a pivot that is not positive."""

    def __init__(self, code: int, n: int):
        self.code = int(code)
        self.block = (self.code - 1) // n
        self.column = (self.code - 1) % n
        super().__init__(f"not SPD: pivot of block {self.block}, column {self.column}")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, -O2, OpenMP)."""
    stale = not os.path.exists(_LIB_PATH) or any(
        os.path.getmtime(s) > os.path.getmtime(_LIB_PATH) for s in _SOURCES)
    if force or stale:
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", _SOURCES[0],
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int64
    lib.oracle_factor.argtypes = [I, I, P, P, P, P]
    lib.oracle_factor.restype = I
    lib.oracle_solve.argtypes = [I, I, I, P, P, P, P]
    lib.oracle_solve.restype = None
    lib.oracle_matvec.argtypes = [I, I, I, P, P, P, P]
    lib.oracle_matvec.restype = None
    lib.oracle_logdet.argtypes = [I, I, P]
    lib.oracle_logdet.restype = ctypes.c_double
    lib.oracle_backward.argtypes = [I, I, I, P, P, P, P, P, P, P]
    lib.oracle_backward.restype = None
    lib.oracle_solve_ld.argtypes = [I, I, I, P, P, P, P]
    lib.oracle_solve_ld.restype = I
    lib.oracle_loss_ld.argtypes = [I, I, I, P, P, P, P, P]
    lib.oracle_loss_ld.restype = I
    lib.oracle_solve_batched.argtypes = [I, P, P, P, P, P, P, P, P, P, P, P]
    lib.oracle_solve_batched.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _shapes(Ad, As):
    Ad = _f64(Ad)
    N, n, n2 = Ad.shape
    assert n == n2, "diagonal blocks must be square"
    As = _f64(As) if N > 1 else np.zeros((1, n, n))
    if N > 1:
        assert As.shape == (N - 1, n, n), "expected As of shape (N-1, n, n)"
    return Ad, As, N, n


def factor(Ad, As):
    """Block Cholesky factor (Ld, Ls); raises OracleError if A is not SPD."""
    Ad, As, N, n = _shapes(Ad, As)
    Ld = np.zeros((N, n, n))
    Ls = np.zeros((max(N - 1, 1), n, n))
    code = _load().oracle_factor(N, n, _p(Ad), _p(As), _p(Ld), _p(Ls))
    if code != 0:
        raise OracleError(code, n)
    return Ld, Ls[: N - 1]


def solve_factored(Ld, Ls, B):
    Ld = _f64(Ld)
    N, n, _ = Ld.shape
    Ls = _f64(Ls) if N > 1 else np.zeros((1, n, n))
    B = _f64(B)
    assert B.shape[:2] == (N, n)
    d = B.shape[2]
    X = np.empty_like(B)
    _load().oracle_solve(N, n, d, _p(Ld), _p(Ls), _p(B), _p(X))
    return X


def solve(Ad, As, B):
    """X = A^{-1} B in FP64 (block Cholesky, natural order)."""
    Ld, Ls = factor(Ad, As)
    return solve_factored(Ld, Ls, B)


def matvec(Ad, As, X):
    Ad, As, N, n = _shapes(Ad, As)
    X = _f64(X)
    d = X.shape[2]
    Y = np.empty_like(X)
    _load().oracle_matvec(N, n, d, _p(Ad), _p(As), _p(X), _p(Y))
    return Y


def logdet(Ld) -> float:
    Ld = _f64(Ld)
    N, n, _ = Ld.shape
    return float(_load().oracle_logdet(N, n, _p(Ld)))


def backward(Ad, As, X, W):
    """Gradients (dAd, dAs, dB) of sum(W * X) with X = A^{-1} B."""
    Ld, Ls = factor(Ad, As)
    N, n, _ = Ld.shape
    X = _f64(X)
    W = _f64(W)
    d = X.shape[2]
    Lsp = Ls if N > 1 else np.zeros((1, n, n))
    dAd = np.empty((N, n, n))
    dAs = np.zeros((max(N - 1, 1), n, n))
    dB = np.empty_like(X)
    _load().oracle_backward(N, n, d, _p(Ld), _p(_f64(Lsp)), _p(X), _p(W), _p(dAd), _p(dAs), _p(dB))
    return dAd, dAs[: N - 1], dB


def solve_ld(Ad, As, B):
    """X = A^{-1} B computed in long double, rounded to FP64."""
    Ad, As, N, n = _shapes(Ad, As)
    B = _f64(B)
    X = np.empty_like(B)
    code = _load().oracle_solve_ld(N, n, B.shape[2], _p(Ad), _p(As), _p(B), _p(X))
    if code != 0:
        raise OracleError(code, n)
    return X


def loss_ld(Ad, As, B, W):
    """sum(W * A^{-1} B) in long double, returned as a (hi, lo) pair of floats."""
    Ad, As, N, n = _shapes(Ad, As)
    B = _f64(B)
    W = _f64(W)
    out = np.zeros(2)
    code = _load().oracle_loss_ld(N, n, B.shape[2], _p(Ad), _p(As), _p(B), _p(W), _p(out))
    if code != 0:
        raise OracleError(code, n)
    return float(out[0]), float(out[1])


def solve_batched(systems):
    """Solve a list of (Ad, As, B) systems; returns (list of X, threads used)."""
    K = len(systems)
    Ns = np.array([s[0].shape[0] for s in systems], dtype=np.int64)
    ns = np.array([s[0].shape[1] for s in systems], dtype=np.int64)
    ds = np.array([s[2].shape[2] for s in systems], dtype=np.int64)
    sAd = Ns * ns * ns
    sAs = np.maximum(Ns - 1, 0) * ns * ns
    sB = Ns * ns * ds
    offAd = np.concatenate([[0], np.cumsum(sAd)[:-1]]).astype(np.int64)
    offAs = np.concatenate([[0], np.cumsum(sAs)[:-1]]).astype(np.int64)
    offB = np.concatenate([[0], np.cumsum(sB)[:-1]]).astype(np.int64)
    Ad = np.concatenate([_f64(s[0]).ravel() for s in systems])
    As = np.concatenate([_f64(s[1]).ravel() for s in systems] + [np.zeros(1)])
    B = np.concatenate([_f64(s[2]).ravel() for s in systems])
    X = np.empty_like(B)
    info = np.zeros(K, dtype=np.int64)
    used = _load().oracle_solve_batched(K, _p(Ns), _p(ns), _p(ds), _p(offAd), _p(offAs), _p(offB),
                                        _p(Ad), _p(As), _p(B), _p(X), _p(info))
    for k in range(K):
        if info[k] != 0:
            raise OracleError(int(info[k]), int(ns[k]))
    Xs = [X[offB[k]: offB[k] + sB[k]].reshape(Ns[k], ns[k], ds[k]) for k in range(K)]
    return Xs, int(used)
