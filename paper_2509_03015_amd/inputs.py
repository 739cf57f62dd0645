"""Seeded synthetic inputs for the block-tridiagonal SPD solver.

This module only draws and assembles inputs; it holds none of the solver's
arithmetic (no factorisation, no substitution, no refinement).  The same bits
are handed to the GPU library and to the CPU oracle.

Layout of every system (float64, C order):

* ``Ad`` (N, n, n): diagonal blocks ``A[i, i]``, symmetric;
* ``As`` (N-1, n, n): sub-diagonal blocks, ``As[i] = A[i+1, i]`` (the block
  above the diagonal is its transpose, as in eq. (1) of the paper);
* ``X_true`` and ``B = A @ X_true`` (N, n, d): a manufactured solution and the
  right-hand side built from it.

Generators
----------
``gen_dd``      block diagonally dominant systems: ``As[i] ~ N(0,1)/sqrt(n)``,
                ``Ad[i] = G G^T / n + 5 I`` with ``G ~ N(0,1)``.  The paper's
                synthetic sweep uses "randomly generated, well-conditioned" SPD
                block-tridiagonal matrices (Sec. 4.1) without naming the
                generator; this one has kappa(A) of about 4.
``gen_kalman``  the MAP normal equations of a linear-Gaussian smoother
                (Sec. 4.2): ``A[k,k] = Q^-1 + F^T Q^-1 F + H_k^T R^-1 H_k`` with
                the ``F^T Q^-1 F`` term absent in the last block (the paper's
                convention G_{N+1} = 0), ``A[k+1,k] = -Q^-1 F``.  Here
                ``F = 0.99 U`` with U Haar-orthogonal, ``Q = I``, ``R = I/rho``,
                ``H_k ~ N(0,1)`` with m = n/2 rows, drawn per step.  ``rho``
                sets the conditioning.
``gen_batched`` K independent systems of uneven size, each from ``gen_dd``.
``gen_kalman_neuro``  the smoothing problem of the paper's neuroscience example
                (Sec. 4.2): a latent state of dimension n driven by damped
                two-dimensional rotations, observed through a tall
                well-conditioned H (m rows) with diagonal measurement noise R
                larger than the dense SPD process noise Q, over N steps; the
                right-hand side is the measurement one, ``b = H^T R^-1 z +
                G^T Q^-1 zeta`` (not manufactured), so the exact X is the MAP
                trajectory, which a Rauch-Tung-Striebel smoother also gives.
"""
from __future__ import annotations

import numpy as np


def block_matvec(Ad: np.ndarray, As: np.ndarray, X: np.ndarray) -> np.ndarray:
    """``A @ X`` for the block-tridiagonal A; used to manufacture ``B`` from ``X_true``.

    Only the lower triangle of each diagonal block is used (its symmetric
    completion), matching how the solvers read ``Ad``.
    """
    N, n, _ = Ad.shape
    low = np.tril(Ad)
    sym = low + np.transpose(np.tril(Ad, -1), (0, 2, 1))
    Y = np.matmul(sym, X)
    if N > 1:
        Y[1:] += np.matmul(As, X[:-1])
        Y[:-1] += np.matmul(np.transpose(As, (0, 2, 1)), X[1:])
    return Y


def gen_dd(N: int, n: int, d: int, seed: int = 0):
    """Block diagonally dominant SPD system.  Draw order: As, G, X_true."""
    rng = np.random.default_rng(seed)
    As = rng.standard_normal((max(N - 1, 0), n, n)) / np.sqrt(n)
    G = rng.standard_normal((N, n, n))
    Ad = np.matmul(G, np.transpose(G, (0, 2, 1))) / n
    del G
    Ad = 0.5 * (Ad + np.transpose(Ad, (0, 2, 1)))
    Ad += 5.0 * np.eye(n)
    X = rng.standard_normal((N, n, d))
    B = block_matvec(Ad, As, X)
    return Ad, As, X, B


def haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian with the sign of diag(R) fixed."""
    Z = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    return Q * np.sign(np.diag(R))[None, :]


# rho = q/r giving kappa(A) near the target on the high-rho branch (kappa grows
# about linearly in rho there; at rho -> 0 the dynamics alone give kappa ~ 4e4,
# with a minimum near 70 in between).  Measured with the Lanczos estimate in
# tests/kalman_kappa.py at (N, n) = (1024, 32) and (128, 256), seed 0:
#   n=32:  rho 0.085 -> 99.3,   14.7 -> 1.001e4,  1470 -> 9.96e5
#   n=256: rho 0.0135 -> 100.4, 2.32 -> 1.003e4,  232 -> 9.98e5
# lambda_min settles near 0.18 and lambda_max grows like rho, so kappa depends
# only weakly on N once N >> 1.
KALMAN_RHO = {
    32: {1e2: 0.085, 1e4: 14.7, 1e6: 1470.0},
    256: {1e2: 0.0135, 1e4: 2.32, 1e6: 232.0},
}


def gen_kalman(N: int, n: int, d: int, rho: float, seed: int = 0, m: int | None = None):
    """Kalman-smoother Hessian (normal equations) with q = 1, r = 1/rho.  Draw order: U, H, X_true."""
    rng = np.random.default_rng(seed)
    m = n // 2 if m is None else m
    F = 0.99 * haar_orthogonal(rng, n)
    H = rng.standard_normal((N, m, n))
    Ad = rho * np.matmul(np.transpose(H, (0, 2, 1)), H)
    del H
    Ad += np.eye(n)
    if N > 1:
        Ad[:-1] += F.T @ F
    Ad = 0.5 * (Ad + np.transpose(Ad, (0, 2, 1)))
    As = np.broadcast_to(-F, (max(N - 1, 0), n, n)).copy()
    X = rng.standard_normal((N, n, d))
    B = block_matvec(Ad, As, X)
    return Ad, As, X, B


def batched_sizes(K: int = 512, seed: int = 0, n_choices=(8, 16, 32, 64), d_choices=(1, 4),
                  N_range=(32, 2048)):
    """Per-system (N, n, d): N ~ U{N_range}, n and d uniform over the choices."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(N_range[0], N_range[1] + 1, size=K)
    ns = rng.choice(np.asarray(n_choices), size=K)
    ds = rng.choice(np.asarray(d_choices), size=K)
    return [(int(a), int(b), int(c)) for a, b, c in zip(Ns, ns, ds)]


def gen_batched(K: int = 512, seed: int = 0, **size_kw):
    """K uneven systems; system k is ``gen_dd(N_k, n_k, d_k, seed=seed * 100003 + k + 1)``."""
    out = []
    for k, (N, n, d) in enumerate(batched_sizes(K, seed, **size_kw)):
        out.append(gen_dd(N, n, d, seed=seed * 100003 + k + 1))
    return out


def kalman_neuro_model(N: int = 100, n: int = 256, m: int = 1024, seed: int = 0, dt: float = 0.1):
    """Model and simulated data of the neuroscience-style smoothing example.

    The paper fixes n, m, N and dt and describes the matrices only in words; the
    parameters below are this generator's reading:

    * ``G = U diag(lam_i R(theta_i)) U^T``: n/2 damped 2 x 2 rotations in a
      Haar-random basis, decay ``lam_i = exp(-dt / tau_i)`` with tau_i ~ U(0.5, 2) s
      and ``theta_i = 2 pi f_i dt`` with f_i ~ U(0.5, 2) Hz (slow rotational
      dynamics); ``G_1 = I`` (the known initial state enters through zeta);
    * ``Q = q (0.5 I + V V^T / n)`` with V ~ N(0, 1) (dense SPD), q = 0.01;
    * ``R = diag(r_j)`` with r_j = 10 q U(0.5, 1.5) (measurements less reliable
      than the dynamics);
    * ``H ~ N(0, 1) / sqrt(m)`` (m x n, condition number about
      (1 + sqrt(n/m)) / (1 - sqrt(n/m)) = 3 for m = 4n);
    * x_0 ~ N(0, I) known; x_k = G_k x_{k-1} + w_k, z_k = H x_k + v_k with
      w_k ~ N(0, Q), v_k ~ N(0, R).

    Returns a dict with G, Q, r (the diagonal of R), H, x0, the simulated states
    x (N, n) and measurements z (N, m).  Draw order: U, tau, f, V, r, H, x0, w, v.
    """
    if n % 2:
        raise ValueError("n must be even (pairs of rotating coordinates)")
    rng = np.random.default_rng(seed)
    U = haar_orthogonal(rng, n)
    tau = rng.uniform(0.5, 2.0, n // 2)
    f = rng.uniform(0.5, 2.0, n // 2)
    lam = np.exp(-dt / tau)
    th = 2.0 * np.pi * f * dt
    D = np.zeros((n, n))
    for i in range(n // 2):
        c, s_ = np.cos(th[i]), np.sin(th[i])
        D[2 * i:2 * i + 2, 2 * i:2 * i + 2] = lam[i] * np.array([[c, -s_], [s_, c]])
    G = U @ D @ U.T
    q = 0.01
    V = rng.standard_normal((n, n))
    Q = q * (0.5 * np.eye(n) + V @ V.T / n)
    Q = 0.5 * (Q + Q.T)
    r = 10.0 * q * rng.uniform(0.5, 1.5, m)
    H = rng.standard_normal((m, n)) / np.sqrt(m)
    x0 = rng.standard_normal(n)
    Lq = np.linalg.cholesky(Q)
    w = rng.standard_normal((N, n)) @ Lq.T
    v = rng.standard_normal((N, m)) * np.sqrt(r)[None, :]
    x = np.empty((N, n))
    prev = x0
    for k in range(N):
        prev = (prev if k == 0 else G @ prev) + w[k]
        x[k] = prev
    z = x @ H.T + v
    return {"G": G, "Q": Q, "r": r, "H": H, "x0": x0, "x": x, "z": z}


def gen_kalman_neuro(N: int = 100, n: int = 256, m: int = 1024, seed: int = 0):
    """The MAP normal equations of ``kalman_neuro_model`` as a block-tridiagonal system.

    Blocks as the paper writes them (Sec. 4.2), with G_1 = I, G_{N+1} = 0 and
    time-invariant G, Q, H, R otherwise:
    ``A[k,k] = Q^-1 + G^T Q^-1 G (k < N) + H^T R^-1 H``, ``A[k+1,k] = -Q^-1 G``;
    ``b_k = H^T R^-1 z_k``, plus ``Q^-1 x_0`` in the first block (the term
    ``G^T Q^-1 zeta`` with zeta = (G_1 x_0, 0, ..., 0)).  Returns
    ``(Ad, As, x, B, model)``: x is the simulated trajectory (not the solution),
    B has shape (N, n, 1).
    """
    mdl = kalman_neuro_model(N, n, m, seed)
    G, Q, r, H = mdl["G"], mdl["Q"], mdl["r"], mdl["H"]
    Qi = np.linalg.inv(Q)
    Qi = 0.5 * (Qi + Qi.T)
    HtRiH = H.T @ (H / r[:, None])
    Ad = np.broadcast_to(Qi + HtRiH, (N, n, n)).copy()
    if N > 1:
        Ad[:-1] += G.T @ Qi @ G
    Ad = 0.5 * (Ad + np.transpose(Ad, (0, 2, 1)))
    As = np.broadcast_to(-Qi @ G, (max(N - 1, 0), n, n)).copy()
    B = ((mdl["z"] / r[None, :]) @ H)[:, :, None].copy()
    B[0, :, 0] += Qi @ mdl["x0"]
    return Ad, As, mdl["x"][:, :, None].copy(), B, mdl

