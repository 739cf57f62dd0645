"""The neuroscience-style smoothing workload (paper Sec. 4.2): generator and oracle pins.

The system's exact solution is the MAP trajectory of a linear-Gaussian model.
A Rauch-Tung-Striebel smoother (Kalman filter forward, then the RTS backward
recursion; Rauch, Tung and Striebel 1965) computes the same means from the
model itself, without forming A: agreement pins both the generator's assembly
of A and b and the oracle's solve.  A dropped term in either (the
G^T Q^-1 G block, the x_0 term of b, a sign of the coupling) moves the
solution far beyond the tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_2509_03015_amd import inputs
from tests.dense import dense, flat


def rts_smoother(mdl, N):
    """Smoothed means E[x_k | z_1..z_N] of the model (x_0 known, G_1 = I)."""
    G, Q, r, H, x0, z = mdl["G"], mdl["Q"], mdl["r"], mdl["H"], mdl["x0"], mdl["z"]
    n = x0.shape[0]
    I = np.eye(n)
    R = np.diag(r)
    xp, Pp, xf, Pf = [], [], [], []
    x, P = x0, np.zeros((n, n))
    for k in range(N):
        Gk = I if k == 0 else G
        x_pred = Gk @ x
        P_pred = Gk @ P @ Gk.T + Q
        S = H @ P_pred @ H.T + R
        K = np.linalg.solve(S, H @ P_pred).T       # P_pred H^T S^-1 (S, P_pred symmetric)
        x = x_pred + K @ (z[k] - H @ x_pred)
        P = (I - K @ H) @ P_pred
        P = 0.5 * (P + P.T)
        xp.append(x_pred), Pp.append(P_pred), xf.append(x), Pf.append(P)
    xs = [None] * N
    xs[N - 1] = xf[N - 1]
    for k in range(N - 2, -1, -1):
        C = np.linalg.solve(Pp[k + 1], G @ Pf[k]).T   # Pf G^T Pp^-1
        xs[k] = xf[k] + C @ (xs[k + 1] - xp[k + 1])
    return np.stack(xs)


@pytest.mark.parametrize("N,n,m", [(1, 8, 32), (2, 8, 32), (30, 16, 64), (12, 32, 128)])
def test_oracle_solution_is_the_rts_smoother(N, n, m):
    Ad, As, x, B, mdl = inputs.gen_kalman_neuro(N, n, m, seed=N + n)
    X = oracle.solve(Ad, As, B)[:, :, 0]
    Xs = rts_smoother(mdl, N)
    assert np.linalg.norm(X - Xs) <= 1e-10 * np.linalg.norm(Xs)


def test_generator_structure():
    N, n, m = 5, 8, 32
    Ad, As, x, B, mdl = inputs.gen_kalman_neuro(N, n, m, seed=2)
    G, Q, r, H = mdl["G"], mdl["Q"], mdl["r"], mdl["H"]
    # damped rotations: eigenvalues in conjugate pairs with modulus exp(-dt / tau) in [exp(-0.2), exp(-0.05)]
    mod = np.abs(np.linalg.eigvals(G))
    assert mod.min() >= np.exp(-0.2) - 1e-12 and mod.max() <= np.exp(-0.05) + 1e-12
    assert np.all(np.linalg.eigvalsh(Q) > 0) and np.count_nonzero(Q) == n * n
    assert r.min() > 10 * 0.01 * 0.5 - 1e-15 and r.max() < 10 * 0.01 * 1.5
    sv = np.linalg.svd(H, compute_uv=False)
    assert H.shape == (m, n) and sv.max() / sv.min() < 10
    # A is SPD, blocks as in the paper; the last block lacks G^T Q^-1 G
    A = dense(Ad, As)
    np.testing.assert_allclose(A, A.T, atol=1e-12)
    assert np.linalg.eigvalsh(A).min() > 0
    Qi = np.linalg.inv(Q)
    np.testing.assert_allclose(Ad[-2] - Ad[-1], G.T @ Qi @ G, rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(As[0], -Qi @ G, rtol=1e-10, atol=1e-9)
    # seeded: the same seed gives the same bits
    again = inputs.gen_kalman_neuro(N, n, m, seed=2)
    for a, b in zip((Ad, As, x, B), again[:4]):
        np.testing.assert_array_equal(a, b)


def test_full_size_residual_at_the_papers_level():
    """At the paper's size (N=100, n=256, m=1024) the FP64 oracle's residual is of the order the paper reports."""
    Ad, As, x, B, _ = inputs.gen_kalman_neuro()
    X = oracle.solve(Ad, As, B)
    res = np.linalg.norm(flat(oracle.matvec(Ad, As, X) - B))
    assert res <= 1e-9 * np.linalg.norm(flat(B))
