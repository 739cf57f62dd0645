"""GPU parity of the adjoint (bds_backward and the autograd wrapper).

The loss is L = sum(W * X) with X = A^{-1} B.  Checks: the GPU gradients against the oracle's adjoint
(element-wise), against central finite differences of the long-double oracle's loss on random
entries, and the dot-product identity <W, -A^{-1}(E X)> = <dL/dA, E> for a random symmetric
block-tridiagonal direction E.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_2509_03015_amd import inputs
from tests.dense import relerr

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


@pytest.fixture(scope="module")
def S():
    from paper_2509_03015_amd import solver
    solver.bb.load()
    return solver


def gpu_grads(S, Ad, As, B, W, prec="f64"):
    F = S.factor(dev(Ad), dev(As) if Ad.shape[0] > 1 else None, prec=prec)
    X = F.solve(dev(B))
    dAd, dAs, dB = F.backward(X, dev(W))
    torch.cuda.synchronize()
    return X.cpu().numpy(), dAd.cpu().numpy(), dAs.cpu().numpy(), dB.cpu().numpy()


@pytest.mark.parametrize("N,n,d", [(1, 8, 2), (2, 16, 1), (9, 17, 3), (64, 32, 4), (33, 128, 2)])
def test_backward_matches_oracle_adjoint(S, N, n, d):
    _say("adjoint vs oracle", N, n, d)
    Ad, As, _, B = inputs.gen_dd(N, n, d, seed=40 + N)
    W = np.random.default_rng(N).standard_normal((N, n, d))
    X, dAd, dAs, dB = gpu_grads(S, Ad, As, B, W)
    rX = oracle.solve(Ad, As, B)
    rAd, rAs, rB = oracle.backward(Ad, As, rX, W)
    assert relerr(dB, rB) <= 1e-12
    assert relerr(dAd, rAd) <= 1e-12
    if N > 1:
        assert relerr(dAs, rAs) <= 1e-12


def test_adjoint_N4096_n32_d4_against_oracle_and_fd(S):
    """N=4096, n=32, d=4, Kalman Hessian at kappa ~ 1e4: 64 random entries by central differences."""
    _say("adjoint N=4096 n=32 d=4")
    N, n, d = 4096, 32, 4
    rho = inputs.KALMAN_RHO[n][1e4]
    Ad, As, _, B = inputs.gen_kalman(N, n, d, rho, seed=0)
    rng = np.random.default_rng(11)
    W = rng.standard_normal((N, n, d))
    X, dAd, dAs, dB = gpu_grads(S, Ad, As, B, W)
    rX = oracle.solve(Ad, As, B)
    rAd, rAs, rB = oracle.backward(Ad, As, rX, W)
    # gradients carry the kappa * u error of two solves
    assert relerr(dB, rB) <= 1e-11
    assert relerr(dAd, rAd) <= 1e-11
    assert relerr(dAs, rAs) <= 1e-11

    # central differences of the long-double loss on 64 entries: 24 symmetric diagonal-block
    # directions, 24 coupling-block entries, 16 right-hand-side entries
    h = 1e-6
    cases = []
    for _ in range(24):
        i, a, b = rng.integers(N), rng.integers(n), rng.integers(n)
        cases.append(("Ad", i, a, b))
    for _ in range(24):
        cases.append(("As", rng.integers(N - 1), rng.integers(n), rng.integers(n)))
    for _ in range(16):
        cases.append(("B", rng.integers(N), rng.integers(n), rng.integers(d)))

    def loss_at(kind, i, a, b, step):
        Ad2, As2, B2 = Ad, As, B
        if kind == "Ad":
            Ad2 = Ad.copy()
            Ad2[i, a, b] += step
            if a != b:
                Ad2[i, b, a] += step
        elif kind == "As":
            As2 = As.copy()
            As2[i, a, b] += step
        else:
            B2 = B.copy()
            B2[i, a, b] += step
        hi, lo = oracle.loss_ld(Ad2, As2, B2, W)
        return hi, lo

    def fd(case):
        p_hi, p_lo = loss_at(*case, h)
        m_hi, m_lo = loss_at(*case, -h)
        return ((p_hi - m_hi) + (p_lo - m_lo)) / (2 * h)

    with ThreadPoolExecutor(max_workers=16) as ex:
        fds = list(ex.map(fd, cases))
    for case, g_fd in zip(cases, fds):
        kind, i, a, b = case
        if kind == "Ad":
            # direction e_a e_b^T + e_b e_a^T (or e_a e_a^T): <dAd, E> with dAd symmetric
            g = dAd[i, a, b] * (2 if a != b else 1)
        elif kind == "As":
            g = dAs[i, a, b]
        else:
            g = dB[i, a, b]
        assert abs(g - g_fd) <= 1e-6 * max(1.0, abs(g_fd)), (case, g, g_fd)


def test_dot_product_identity(S):
    _say("adjoint dot product")
    N, n, d = 100, 24, 3
    Ad, As, _, B = inputs.gen_dd(N, n, d, seed=123)
    rng = np.random.default_rng(5)
    W = rng.standard_normal((N, n, d))
    X, dAd, dAs, dB = gpu_grads(S, Ad, As, B, W)
    Ed = rng.standard_normal((N, n, n))
    Ed = Ed + np.transpose(Ed, (0, 2, 1))
    Es = rng.standard_normal((N - 1, n, n))
    EX = inputs.block_matvec(Ed, Es, X)
    F = S.factor(dev(Ad), dev(As))
    dX = -F.solve(dev(EX)).cpu().numpy()
    lhs = float(np.sum(W * dX))
    rhs = float(np.sum(dAd * Ed) + np.sum(dAs * Es))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


def test_autograd_function_matches_backward(S):
    _say("autograd")
    N, n, d = 40, 16, 2
    Ad, As, _, B = inputs.gen_dd(N, n, d, seed=9)
    W = np.random.default_rng(1).standard_normal((N, n, d))
    Adt = dev(Ad).requires_grad_(True)
    Ast = dev(As).requires_grad_(True)
    Bt = dev(B).requires_grad_(True)
    X = S.solve(Adt, Ast, Bt)
    (X * dev(W)).sum().backward()
    rX = oracle.solve(Ad, As, B)
    rAd, rAs, rB = oracle.backward(Ad, As, rX, W)
    assert relerr(Adt.grad.cpu().numpy(), rAd) <= 1e-12
    assert relerr(Ast.grad.cpu().numpy(), rAs) <= 1e-12
    assert relerr(Bt.grad.cpu().numpy(), rB) <= 1e-12


def test_f32_refined_backward(S):
    _say("adjoint f32")
    N, n, d = 300, 32, 2
    Ad, As, _, B = inputs.gen_dd(N, n, d, seed=31)
    W = np.random.default_rng(2).standard_normal((N, n, d))
    X, dAd, dAs, dB = gpu_grads(S, Ad, As, B, W, prec="f32")
    rX = oracle.solve(Ad, As, B)
    rAd, rAs, rB = oracle.backward(Ad, As, rX, W)
    assert relerr(dB, rB) <= 1e-10
    assert relerr(dAd, rAd) <= 1e-10
