"""GPU parity on the neuroscience-style smoothing workload (paper Sec. 4.2: N=100, n=256, m=1024).

The right-hand side is the measurement one, so the reference solution is the oracle's (whose
agreement with a Rauch-Tung-Striebel smoother is pinned on the CPU).  Bars: FP64 relative error
<= 1e-12 against the oracle and a residual at the paper's level; FP32 factor with FP64 refinement
<= 1e-10 against the long-double oracle.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2509_03015_amd import inputs
from tests.dense import flat, relerr

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


@pytest.fixture(scope="module")
def neuro():
    Ad, As, x, B, _ = inputs.gen_kalman_neuro(100, 256, 1024, seed=0)
    return Ad, As, B, oracle.solve(Ad, As, B)


@pytest.mark.parametrize("nstar", [0, 1, 8])
def test_fp64_matches_oracle_and_residual(S, neuro, nstar):
    _say("kalman-neuro fp64 nstar", nstar)
    Ad, As, B, Xo = neuro
    F = S.factor(dev(Ad), dev(As), nstar=nstar)
    X = F.solve(dev(B)).cpu().numpy()
    assert F.info()["status"] == 0
    assert relerr(X, Xo) <= 1e-12
    res = np.linalg.norm(flat(oracle.matvec(Ad, As, X) - B))
    assert res <= 1e-12 * np.linalg.norm(flat(B))


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_low_precision_factor_refines_to_oracle(S, neuro, prec):
    _say("kalman-neuro refined", prec)
    Ad, As, B, _ = neuro
    F = S.factor(dev(Ad), dev(As), prec=prec)
    X = F.solve(dev(B), refine_tol=1e-11).cpu().numpy()
    inf = F.info()
    assert inf["status"] == 0 and inf["converged"] == 1
    assert relerr(X, oracle.solve_ld(Ad, As, B)) <= 1e-10
