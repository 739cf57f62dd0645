"""Graph replay of the launch sequences (csrc/bds_graph.*).

The first bds_factor / FP64 bds_solve with a given argument set records its
launches into a HIP graph; later identical calls replay it.  Replays must give
the same bits as direct launches (kernel timing on forces direct launches),
must read the buffers' current contents, and must stay correct over several
replays with eager work on the stream in between.
"""
import sys

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


@pytest.mark.parametrize("N,n,d", [(64, 16, 1), (100, 32, 4), (45, 128, 16), (33, 40, 3)])
def test_replay_matches_direct_launches(S, N, n, d):
    _say("graph replay", N, n, d)
    Ad, As, _, B = inputs.gen_dd(N, n, d, seed=70 + N)
    Ad_t, As_t, B_t = dev(Ad), dev(As), dev(B)
    # direct launches (timing on)
    S.bb.trace_enable(4096)
    F = S.factor(Ad_t, As_t)
    X_direct = F.solve(B_t).clone()
    torch.cuda.synchronize()
    S.bb.trace_read()
    S.bb.trace_enable(0)
    # first untimed call records, the following ones replay
    X = torch.empty_like(B_t)
    for rep in range(4):
        F.refactor()
        F.solve(B_t, out=X)
        torch.cuda.synchronize()
        assert torch.equal(X, X_direct), f"replay {rep} differs from direct launches"
        # eager work on the stream between replays
        _ = (Ad_t * 2.0).sum()
    assert relerr(X.cpu().numpy(), oracle.solve(Ad, As, B)) <= 1e-12


def test_replay_reads_current_buffer_contents(S):
    _say("graph replay new contents")
    N, n, d = 77, 32, 2
    Ad, As, _, B = inputs.gen_dd(N, n, d, seed=81)
    Ad_t, As_t, B_t = dev(Ad), dev(As), dev(B)
    F = S.factor(Ad_t, As_t)
    X = torch.empty_like(B_t)
    F.solve(B_t, out=X)
    F.solve(B_t, out=X)  # graph recorded and replayed
    rng = np.random.default_rng(5)
    for _ in range(3):
        # new matrix and right-hand side in the same buffers: refactor + solve replay the graphs
        Ad2, As2, _, B2 = inputs.gen_dd(N, n, d, seed=int(rng.integers(1 << 30)))
        Ad_t.copy_(dev(Ad2))
        As_t.copy_(dev(As2))
        B_t.copy_(dev(B2))
        F.refactor(check=True)
        F.solve(B_t, out=X)
        torch.cuda.synchronize()
        assert relerr(X.cpu().numpy(), oracle.solve(Ad2, As2, B2)) <= 1e-12


def test_replay_reports_not_spd(S):
    _say("graph replay not spd")
    N, n = 40, 16
    Ad, As, _, _ = inputs.gen_dd(N, n, 1, seed=90)
    Ad_t, As_t = dev(Ad), dev(As)
    F = S.factor(Ad_t, As_t)
    F.refactor(check=True)  # replay, SPD
    bad = Ad.copy()
    bad[11] = -np.eye(n)
    Ad_t.copy_(dev(bad))
    F.refactor(check=False)  # replay, info written by the graph's kernels
    assert F.info()["status"] == S.bb.BDS_ENOTSPD
    Ad_t.copy_(dev(Ad))
    F.refactor(check=False)
    assert F.info()["status"] == 0  # the graph's first kernel clears the info record
