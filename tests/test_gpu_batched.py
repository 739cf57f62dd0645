"""GPU parity of the batched form (bds_factor_batched / bds_solve_batched) against the CPU oracle.

Each system of a batch is compared with the oracle's solve of that system alone: FP64 relative error
<= 1e-12; FP32 factor + FP64 refinement <= 1e-10 (the systems here have kappa ~ 4).
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


def run_batch(S, systems, prec="f64", nstar=0):
    Ads = [dev(s[0]) for s in systems]
    Ass = [dev(s[1]) if s[0].shape[0] > 1 else None for s in systems]
    Bs = [dev(s[3]) for s in systems]
    F = S.factor_batched(Ads, Ass, prec=prec, nstar=nstar)
    Xs = F.solve(Bs)
    torch.cuda.synchronize()
    return [X.cpu().numpy() for X in Xs], F


UNEVEN = [(1, 16, 1), (2, 3, 2), (7, 8, 1), (33, 17, 3), (64, 32, 4), (100, 16, 17), (5, 64, 1), (128, 1, 2),
          (31, 40, 5), (200, 8, 4), (3, 128, 2), (17, 24, 33)]


def uneven_systems(seed0=0):
    return [inputs.gen_dd(N, n, d, seed=seed0 + 17 * k + 1) for k, (N, n, d) in enumerate(UNEVEN)]


@pytest.mark.parametrize("nstar", [0, 3])
def test_batched_fp64_uneven_matches_oracle(S, nstar):
    _say("batched fp64 uneven nstar", nstar)
    systems = uneven_systems()
    Xs, F = run_batch(S, systems, nstar=nstar)
    assert all(inf["status"] == 0 for inf in F.info())
    for (Ad, As, _, B), X in zip(systems, Xs):
        assert relerr(X, oracle.solve(Ad, As, B)) <= 1e-12, Ad.shape


def test_batched_fp32_refined_matches_oracle(S):
    _say("batched fp32 uneven")
    systems = uneven_systems(seed0=500)
    Xs, F = run_batch(S, systems, prec="f32")
    infos = F.info()
    for (Ad, As, _, B), X, inf in zip(systems, Xs, infos):
        assert inf["status"] == 0 and inf["converged"] == 1 and 1 <= inf["iters"] <= 30, inf
        assert relerr(X, oracle.solve_ld(Ad, As, B)) <= 1e-10, Ad.shape


def test_batched_equals_single_system_solves(S):
    _say("batched vs single")
    systems = uneven_systems(seed0=900)
    Xs, _ = run_batch(S, systems)
    for (Ad, As, _, B), X in zip(systems, Xs):
        F1 = S.factor(dev(Ad), dev(As) if Ad.shape[0] > 1 else None)
        X1 = F1.solve(dev(B)).cpu().numpy()
        assert relerr(X, X1) <= 1e-13


def test_batched_single_member(S):
    _say("batched K=1")
    sysm = [inputs.gen_dd(50, 16, 2, seed=3)]
    Xs, _ = run_batch(S, sysm)
    Ad, As, _, B = sysm[0]
    assert relerr(Xs[0], oracle.solve(Ad, As, B)) <= 1e-12


def test_batched_not_spd_flags_only_that_system(S):
    _say("batched not spd")
    systems = uneven_systems(seed0=1300)
    bad = 4
    Ad = systems[bad][0].copy()
    Ad[3] = -np.eye(Ad.shape[1])
    systems[bad] = (Ad,) + tuple(systems[bad][1:])
    Ads = [dev(s[0]) for s in systems]
    Ass = [dev(s[1]) if s[0].shape[0] > 1 else None for s in systems]
    F = S.factor_batched(Ads, Ass, check=False)
    infos = F.info()
    for k, inf in enumerate(infos):
        if k == bad:
            assert inf["status"] == S.bb.BDS_ENOTSPD
        else:
            assert inf["status"] == 0, (k, inf)


def test_batched_repeat_is_bitwise_deterministic(S):
    _say("batched determinism")
    systems = uneven_systems(seed0=77)
    X1, _ = run_batch(S, systems)
    X2, _ = run_batch(S, systems)
    for a, b in zip(X1, X2):
        np.testing.assert_array_equal(a, b)


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batched_512_uneven_systems(S, prec):
    """The full uneven batch: 512 systems, N ~ U{32..2048}, n in {8,16,32,64}, d in {1,4}."""
    _say("batched 512", prec)
    systems = inputs.gen_batched(512, seed=0)
    Xs, F = run_batch(S, systems, prec=prec)
    infos = F.info()
    assert all(inf["status"] == 0 for inf in infos)
    # every system against its manufactured solution (kappa <= 5 here)
    worst = max(relerr(X, s[2]) for X, s in zip(Xs, systems))
    assert worst <= 1e-12
    # a sample of systems against the oracle, element by element
    rng = np.random.default_rng(0)
    for k in rng.choice(512, size=24, replace=False):
        Ad, As, _, B = systems[k]
        ref = oracle.solve(Ad, As, B) if prec == "f64" else oracle.solve_ld(Ad, As, B)
        assert relerr(Xs[k], ref) <= (1e-12 if prec == "f64" else 1e-10), (k, Ad.shape)


def test_batched_factor_replay_reads_current_values(S):
    """The batched factor's launch sequence is replayed as a graph; a refactor after the matrices changed
    in place (same buffers) must use the new values, and the task tables of another batch in between
    must not leak into the replay."""
    _say("batched graph replay")
    systems = uneven_systems(seed0=40)
    Ads = [dev(s[0]) for s in systems]
    Ass = [dev(s[1]) if s[0].shape[0] > 1 else None for s in systems]
    Bs = [dev(s[3]) for s in systems]
    F = S.factor_batched(Ads, Ass)
    F.solve(Bs)
    # another batch of different shapes factorised in between
    other = uneven_systems(seed0=90)[:5]
    S.factor_batched([dev(s[0]) for s in other], [dev(s[1]) if s[0].shape[0] > 1 else None for s in other])
    for k, (Ad, As, _, _) in enumerate(systems):
        Ads[k].copy_(dev(2.0 * Ad))
        if Ass[k] is not None:
            Ass[k].copy_(dev(2.0 * As))
    for _ in range(2):
        F.refactor(check=True)
        Xs = F.solve(Bs)
        for (Ad, As, _, B), X in zip(systems, Xs):
            assert relerr(X.cpu().numpy(), oracle.solve(2.0 * Ad, 2.0 * As, B)) <= 1e-12, Ad.shape
