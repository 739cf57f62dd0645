"""GPU parity of libbds against the CPU oracle (through the C ABI via the ctypes binding).

FP64 bar: relative Frobenius error <= 1e-12 against the FP64 oracle at the
well-conditioned sizes (kappa ~ 4).  Mixed-precision bar: <= 1e-10 after
refinement, against the long-double oracle.
"""
import os
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


def gpu_solve(S, Ad, As, B, prec="f64", nstar=0, **kw):
    F = S.factor(dev(Ad), dev(As) if Ad.shape[0] > 1 else None, prec=prec, nstar=nstar)
    X = F.solve(dev(B), **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy(), F


def test_fp64_N64_n16_d1_matches_oracle(S):
    _say("fp64 N=64 n=16 d=1")
    Ad, As, Xt, B = inputs.gen_dd(64, 16, 1, seed=0)
    X, F = gpu_solve(S, Ad, As, B)
    assert F.info()["status"] == 0
    Xo = oracle.solve(Ad, As, B)
    assert relerr(X, Xo) <= 1e-12
    assert relerr(X, Xt) <= 1e-12


SWEEP = [(N, n, d) for N in (1, 2, 3, 4, 5, 7, 8, 9, 16, 17, 31, 33, 64, 100)
         for n, d in ((1, 1), (3, 2), (16, 1), (17, 3), (32, 16), (40, 17))]


@pytest.mark.parametrize("N,n,d", SWEEP)
def test_fp64_sweep_matches_oracle(S, N, n, d):
    _say("sweep", N, n, d)
    Ad, As, _, B = inputs.gen_dd(N, n, d, seed=1000 + N * 7 + n)
    X, _ = gpu_solve(S, Ad, As, B)
    assert relerr(X, oracle.solve(Ad, As, B)) <= 1e-12


@pytest.mark.parametrize("nstar", [1, 2, 3, 5, 8, 64, 200])
@pytest.mark.parametrize("n", [8, 64])
def test_fp64_crossover_nstar(S, nstar, n):
    _say("nstar", nstar, n)
    N, d = 77, 2
    Ad, As, _, B = inputs.gen_dd(N, n, d, seed=nstar)
    X, _ = gpu_solve(S, Ad, As, B, nstar=nstar)
    assert relerr(X, oracle.solve(Ad, As, B)) <= 1e-12


@pytest.mark.parametrize("n", [128, 256])
def test_fp64_large_blocks(S, n):
    _say("large n", n)
    N, d = 45, 3
    Ad, As, _, B = inputs.gen_dd(N, n, d, seed=n)
    X, _ = gpu_solve(S, Ad, As, B)
    assert relerr(X, oracle.solve(Ad, As, B)) <= 1e-12


def test_fp64_repeat_is_bitwise_deterministic(S):
    _say("determinism")
    Ad, As, _, B = inputs.gen_dd(300, 32, 4, seed=5)
    X1, _ = gpu_solve(S, Ad, As, B)
    X2, _ = gpu_solve(S, Ad, As, B)
    np.testing.assert_array_equal(X1, X2)


def test_factor_reused_for_many_solves(S):
    _say("reuse")
    Ad, As, _, _ = inputs.gen_dd(50, 16, 1, seed=6)
    F = S.factor(dev(Ad), dev(As))
    rng = np.random.default_rng(0)
    for d in (1, 5, 16, 33):
        B = rng.standard_normal((50, 16, d))
        X = F.solve(dev(B)).cpu().numpy()
        assert relerr(X, oracle.solve(Ad, As, B)) <= 1e-12


def test_upper_triangle_of_diagonal_blocks_not_read(S):
    _say("lower only")
    Ad, As, _, B = inputs.gen_dd(40, 32, 2, seed=7)
    junk = Ad.copy()
    iu = np.triu_indices(32, 1)
    for i in range(40):
        junk[i][iu] = np.nan
    X, _ = gpu_solve(S, junk, As, B)
    assert relerr(X, oracle.solve(Ad, As, B)) <= 1e-12


@pytest.mark.parametrize("N,bad", [(1, 0), (2, 1), (33, 0), (33, 17), (33, 32), (64, 40)])
def test_not_spd_is_reported(S, N, bad):
    _say("not spd", N, bad)
    Ad, As, _, _ = inputs.gen_dd(N, 16, 1, seed=8)
    Ad = Ad.copy()
    Ad[bad] = -np.eye(16)
    F = S.factor(dev(Ad), dev(As) if N > 1 else None, check=False)
    inf = F.info()
    assert inf["status"] == S.bb.BDS_ENOTSPD
    with pytest.raises(oracle.OracleError):
        oracle.factor(Ad, As)


@pytest.mark.parametrize("half,col", [(0, 5), (1, 131), (1, 255)])
def test_not_spd_in_either_half_of_a_256_block(S, half, col):
    """Blocks of 256 rows are factorised as two 128-row halves; a non-positive pivot in either half is
    reported, with its column counted from the start of the block."""
    _say("not spd 256", half, col)
    N, n = 9, 256
    Ad, As, _, _ = inputs.gen_dd(N, n, 1, seed=21)
    Ad = Ad.copy()
    # make the leading (col + 1) x (col + 1) block of an interior singular at column col: a Schur pivot of zero
    blk = 3                                   # an interior at level 0 (odd position)
    v = np.linalg.cholesky(Ad[blk][:col, :col]) if col > 0 else None
    row = Ad[blk][col, :col]
    y = np.linalg.solve(v, row) if col > 0 else np.zeros(0)
    Ad[blk][col, col] = float(y @ y) - 1.0    # pivot col becomes -1
    F = S.factor(dev(Ad), dev(As), check=False)
    inf = F.info()
    assert inf["status"] == S.bb.BDS_ENOTSPD, inf
    assert (inf["level"], inf["orig_block"], inf["column"]) == (0, blk, col), inf
    with pytest.raises(oracle.OracleError):
        oracle.factor(Ad, As)


def test_nan_input_is_reported(S):
    _say("nan")
    Ad, As, _, _ = inputs.gen_dd(20, 16, 1, seed=9)
    Ad = Ad.copy()
    Ad[6, 3, 3] = np.nan
    F = S.factor(dev(Ad), dev(As), check=False)
    assert F.info()["status"] == S.bb.BDS_ENOTSPD


@pytest.mark.slow
def test_fp64_N16384_n128_d16_full_size_properties(S):
    """N=16384, n=128, d=16 (the benchmark configuration): manufactured solution and backward error."""
    _say("fp64 N=16384 n=128 d=16 full size")
    Ad, As, Xt, B = inputs.gen_dd(16384, 128, 16, seed=0)
    X, F = gpu_solve(S, Ad, As, B)
    assert F.info()["status"] == 0
    assert relerr(X, Xt) <= 1e-12
    R = B - inputs.block_matvec(Ad, As, X)
    eta = np.linalg.norm(R) / (np.linalg.norm(Ad) * np.linalg.norm(X) + np.linalg.norm(B))
    assert eta <= 1e-15
    # sampled blocks: the first 64 block rows equal the oracle's solve of the whole system
    # restricted there is not computable alone; compare against the oracle on a leading
    # subsystem is invalid, so sample via the residual instead (done above).


@pytest.mark.parametrize("N,n,d,prec", [(1200, 128, 16, "f64"), (600, 256, 1, "f64"), (1100, 128, 2, "f32")])
def test_levels_across_the_small_launch_forms(S, N, n, d, prec):
    """Sizes whose top levels have more interiors than CUs and whose deeper levels have fewer, so that
    one solve runs both launch forms of every kernel that has two (16-wave factor work-groups and
    unrolled or 8-wave solve sweeps on small levels, the 256-row split with its per-tile link products)."""
    _say("small-launch crossover", N, n, d, prec)
    Ad, As, Xt, B = inputs.gen_dd(N, n, d, seed=N + n)
    X, F = gpu_solve(S, Ad, As, B, prec=prec, **({"refine_tol": 1e-12} if prec != "f64" else {}))
    assert F.info()["status"] == 0
    assert relerr(X, oracle.solve(Ad, As, B)) <= (1e-12 if prec == "f64" else 1e-10)
