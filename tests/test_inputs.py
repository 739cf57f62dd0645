"""Properties of the seeded input generators (no solver arithmetic involved)."""
import numpy as np

import oracle
from paper_2509_03015_amd import inputs
from tests.dense import dense, flat
from tests.kalman_kappa import kappa


def test_gen_dd_is_seeded_symmetric_spd():
    a = inputs.gen_dd(16, 8, 2, seed=3)
    b = inputs.gen_dd(16, 8, 2, seed=3)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    Ad, As, X, B = a
    np.testing.assert_array_equal(Ad, np.transpose(Ad, (0, 2, 1)))
    w = np.linalg.eigvalsh(dense(Ad, As))
    assert w.min() > 1.0 and w.max() / w.min() < 10
    np.testing.assert_allclose(flat(B), dense(Ad, As) @ flat(X), rtol=1e-13, atol=1e-12)


def test_gen_kalman_structure():
    N, n, rho = 6, 4, 3.0
    Ad, As, X, B = inputs.gen_kalman(N, n, 1, rho, seed=1)
    F = -As[0]
    for i in range(N - 1):
        np.testing.assert_array_equal(As[i], -F)
    np.testing.assert_allclose(F @ F.T, 0.99 ** 2 * np.eye(n), atol=1e-14)
    # the last block lacks the F^T Q^-1 F term (G_{N+1} = 0)
    rng = np.random.default_rng(1)
    inputs.haar_orthogonal(rng, n)
    H = rng.standard_normal((N, n // 2, n))
    for k in range(N):
        ref = np.eye(n) + rho * H[k].T @ H[k] + (F.T @ F if k < N - 1 else 0)
        np.testing.assert_allclose(Ad[k], ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(flat(B), dense(Ad, As) @ flat(X), rtol=1e-13, atol=1e-12)


def test_kalman_rho_table_hits_kappa_targets_at_small_n():
    for target, rho in inputs.KALMAN_RHO[32].items():
        Ad, As, _, _ = inputs.gen_kalman(256, 32, 1, rho, seed=0)
        k, _, _ = kappa(Ad, As)
        assert target / 2 < k < target * 2, (target, k)


def test_batched_sizes_in_range():
    sizes = inputs.batched_sizes(512, seed=0)
    assert len(sizes) == 512
    Ns, ns, ds = zip(*sizes)
    assert min(Ns) >= 32 and max(Ns) <= 2048
    assert set(ns) == {8, 16, 32, 64} and set(ds) == {1, 4}
    assert sizes == inputs.batched_sizes(512, seed=0)


def test_generated_systems_factor_in_oracle():
    for Ad, As, _, _ in inputs.gen_batched(6, seed=2, N_range=(3, 40)):
        oracle.factor(Ad, As)
