"""Pins of the scoring used by the synthetic ablation (CPU).

The oracle's RMSE (eq. RMSE), SAD (eq. SAD) and endmember pairing are
checked against closed forms, constructed angles, a library assignment
solver and brute force; the package's scoring (host code over torch CPU
tensors) is then checked against the oracle's.
"""
import itertools

import numpy as np
import pytest
import torch
from scipy.optimize import linear_sum_assignment

from oracle import edaa as O
from paper_2209_11002_amd import ablation


def _orthonormal(rng, L, k):
    q, _ = np.linalg.qr(rng.standard_normal((L, k)))
    return q


def test_rmse_closed_forms():
    rng = np.random.default_rng(0)
    p, N = 4, 37
    A = rng.dirichlet(np.ones(p), size=N).T
    # a constant offset c moves every entry by c: RMSE = 100 |c|
    assert O.rmse_abundance(A, A + 0.03) == pytest.approx(3.0, rel=1e-12)
    # one entry off by d: RMSE = 100 |d| / sqrt(p N)
    B = A.copy()
    B[2, 5] += 0.5
    assert O.rmse_abundance(A, B) == pytest.approx(50.0 / np.sqrt(p * N), rel=1e-12)
    assert O.rmse_abundance(A, A) == 0.0


def test_sad_of_constructed_angles():
    """Columns rotated by known angles theta_i inside planes orthogonal to
    each other: SAD is the mean of the theta_i in degrees, for any scale."""
    rng = np.random.default_rng(1)
    L, p = 30, 5
    Q = _orthonormal(rng, L, 2 * p)
    M, U = Q[:, :p], Q[:, p:]
    th = np.radians([1.0, 7.5, 20.0, 45.0, 90.0])
    E = (np.cos(th) * M + np.sin(th) * U) * rng.uniform(0.5, 3.0, size=p)
    assert O.sad_degrees(M * 2.0, E) == pytest.approx(np.mean([1.0, 7.5, 20.0, 45.0, 90.0]), rel=1e-12)


@pytest.mark.parametrize("p", [2, 4, 6])
def test_matching_recovers_a_permutation(p):
    """A scaled, column-permuted copy of M pairs back exactly: zero SAD and
    the abundances permuted the same way give zero RMSE."""
    rng = np.random.default_rng(p)
    M = np.abs(rng.standard_normal((25, p))) + 0.1
    A = rng.dirichlet(np.ones(p), size=50).T
    sigma = rng.permutation(p)                   # E column j = M column sigma[j]
    E = M[:, sigma] * rng.uniform(0.2, 5.0, size=p)
    Ah = A[sigma, :]
    perm = O.match_endmembers(M, E)
    assert [int(sigma[j]) for j in perm] == list(range(p))
    r = O.score(M, A, E, Ah)
    assert r["sad"] == pytest.approx(0.0, abs=1e-6)
    assert r["rmse"] == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("p", [3, 5, 8])
def test_matching_total_angle_is_the_assignment_optimum(p):
    """The exhaustive pairing reaches the optimum of the linear assignment
    problem on the angle matrix (solved by a library Hungarian solver)."""
    rng = np.random.default_rng(10 + p)
    M = np.abs(rng.standard_normal((40, p)))
    E = M[:, rng.permutation(p)] + 0.4 * np.abs(rng.standard_normal((40, p)))
    ang = np.degrees(np.arccos(np.clip((M.T @ E) / np.outer(np.linalg.norm(M, axis=0),
                                                           np.linalg.norm(E, axis=0)), -1, 1)))
    r, c = linear_sum_assignment(ang)
    perm = O.match_endmembers(M, E)
    assert sum(ang[i, perm[i]] for i in range(p)) == pytest.approx(ang[r, c].sum(), rel=1e-12)


@pytest.mark.parametrize("p", [3, 6, 9])
def test_package_scoring_matches_oracle(p):
    """The package's pairing (exhaustive up to p = 8, Hungarian above) and
    metrics agree with the oracle's on noisy estimates."""
    rng = np.random.default_rng(20 + p)
    M = np.abs(rng.standard_normal((33, p))) + 0.05
    A = rng.dirichlet(np.ones(p), size=70).T
    sigma = rng.permutation(p)
    E = M[:, sigma] + 0.3 * np.abs(rng.standard_normal((33, p)))
    Ah = np.abs(A[sigma, :] + 0.05 * rng.standard_normal((p, 70)))
    ro = O.score(M, A, E, Ah)
    rp = ablation.score(M, A, torch.from_numpy(E), torch.from_numpy(Ah))
    assert rp["perm"] == ro["perm"]
    assert rp["rmse"] == pytest.approx(ro["rmse"], rel=1e-12)
    assert rp["sad"] == pytest.approx(ro["sad"], rel=1e-12)


def test_run_draws_follow_the_step_set():
    """Seeds 0..M-1; gammas drawn from S, every value of S present at M = 100."""
    seeds, gammas = ablation.draw_runs(100, gamma_seed=0)
    assert seeds == list(range(100))
    assert set(gammas) == set(O.GAMMA_SET)
    assert ablation.GAMMA_SET == O.GAMMA_SET
    # the K sweep keeps the budget of 1000 updates: T (K1 + K2) = 1000
    assert all((500 // K) * 2 * K == 1000 for K in ablation.K_BUDGET)


def test_normalised_abundances_pins():
    """normalised_abundances (the reference restated for l2-normalised pixels):
    columns on the simplex; pure pixels stay pure; equal endmember norms leave
    the abundances unchanged; and a noise-free normalised pixel x / ||x|| lies
    on the ray of M_hat a^ (M_hat: endmembers scaled to unit norm), checked by
    a cosine of 1 and by least squares."""
    rng = np.random.default_rng(7)
    L, p, N = 30, 4, 200
    M = rng.uniform(0.1, 1.0, size=(L, p)) * rng.uniform(0.5, 3.0, size=p)[None, :]
    A = rng.dirichlet(np.ones(p), size=N).T
    A[:, :p] = np.eye(p)                                     # the first p pixels are pure
    Ah = ablation.normalised_abundances(M, A).numpy()
    assert np.all(Ah >= 0) and np.allclose(Ah.sum(axis=0), 1.0, atol=1e-14)
    assert np.allclose(Ah[:, :p], np.eye(p), atol=1e-15)
    Mu = M / np.linalg.norm(M, axis=0)
    assert np.allclose(ablation.normalised_abundances(Mu, A).numpy(), A, atol=1e-14)
    X = M @ A
    Xn = X / np.linalg.norm(X, axis=0)
    Y = Mu @ Ah
    cos = np.sum(Xn * Y, axis=0) / np.linalg.norm(Y, axis=0)
    assert np.allclose(cos, 1.0, atol=1e-12)
    # the direction determines a^: least squares of Xn on Mu, renormalised to sum 1
    C, *_ = np.linalg.lstsq(Mu, Xn, rcond=None)
    assert np.allclose(C / C.sum(axis=0), Ah, atol=1e-10)


def test_score_reports_both_references():
    rng = np.random.default_rng(8)
    L, p, N = 20, 3, 50
    M = rng.uniform(0.1, 1.0, size=(L, p))
    A = rng.dirichlet(np.ones(p), size=N).T
    r = ablation.score(M, A, M, ablation.normalised_abundances(M, A))
    assert r["rmse_normalised"] < 1e-12 and r["sad"] < 1e-5
    r = ablation.score(M, A, M, A)
    assert r["rmse"] < 1e-12
