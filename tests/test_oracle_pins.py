"""Pins of the float64 oracle (oracle/edaa.py) against what the paper and the
mathematics fix: finite differences, the mirror-step optimality conditions,
closed forms, brute force on tiny inputs, invariants and the paper's
constants.  None of these re-types an oracle formula: each check would fail
on a dropped term, a wrong sign or index, or a transposed operand.
"""
import itertools
import os

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import edaa as O
from paper_2209_11002_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_simplex_cols(rng, d, n):
    Z = rng.gamma(1.0, 1.0, size=(d, n)) + 1e-3
    return Z / Z.sum(axis=0, keepdims=True)


def _tiny(seed=0, L=5, N=7, p=3):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.1, 1.0, size=(L, N))
    A = _rand_simplex_cols(rng, p, N)
    B = _rand_simplex_cols(rng, N, p)
    return X, A, B


# --------------------------------------------------------------------------
# paper constants (golden fixture with citations)
# --------------------------------------------------------------------------
def _golden_constants():
    vals = {}
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (s.strip() for s in line.split("=", 1))
                vals[k] = [float(t) for t in v.split()]
    return vals


def test_paper_constants():
    g = _golden_constants()
    assert list(O.GAMMA_SET) == g["gamma_set"]
    assert O.INIT_SCALE == g["init_scale"][0]
    assert (O.DEFAULT_T, O.DEFAULT_K1, O.DEFAULT_K2) == (g["T"][0], g["K1"][0], g["K2"][0])
    assert O.SELECT_THRESHOLD == g["select_threshold"][0]
    assert O.DEFAULT_M == g["M"][0]
    X, A, B = _tiny(1, L=6, N=50, p=4)
    B0 = O.init_B_from_seed(0, 50, 4)
    e1, e2 = O.step_sizes(X, B0, 1.0)
    assert e2 / e1 == pytest.approx((4 / 50) ** g["eta2_over_eta1_exponent"][0], rel=1e-14)


# --------------------------------------------------------------------------
# P1: gradients against central finite differences.  f restricted to one
# entry of A (or of B) is an exact quadratic, so the central difference has no
# truncation error, only rounding.
# --------------------------------------------------------------------------
def _fd(f, Z, h=1e-3):
    G = np.zeros_like(Z)
    for idx in np.ndindex(Z.shape):
        Zp = Z.copy(); Zp[idx] += h
        Zm = Z.copy(); Zm[idx] -= h
        G[idx] = (f(Zp) - f(Zm)) / (2 * h)
    return G


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_grad_A_finite_differences(seed):
    X, A, B = _tiny(seed)
    fd = _fd(lambda Z: O.loss(X, Z, B), A)
    g = O.grad_A(X, A, B)
    assert np.linalg.norm(g - fd) <= 1e-9 * np.linalg.norm(fd)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_grad_B_finite_differences(seed):
    X, A, B = _tiny(seed)
    fd = _fd(lambda Z: O.loss(X, A, Z), B)
    g = O.grad_B(X, A, B)
    assert g.shape == B.shape
    assert np.linalg.norm(g - fd) <= 1e-9 * np.linalg.norm(fd)


def test_grad_crop_of_mixed_scene():
    """32-pixel crop of the Jasper-Ridge-shaped scene, at a non-uniform point."""
    s, _ = synth.jasper_like()
    Xn, _ = O.normalize_pixels(s.X[:, :32].astype(np.float64))
    rng = np.random.default_rng(5)
    A = _rand_simplex_cols(rng, 4, 32)
    B = _rand_simplex_cols(rng, 32, 4)
    fdA = _fd(lambda Z: O.loss(Xn, Z, B), A, h=1e-4)
    fdB = _fd(lambda Z: O.loss(Xn, A, Z), B, h=1e-4)
    assert np.linalg.norm(O.grad_A(Xn, A, B) - fdA) <= 1e-8 * np.linalg.norm(fdA)
    assert np.linalg.norm(O.grad_B(Xn, A, B) - fdB) <= 1e-8 * np.linalg.norm(fdB)


# --------------------------------------------------------------------------
# P2: the mirror step is the minimiser of eq. EMDA.  Optimality on the
# simplex interior: log z+_j - log z_j + eta grad_j is the same for every j.
# --------------------------------------------------------------------------
def _kkt_spread(Znew, Z, G, eta):
    c = np.log(Znew) - np.log(Z) + eta * G
    return np.max(np.abs(c - c.mean(axis=0, keepdims=True)))


def test_update_A_kkt_with_fd_gradient():
    X, A, B = _tiny(3, L=6, N=9, p=3)
    eta = 0.37
    An = O.update_A(X, A, B, eta)
    fd = _fd(lambda Z: O.loss(X, Z, B), A)
    assert _kkt_spread(An, A, fd, eta) < 1e-9


def test_update_B_kkt_with_fd_gradient():
    X, A, B = _tiny(4, L=6, N=9, p=3)
    eta = 0.21
    Bn = O.update_B(X, A, B, eta)
    fd = _fd(lambda Z: O.loss(X, A, Z), B)
    assert _kkt_spread(Bn, B, fd, eta) < 1e-9
    assert np.allclose(Bn.sum(axis=0), 1.0, atol=1e-14)


def test_mirror_step_is_prox_minimiser():
    """Compare eq. update with a numerical minimisation of eq. EMDA on Delta_3."""
    rng = np.random.default_rng(0)
    for _ in range(5):
        z = _rand_simplex_cols(rng, 3, 1)[:, 0]
        g = rng.normal(size=3)
        eta = 0.8
        obj = lambda w: g @ (w - z) + (np.sum(w * np.log(w / z)) - np.sum(w) + np.sum(z)) / eta
        res = minimize(obj, z, method="SLSQP", bounds=[(1e-12, 1)] * 3,
                       constraints=[{"type": "eq", "fun": lambda w: np.sum(w) - 1}],
                       options=dict(ftol=1e-15, maxiter=500))
        zn = O.mirror_step(z[:, None], g[:, None], eta)[:, 0]
        assert np.max(np.abs(zn - res.x)) < 1e-6
        # explicit form of eq. update
        w = z * np.exp(-eta * g)
        assert np.allclose(zn, w / w.sum(), rtol=1e-14, atol=0)


# --------------------------------------------------------------------------
# P3: simplex invariants after every update (eq. simplex).
# --------------------------------------------------------------------------
def test_simplex_invariants_along_trajectory():
    s = synth.small_case(seed=21, L=24, N=300, p=4)
    X, _ = O.normalize_pixels(s.X)

    def check(t, A, B):
        assert np.all(A >= 0) and np.all(B >= 0)
        assert np.max(np.abs(np.sum(A, axis=0) - 1.0)) < 1e-12
        assert np.max(np.abs(np.sum(B, axis=0) - 1.0)) < 1e-12
        assert np.all(A > 0)          # positive start keeps entries positive

    r = O.edaa_fit(X, 4, T=20, gamma=2.0, seed=1, callback=check)
    assert np.all(np.isfinite(r["loss"]))


# --------------------------------------------------------------------------
# P4 / P5: the A-subproblem with B frozen (K2 = 0) converges to the
# simplex-constrained least-squares solution of every pixel.
# --------------------------------------------------------------------------
def _bruteforce_simplex_ls(E, x):
    """min ||x - E a||^2 over a in the simplex, by enumerating supports."""
    L, p = E.shape
    best, best_a = np.inf, None
    for k in range(1, p + 1):
        for S in itertools.combinations(range(p), k):
            Es = E[:, S]
            K = np.zeros((k + 1, k + 1))
            K[:k, :k] = Es.T @ Es
            K[:k, k] = 1.0
            K[k, :k] = 1.0
            rhs = np.concatenate([Es.T @ x, [1.0]])
            try:
                sol = np.linalg.solve(K, rhs)
            except np.linalg.LinAlgError:
                continue
            a_s = sol[:k]
            if np.any(a_s < -1e-12):
                continue
            a = np.zeros(p)
            a[list(S)] = a_s
            v = float(np.sum((x - E @ a) ** 2))
            if v < best:
                best, best_a = v, a
    return best, best_a


def _a_steps(X, B, n_steps, eta1):
    A = O.init_A(B.shape[1], X.shape[1])
    for _ in range(n_steps):
        A = O.update_A(X, A, B, eta1)
    return A


def test_A_subproblem_p2_closed_form():
    s = synth.small_case(seed=31, L=20, N=150, p=2, sigma=0.02)
    X = s.X.astype(np.float64)
    N = X.shape[1]
    # endmembers: two far-apart pixels, selected by a one-hot B
    d = np.linalg.norm(X[:, :, None] - X[:, None, :], axis=0)
    i0, i1 = np.unravel_index(np.argmax(d), d.shape)
    B = np.zeros((N, 2)); B[i0, 0] = 1.0; B[i1, 1] = 1.0
    e1, e2 = X[:, i0], X[:, i1]
    t = np.clip((X - e2[:, None]).T @ (e1 - e2) / np.sum((e1 - e2) ** 2), 0.0, 1.0)
    E = X @ B
    A = _a_steps(X, B, 4000, 1.0 / np.max(np.diag(E.T @ E)))
    interior = (t > 0.05) & (t < 0.95)
    assert interior.sum() > 50
    assert np.max(np.abs(A[0] - t)[interior]) < 1e-6
    assert np.max(np.abs(A[0] - t)) < 2e-2          # boundary solutions approach slowly


def test_A_subproblem_bruteforce_p3():
    s = synth.small_case(seed=32, L=16, N=60, p=3, sigma=0.03)
    X = s.X.astype(np.float64)
    N = X.shape[1]
    # endmembers: three mutually far-apart pixels (greedy), selected by a one-hot B
    sel = [int(np.argmax(np.linalg.norm(X - X.mean(axis=1, keepdims=True), axis=0)))]
    while len(sel) < 3:
        d = np.min(np.linalg.norm(X[:, :, None] - X[:, sel][:, None, :], axis=0), axis=1)
        sel.append(int(np.argmax(d)))
    B = np.zeros((N, 3)); B[sel, [0, 1, 2]] = 1.0
    E = X @ B
    A = _a_steps(X, B, 30000, 1.0 / np.max(np.diag(E.T @ E)))
    for i in range(N):
        fbest, abest = _bruteforce_simplex_ls(E, X[:, i])
        fe = float(np.sum((X[:, i] - E @ A[:, i]) ** 2))
        assert fe >= fbest - 1e-12
        assert fe - fbest <= 1e-5 * fbest + 1e-6
        assert np.max(np.abs(A[:, i] - abest)) < 2e-2


# --------------------------------------------------------------------------
# P6: the B-subproblem with A frozen (K1 = 0) on a tiny image reaches the
# optimum of the convex problem over the product of simplices.
# --------------------------------------------------------------------------
def test_B_subproblem_tiny_qp():
    rng = np.random.default_rng(7)
    L, N, p = 4, 6, 2
    X = rng.uniform(0.0, 1.0, size=(L, N))
    A = _rand_simplex_cols(rng, p, N)
    B = np.full((N, p), 1.0 / N)
    Lb = np.linalg.eigvalsh(X.T @ X)[-1] * np.linalg.eigvalsh(A @ A.T)[-1]
    for _ in range(20000):
        B = O.update_B(X, A, B, 1.0 / Lb)
    f_eda = O.loss(X, A, B)

    def f(v):
        return O.loss(X, A, v.reshape(N, p))
    cons = [{"type": "eq", "fun": (lambda v, j=j: v.reshape(N, p)[:, j].sum() - 1.0)} for j in range(p)]
    best = np.inf
    for s0 in range(5):
        v0 = _rand_simplex_cols(np.random.default_rng(s0), N, p).ravel()
        res = minimize(f, v0, method="SLSQP", bounds=[(0, 1)] * (N * p), constraints=cons,
                       options=dict(ftol=1e-16, maxiter=2000))
        best = min(best, res.fun)
    assert f_eda >= best - 1e-9
    assert f_eda - best <= 1e-6 * best


# --------------------------------------------------------------------------
# P7: p = 1.  A is identically 1 and the best B gives X b = mean pixel, so the
# objective tends to 1/2 sum_i ||x_i - xbar||^2.
# --------------------------------------------------------------------------
def test_p1_closed_form():
    s = synth.small_case(seed=41, L=12, N=200, p=2)
    X, _ = O.normalize_pixels(s.X)
    r = O.edaa_fit(X, 1, T=30, seed=3)
    assert np.allclose(r["A"], 1.0)
    xbar = X.mean(axis=1, keepdims=True)
    target = 0.5 * float(np.sum((X - xbar) ** 2))
    # target is the minimum; the iterates approach it from above (gap ~ 1/T)
    assert target * (1 - 1e-13) <= r["loss"][-1] <= target * (1 + 5e-8)
    assert r["loss"][0] - target > 10 * (r["loss"][-1] - target)
    assert np.all(np.diff(r["loss"]) <= 1e-12 * r["loss"][0])


# --------------------------------------------------------------------------
# P8: exact recovery on noiseless data with a pure pixel per endmember
# (without normalisation, which would move mixed pixels off the simplex).
# --------------------------------------------------------------------------
def test_exact_recovery_B_frozen_at_pure_pixels():
    s = synth.scene(7, 30, 400, 3, alpha=1.0, sigma=0.0, pure_pixels=True)
    X = s.X.astype(np.float64)
    N = X.shape[1]
    B = np.zeros((N, 3)); B[np.arange(3), np.arange(3)] = 1.0
    E = X @ B
    A = _a_steps(X, B, 20000, 1.0 / np.linalg.eigvalsh(E.T @ E)[-1])
    assert np.max(np.abs(A - s.A)) < 5e-4
    assert O.loss(X, A, B) < 1e-6


def test_exact_recovery_full_method():
    s = synth.scene(7, 30, 400, 3, alpha=1.0, sigma=0.0, pure_pixels=True)
    X = s.X.astype(np.float64)
    r = O.edaa_fit(X, 3, T=1000, gamma=1.0, seed=0)
    assert r["loss"][-1] < 1e-4 * r["loss"][0]
    perm = min(itertools.permutations(range(3)), key=lambda pm: O.sad_degrees(s.M, r["E"][:, list(pm)]))
    assert O.sad_degrees(s.M, r["E"][:, list(perm)]) < 1.0
    assert O.rmse_abundance(s.A, r["A"][list(perm)]) < 1.0


# --------------------------------------------------------------------------
# P9: step sizes against the SVD (a routine the oracle does not call).
# --------------------------------------------------------------------------
def test_step_size_vs_svd():
    s = synth.small_case(seed=51, L=30, N=500, p=5)
    X, _ = O.normalize_pixels(s.X)
    B0 = O.init_B_from_seed(9, 500, 5)
    for gamma in O.GAMMA_SET:
        e1, e2 = O.step_sizes(X, B0, gamma)
        smax = np.linalg.svd(X @ B0, compute_uv=False)[0]
        assert e1 * smax ** 2 == pytest.approx(gamma, rel=1e-12)
        assert e2 == pytest.approx(np.sqrt(5 / 500) * e1, rel=1e-14)
    r = O.edaa_fit(X, 5, T=1, K1=0, K2=0, gamma=2.0, seed=9)
    assert r["eta1"] * np.linalg.svd(X @ B0, compute_uv=False)[0] ** 2 == pytest.approx(2.0, rel=1e-12)


# --------------------------------------------------------------------------
# P10 / P11: invariances.
# --------------------------------------------------------------------------
def test_scale_invariance():
    s = synth.small_case(seed=61, L=20, N=250, p=3)
    X = s.X.astype(np.float64)
    r1 = O.edaa_fit(X, 3, T=10, gamma=1.0, seed=2)
    r2 = O.edaa_fit(2.0 * X, 3, T=10, gamma=1.0, seed=2)
    assert np.max(np.abs(r1["A"] - r2["A"])) < 1e-12
    assert np.max(np.abs(r1["B"] - r2["B"])) < 1e-12
    assert np.allclose(r2["loss"], 4.0 * r1["loss"], rtol=1e-11)


def test_permutation_equivariance():
    s = synth.small_case(seed=62, L=20, N=250, p=3)
    X, _ = O.normalize_pixels(s.X)
    B0 = O.init_B_from_seed(4, 250, 3)
    r = O.edaa_fit(X, 3, T=8, gamma=1.0, B0=B0)
    perm = np.random.default_rng(0).permutation(250)
    rp = O.edaa_fit(X[:, perm], 3, T=8, gamma=1.0, B0=B0[perm])
    assert np.max(np.abs(rp["A"] - r["A"][:, perm])) < 1e-11
    assert np.max(np.abs(rp["B"] - r["B"][perm])) < 1e-13
    q = [2, 0, 1]
    rq = O.edaa_fit(X, 3, T=8, gamma=1.0, B0=B0[:, q])
    assert np.max(np.abs(rq["A"] - r["A"][q])) < 1e-11
    assert np.max(np.abs(rq["B"] - r["B"][:, q])) < 1e-13
    assert np.allclose(rq["loss"], r["loss"], rtol=1e-12)


# --------------------------------------------------------------------------
# P12: monotone decrease.  An A-step cannot increase the objective when
# eta1 * max_j ||e_j||^2 <= 1 (l1-smoothness plus Pinsker); per outer
# iteration at gamma <= 1 the decrease is checked as an empirical property.
# --------------------------------------------------------------------------
def test_monotone_A_steps_and_outer_iterations():
    s, _ = synth.samson_like()
    X, _ = O.normalize_pixels(s.X[:, :1500])
    B0 = O.init_B_from_seed(0, 1500, 3)
    e1, e2 = O.step_sizes(X, B0, 1.0)
    A, B = O.init_A(3, 1500), B0
    f = O.loss(X, A, B)
    checked = 0
    for t in range(15):
        for _ in range(5):
            E = X @ B
            An = O.update_A(X, A, B, e1)
            fn = O.loss(X, An, B)
            if e1 * np.max(np.sum(E * E, axis=0)) <= 1.0:
                assert fn <= f * (1 + 1e-14)
                checked += 1
            A, f = An, fn
        for _ in range(5):
            B = O.update_B(X, A, B, e2)
        fo = O.loss(X, A, B)
        assert fo <= f * (1 + 1e-12)
        f = fo
    assert checked > 0


# --------------------------------------------------------------------------
# P13: B0 is close to uniform: b0_ij = exp(0.1 u_ij) / sum_i exp(0.1 u_ij),
# so N b0_ij lies in [exp(-0.1), exp(0.1)].
# --------------------------------------------------------------------------
def test_B0_near_uniform():
    N, p = 5000, 6
    B0 = O.init_B_from_seed(11, N, p)
    assert np.allclose(B0.sum(axis=0), 1.0, atol=1e-13)
    assert np.all(N * B0 <= np.exp(0.1) * (1 + 1e-12))
    assert np.all(N * B0 >= np.exp(-0.1) * (1 - 1e-12))
    A0 = O.init_A(p, N)
    assert np.all(A0 == 1.0 / p)


# --------------------------------------------------------------------------
# normalisation, fit and coherence on hand-checkable cases
# --------------------------------------------------------------------------
def test_normalize_pixels():
    X = np.array([[3.0, 0.0, 1.0], [4.0, 0.0, 1.0]])
    Xn, nz = O.normalize_pixels(X)
    assert nz == 1
    assert np.allclose(Xn[:, 0], [0.6, 0.8]) and np.all(Xn[:, 1] == 0)
    assert np.allclose(Xn[:, 2], [2 ** -0.5, 2 ** -0.5])


def test_fit_and_coherence_hand_cases():
    X = np.array([[1.0, 2.0], [0.0, -1.0]])
    E = np.array([[1.0], [1.0]])
    A = np.array([[1.0, 1.0]])
    assert O.fit_l1(X, E, A) == pytest.approx(0 + 1 + 1 + 2)
    Eo = np.array([[1.0, 0.0], [0.0, 2.0], [0.0, 0.0]])
    assert O.coherence(Eo, "raw") == 0.0 and O.coherence(Eo) == 0.0
    Es = np.array([[1.0, 2.0, 0.0], [0.0, 0.0, 1.0]])
    assert O.coherence(Es) == pytest.approx(1.0)
    assert O.coherence(Es, "raw") == pytest.approx(2.0)
    Ec = np.array([[1.0, 1.0], [0.0, 1.0]])
    assert O.coherence(Ec) == pytest.approx(np.cos(np.pi / 4))
    assert O.coherence(np.ones((3, 1))) == -np.inf


# --------------------------------------------------------------------------
# P14: selection (Algorithm 2) unit cases.
# --------------------------------------------------------------------------
def test_select_cases():
    S = O.select
    assert S([1.0], [0.5]) == 0
    assert S([1.0, 1.05, 1.2], [0.9, 0.1, 0.0]) == 1          # threshold is inclusive
    assert S([1.0, 1.0500001, 1.2], [0.9, 0.1, 0.0]) == 0
    assert S([2.0, 2.0, 2.0], [0.3, 0.3, 0.3]) == 0           # ties -> lowest index
    assert S([1.0, 1.01, 1.02], [0.5, 0.2, 0.2]) == 1
    assert S([np.nan, 1.0, np.inf], [0.0, 0.4, 0.0]) == 1     # non-finite fits excluded
    assert S([np.nan, np.inf], [0.0, 0.0]) == -1
    assert S([1.0, 1.0], [np.nan, 0.7]) == 1                  # finite mu beats NaN
    assert S([5.0, 1.0, 1.04], [0.1, 0.5, 0.4], threshold=1.05) == 2


def test_ensemble_selects_per_algorithm_2():
    s = synth.small_case(seed=71, L=20, N=300, p=3)
    X, _ = O.normalize_pixels(s.X)
    seeds, gammas = [0, 0, 1, 1], [0.5, 2.0, 0.5, 2.0]
    e = O.ensemble(X, 3, seeds, gammas, T=10)
    fits = [O.fit_l1(X, r["E"], r["A"]) for r in e["runs"]]
    mus = [O.coherence(r["E"]) for r in e["runs"]]
    fmin = min(fits)
    I = [m for m in range(4) if fits[m] <= 1.05 * fmin]
    assert e["selected"] == min(I, key=lambda m: (mus[m], m))
    for r, s_, g in zip(e["runs"], seeds, gammas):
        assert np.allclose(r["E"], X @ r["B"])
        assert r["eta1"] == pytest.approx(g / O.sigma_max_sq(X, O.init_B_from_seed(s_, 300, 3)))


# --------------------------------------------------------------------------
# Abundance estimation with given endmembers (the A-step of eq. update_A
# with E fixed): its limit is the simplex-constrained least-squares solution
# of every pixel, found here by enumerating supports; and p = 2 reduces to the
# clipped projection onto the segment [e2, e1].
# --------------------------------------------------------------------------
def test_abundances_given_E_reach_bruteforce_optimum():
    rng = np.random.default_rng(11)
    L, N, p = 12, 40, 3
    E = rng.uniform(0.1, 1.0, size=(L, p))              # endmembers not taken from X
    A_true = rng.dirichlet(np.ones(p) * 0.7, size=N).T
    X = E @ A_true + 0.02 * rng.normal(size=(L, N))
    r = O.abundances(X, E, T=4000, K1=5, gamma=1.0)
    assert np.all(np.diff(r["loss"]) <= 1e-12 * r["loss"][:-1])   # eta1 max_j ||e_j||^2 <= 1 here
    for i in range(N):
        fbest, abest = _bruteforce_simplex_ls(E, X[:, i])
        fe = float(np.sum((X[:, i] - E @ r["A"][:, i]) ** 2))
        assert fe >= fbest - 1e-12
        assert fe - fbest <= 1e-6 * fbest + 1e-8
        assert np.max(np.abs(r["A"][:, i] - abest)) < 1e-2


def test_abundances_given_E_p2_closed_form():
    rng = np.random.default_rng(12)
    L, N = 8, 30
    E = rng.uniform(0.1, 1.0, size=(L, 2))
    X = E @ rng.dirichlet([1.0, 1.0], size=N).T + 0.05 * rng.normal(size=(L, N))
    d = E[:, 0] - E[:, 1]
    a1 = np.clip(((X - E[:, [1]]).T @ d) / (d @ d), 0.0, 1.0)
    r = O.abundances(X, E, T=4000, K1=5, gamma=1.0)
    assert np.max(np.abs(r["A"][0] - a1)) < 2e-3


# --------------------------------------------------------------------------
# Algorithm 1's order and the trace timing, pinned through the functions
# already fixed above (the A-subproblem by brute force, the single updates
# by their KKT conditions), so that a loop in the wrong order, a step that
# reuses a stale residual or a trace taken at another point fails here.
# --------------------------------------------------------------------------
def _order_case():
    s = synth.small_case(seed=81, L=18, N=120, p=3)
    X, _ = O.normalize_pixels(s.X)
    rng = np.random.default_rng(81)
    # contrasted pixel weights (sparse Dirichlet columns), so that the
    # endmembers X B0 differ and every step moves the iterate visibly
    B0 = rng.dirichlet(np.full(120, 0.05), size=3).T
    A0 = _rand_simplex_cols(rng, 3, 120)
    e1, e2 = O.step_sizes(X, B0, 2.0)
    return X, A0, B0, e1, e2


def test_fit_with_B_frozen_equals_abundances_for_E_given():
    """K2 = 0: B stays at B0, so Algorithm 1 reduces to the A-steps of
    eq. update_A with E = X B0 fixed, which oracle.abundances runs and the
    brute-force simplex least squares pins (test_abundances_given_E_*)."""
    X, A0, B0, e1, e2 = _order_case()
    r = O.edaa_fit(X, 3, T=7, K1=3, K2=0, B0=B0, A0=A0, eta=(e1, e2))
    ref = O.abundances(X, X @ B0, T=7, K1=3, A0=A0, eta1=e1)
    assert np.max(np.abs(r["A"] - ref["A"])) < 1e-12
    assert np.max(np.abs(r["loss"] - ref["loss"]) / ref["loss"]) < 1e-12
    assert np.array_equal(r["B"], B0)


def test_fit_step_order_and_trace_points():
    """Outer iterations built from the KKT-pinned single updates: K1 A-steps
    on the current B, then K2 B-steps on the new A, each with a fresh
    residual; trace[0] at (A0, B0) and trace[t] after outer iteration t."""
    X, A0, B0, e1, e2 = _order_case()
    K1, K2, T = 2, 3, 2
    A, B = A0, B0
    trace = [O.loss(X, A, B)]
    for _ in range(T):
        for _ in range(K1):
            A = O.update_A(X, A, B, e1)
        for _ in range(K2):
            B = O.update_B(X, A, B, e2)
        trace.append(O.loss(X, A, B))
    r = O.edaa_fit(X, 3, T=T, K1=K1, K2=K2, B0=B0, A0=A0, eta=(e1, e2))
    assert np.max(np.abs(r["A"] - A)) < 1e-13
    assert np.max(np.abs(r["B"] - B)) < 1e-15
    assert np.max(np.abs(r["loss"] - np.array(trace)) / np.array(trace)) < 1e-13
    assert np.max(np.abs(r["E"] - X @ B)) < 1e-13

    # the data separate the orders: B-steps first (or one residual for all
    # the steps of a phase) would move the result by far more than rounding
    Ab, Bb = A0, B0
    for _ in range(T):
        for _ in range(K2):
            Bb = O.update_B(X, Ab, Bb, e2)
        for _ in range(K1):
            Ab = O.update_A(X, Ab, Bb, e1)
    assert np.max(np.abs(Ab - A)) > 1e-6 and np.max(np.abs(Bb - B)) * 120 > 1e-6
    R0 = X - (X @ B0) @ A0
    with np.errstate(divide="ignore"):
        As = O.softmax_cols(np.log(A0) + K1 * e1 * ((X @ B0).T @ R0))    # stale residual
    assert np.max(np.abs(As - O.update_A(X, O.update_A(X, A0, B0, e1), B0, e1))) > 1e-6
    # the trace is taken after the B-steps, not between the phases
    A1 = O.update_A(X, O.update_A(X, A0, B0, e1), B0, e1)
    assert abs(O.loss(X, A1, B0) - r["loss"][1]) > 1e-6 * r["loss"][1]


def test_ensemble_non_finite_run_gets_infinite_fit():
    """A run whose objective is not finite (here eta1 = inf from gamma = inf)
    gets fit = +inf, so Algorithm 2 never selects it; the other runs are the
    plain single runs."""
    s = synth.small_case(seed=82, L=16, N=90, p=3)
    X, _ = O.normalize_pixels(s.X)
    with np.errstate(invalid="ignore", over="ignore"):
        e = O.ensemble(X, 3, [0, 1, 2], [1.0, np.inf, 0.5], T=3)
    assert not np.isfinite(e["runs"][1]["loss"][-1])
    assert e["fit"][1] == np.inf
    assert e["selected"] in (0, 2)
    for m, g in ((0, 1.0), (2, 0.5)):
        one = O.edaa_fit(X, 3, T=3, gamma=g, seed=m)
        assert np.isfinite(e["fit"][m])
        assert e["fit"][m] == O.fit_l1(X, one["E"], one["A"])
    with np.errstate(invalid="ignore", over="ignore"):
        e_all = O.ensemble(X, 3, [0, 1], [np.inf, np.inf], T=2)
    assert np.all(e_all["fit"] == np.inf) and e_all["selected"] == -1


def test_hundred_envelope_fixture_rows():
    """The stored float32 spread of the 100-run GPU test (written by
    tests/golden/make_hundred_envelope.py) is reproduced by the oracle for its
    first rows, and every calm run (gamma <= 1) sits well inside 1e-4."""
    import importlib.util
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_hundred_envelope",
                                                  os.path.join(here, "make_hundred_envelope.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    env = np.loadtxt(os.path.join(here, "hundred_fp32_envelope.txt"))
    X, gammas = mk.case()
    N = X.shape[1]
    assert np.allclose(env[:, 1], gammas)
    assert np.all(env[np.array(gammas) <= 1.0, 3] < 1e-4)
    for m in (0, 1):
        ref = O.edaa_fit(X, 3, T=10, gamma=gammas[m], seed=m)
        B0 = O.init_B_from_seed(m, N, 3)
        dl = []
        for k in range(mk.N_ORDERS):
            perm = np.random.default_rng(k).permutation(N)
            r = O.edaa_fit(X[:, perm], 3, T=10, seed=m, B0=B0[perm], eta=(ref["eta1"], ref["eta2"]),
                           dtype=np.float32)
            dl.append(np.max(np.abs(r["loss"] - ref["loss"]) / ref["loss"]))
        assert np.isclose(np.median(dl), env[m, 2], rtol=1e-3) and np.isclose(np.max(dl), env[m, 3], rtol=1e-3)
