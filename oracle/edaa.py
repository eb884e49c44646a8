"""Plain float64 CPU oracle for Entropic Descent Archetypal Analysis (EDAA).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this module; the HIP library never does, and this
module imports nothing from it.

Every function follows the paper's statement of the method in its own
notation (X is L x N with one pixel per column, A is p x N, B is N x p,
E = X B is L x p), step by step, with no blocking, fusion or reordering
beyond what the cited passage states.  Where the paper is silent the reading
taken is stated in the docstring.

Paper passages followed:
  * Section "Model formulation": the simplex (eq. simplex) and the archetypal
    analysis objective 1/2 ||X - X B A||_F^2 (eq. AA).
  * Section "Entropic descent algorithm": the mirror step in softmax form
    (eq. update, eq. update_softmax).
  * Section "Alternating optimization scheme": eq. update_A, eq. update_B and
    Algorithm 1 (EDAA).
  * Section "Implementation details": per-pixel l2 normalisation
    (eq. normalization), A0 (eq. initA0), B0 (eq. initB0), step sizes
    (eq. eta0A, eq. eta0B) and the defaults T = 100, K1 = K2 = 5.
  * Section "Model selection procedure": l1 fit, coherence (eq. coherence)
    and Algorithm 2 (model selection).
  * Section "Experimental setup": abundance RMSE (eq. RMSE) and
    spectral angle distance (eq. SAD).
"""
import numpy as np

from .philox import uniform_u

# Constants the paper fixes (Section "Implementation details", Section
# "Model selection procedure").
GAMMA_SET = (0.125, 0.25, 0.5, 1.0, 2.0, 4.0, 8.0)   # S, eq. eta0A
INIT_SCALE = 0.1                                      # eq. initB0
DEFAULT_T, DEFAULT_K1, DEFAULT_K2 = 100, 5, 5         # "Hyperparameters"
SELECT_THRESHOLD = 1.05                               # Algorithm 2
DEFAULT_M = 50                                        # Section "Model selection procedure"


def normalize_pixels(X):
    """eq. normalization: x_i <- x_i / ||x_i||_2 for every pixel (column).

    Reading (paper silent): a pixel of zero norm is left as zeros.
    Returns (normalised copy, number of zero-norm pixels)."""
    X = np.array(X, dtype=np.float64, copy=True)
    norms = np.sqrt(np.sum(X * X, axis=0))
    zero = norms == 0.0
    X[:, ~zero] = X[:, ~zero] / norms[~zero]
    X[:, zero] = 0.0
    return X, int(np.count_nonzero(zero))


def softmax_cols(Z):
    """softmax applied independently to every column (the "first dimension"
    of Algorithm 1).  The column maximum is subtracted before exponentiating;
    softmax is invariant to that shift.  Entries equal to -inf give 0."""
    Z = np.asarray(Z)
    m = np.max(Z, axis=0, keepdims=True)
    e = np.exp(Z - m)
    return e / np.sum(e, axis=0, keepdims=True)


def init_A(p, N, dtype=np.float64):
    """eq. initA0: A0 = (1/p) 1_p 1_N^T."""
    return np.full((p, N), 1.0 / p, dtype=dtype)


def init_B(U, scale=INIT_SCALE):
    """eq. initB0: b0_j = softmax(0.1 u) per column j, u ~ U[0,1]^N.
    U is N x p (one column per endmember)."""
    return softmax_cols(scale * np.asarray(U))


def init_B_from_seed(seed, N, p, scale=INIT_SCALE):
    """B0 from the counter-based draw of oracle.philox.uniform_u."""
    return init_B(uniform_u(seed, N, p), scale)


def sigma_max_sq(X, B0):
    """sigma_max^2 of X B0 (eq. eta0A) computed as the largest eigenvalue of
    the p x p Gram matrix (X B0)^T (X B0)."""
    E0 = X @ B0
    return float(np.linalg.eigvalsh(E0.T @ E0)[-1])


def step_sizes(X, B0, gamma):
    """eq. eta0A and eq. eta0B: eta1 = gamma / sigma_max^2(X B0),
    eta2 = sqrt(p / N) eta1.  Constant for the whole run."""
    N, p = B0.shape
    eta1 = gamma / sigma_max_sq(X, B0)
    eta2 = np.sqrt(p / N) * eta1
    return eta1, eta2


def loss(X, A, B):
    """eq. AA objective: 1/2 ||X - X B A||_F^2."""
    R = X - (X @ B) @ A
    return 0.5 * float(np.sum(R * R))


def grad_A(X, A, B):
    """Gradient of 1/2 ||X - XBA||^2 with respect to A: -(XB)^T (X - XBA).
    eq. update_A adds eta times the negative of this to log A."""
    E = X @ B
    return -(E.T @ (X - E @ A))


def grad_B(X, A, B):
    """Gradient with respect to B: -X^T (X - XBA) A^T (eq. update_B),
    associated as X^T ((X - XBA) A^T) so that no N x N matrix is formed."""
    R = X - (X @ B) @ A
    return -(X.T @ (R @ A.T))


def mirror_step(Z, G, eta):
    """eq. update_softmax applied per column: softmax(log Z - eta G).
    Z lies on the simplex column-wise; G is the gradient at Z."""
    with np.errstate(divide="ignore"):
        return softmax_cols(np.log(Z) - eta * G)


def update_A(X, A, B, eta1):
    """eq. update_A: A <- softmax(log A + eta1 B^T X^T (X - X B A)),
    with B^T X^T taken as (X B)^T."""
    E = X @ B
    with np.errstate(divide="ignore"):
        return softmax_cols(np.log(A) + eta1 * (E.T @ (X - E @ A)))


def update_B(X, A, B, eta2):
    """eq. update_B: B <- softmax(log B + eta2 X^T (X - X B A) A^T),
    softmax over the N entries of each column of B."""
    R = X - (X @ B) @ A
    with np.errstate(divide="ignore"):
        return softmax_cols(np.log(B) + eta2 * (X.T @ (R @ A.T)))


def edaa_fit(X, p, T=DEFAULT_T, K1=DEFAULT_K1, K2=DEFAULT_K2, gamma=1.0,
             seed=0, B0=None, A0=None, eta=None, init_scale=INIT_SCALE,
             dtype=np.float64, callback=None):
    """Algorithm 1 (EDAA).

    X       L x N data (Algorithm 1 expects it l2-normalised per pixel; this
            function does not normalise, see normalize_pixels).
    B0, A0  optional explicit starting points (resume, tests); default to
            eq. initB0 drawn with `seed` and eq. initA0.
    eta     optional (eta1, eta2) override; default eq. eta0A / eq. eta0B
            from B0.
    dtype   float64 (the oracle) or float32 (a drift diagnostic only).
    callback(t, A, B) is called after every outer iteration if given.

    Readings (the paper keeps no trace): loss[0] is the objective at
    (A0, B0) and loss[t] the objective after outer iteration t.  The K1
    A-steps of an outer iteration come first, each with a fresh residual,
    then the K2 B-steps (the order of Algorithm 1).

    Returns a dict with E (= X B), A, B, loss (T+1 values), eta1, eta2.
    """
    X = np.asarray(X, dtype=dtype)
    L, N = X.shape
    B = (init_B_from_seed(seed, N, p, init_scale) if B0 is None
         else np.array(B0, dtype=np.float64)).astype(dtype)
    A = (init_A(p, N) if A0 is None else np.array(A0, dtype=np.float64)).astype(dtype)
    if eta is None:
        eta1, eta2 = step_sizes(X.astype(np.float64), B.astype(np.float64), gamma)
    else:
        eta1, eta2 = float(eta[0]), float(eta[1])
    e1, e2 = dtype(eta1), dtype(eta2)
    trace = [loss(X, A, B)]
    for t in range(1, T + 1):
        for _ in range(K1):
            A = update_A(X, A, B, e1)
        for _ in range(K2):
            B = update_B(X, A, B, e2)
        trace.append(loss(X, A, B))
        if callback is not None:
            callback(t, A, B)
    return dict(E=X @ B, A=A, B=B, loss=np.array(trace), eta1=eta1, eta2=eta2)


def abundances(X, E, T=DEFAULT_T, K1=DEFAULT_K1, gamma=1.0, A0=None, eta1=None):
    """Abundance estimation with the endmembers E (L x p) given: minimise
    1/2 ||X - E A||_F^2 over A with every column on the simplex (the
    non-negativity and sum-to-one constraints of the Introduction's
    abundance estimation once endmembers are known), by the entropic steps
    of eq. update_A with the given E in place of X B:
        A <- softmax(log A + eta1 E^T (X - E A)).

    Readings (the paper runs this step only inside Algorithm 1): A0 as in
    eq. initA0; eta1 = gamma / sigma_max^2(E), the rule of eq. eta0A applied
    to the given E; T outer iterations of K1 steps each, loss[0] at A0 and
    loss[t] after outer iteration t.

    Returns a dict with A, loss (T+1 values) and eta1."""
    X = np.asarray(X, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    p = E.shape[1]
    N = X.shape[1]
    A = init_A(p, N) if A0 is None else np.array(A0, dtype=np.float64)
    if eta1 is None:
        eta1 = gamma / float(np.linalg.eigvalsh(E.T @ E)[-1])

    def obj(A):
        R = X - E @ A
        return 0.5 * float(np.sum(R * R))

    trace = [obj(A)]
    for t in range(1, T + 1):
        for _ in range(K1):
            A = mirror_step(A, -(E.T @ (X - E @ A)), eta1)
        trace.append(obj(A))
    return dict(A=A, loss=np.array(trace), eta1=eta1)


def fit_l1(X, E, A):
    """l1 fit of Algorithm 2: ||X - E A||_1, read as the entrywise sum of
    absolute values over the L x N residual (Section "Model selection
    procedure" states the fit once as ||X - XAB||_1, which does not conform
    dimensionally; Algorithm 2 writes ||X - E_m A_m||_1, which is used)."""
    return float(np.sum(np.abs(X - E @ A)))


def coherence(E, mode="cosine"):
    """eq. coherence: mu = max over k != k' of <e_k, e_k'>.

    mode "raw" is the inner product as printed.  mode "cosine" (default)
    first scales every column to unit l2 norm, the reading of the text's
    "maximal pairwise spectral correlation"; the two coincide for unit-norm
    endmembers.  For p = 1 there is no pair and mu = -inf."""
    E = np.asarray(E, dtype=np.float64)
    if mode == "cosine":
        n = np.sqrt(np.sum(E * E, axis=0))
        E = E / np.where(n > 0, n, 1.0)
    elif mode != "raw":
        raise ValueError(mode)
    p = E.shape[1]
    if p < 2:
        return float("-inf")
    Gm = E.T @ E
    off = ~np.eye(p, dtype=bool)
    return float(np.max(Gm[off]))


def select(fit, mu, threshold=SELECT_THRESHOLD):
    """Algorithm 2 selection: fit_min = min fit; I = {m : fit_m <=
    threshold * fit_min} (inclusive); best = argmin over I of mu.

    Readings (paper silent): non-finite fits are excluded before fit_min is
    taken; equal mu values resolve to the lowest run index; a non-finite mu
    never wins over a finite one.  Returns -1 when no fit is finite."""
    fit = np.asarray(fit, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    ok = np.isfinite(fit)
    if not np.any(ok):
        return -1
    fmin = np.min(fit[ok])
    best, best_mu = -1, None
    for m in range(len(fit)):
        if not ok[m] or not (fit[m] <= threshold * fmin):
            continue
        if best < 0:
            best, best_mu = m, mu[m]
            continue
        if np.isnan(best_mu) and not np.isnan(mu[m]):
            best, best_mu = m, mu[m]
        elif mu[m] < best_mu:
            best, best_mu = m, mu[m]
    return best


def ensemble(X, p, seeds, gammas, T=DEFAULT_T, K1=DEFAULT_K1, K2=DEFAULT_K2,
             coherence_mode="cosine", threshold=SELECT_THRESHOLD,
             init_scale=INIT_SCALE, dtype=np.float64):
    """Algorithm 2: one EDAA run per (seed_m, gamma_m), its l1 fit and
    coherence, then the selection.  Returns a dict with the list of runs,
    fit, mu and the selected index."""
    runs, fits, mus = [], [], []
    for s, g in zip(seeds, gammas):
        r = edaa_fit(X, p, T=T, K1=K1, K2=K2, gamma=g, seed=s,
                     init_scale=init_scale, dtype=dtype)
        runs.append(r)
        f = fit_l1(X, r["E"], r["A"])
        fits.append(f if np.isfinite(r["loss"][-1]) else np.inf)
        mus.append(coherence(r["E"], coherence_mode))
    fits = np.array(fits)
    mus = np.array(mus)
    return dict(runs=runs, fit=fits, mu=mus, selected=select(fits, mus, threshold))


def rmse_abundance(A_true, A_hat):
    """eq. RMSE (Section "Experimental setup"): 100 sqrt(sum (A - A_hat)^2 / (p N))."""
    A_true = np.asarray(A_true)
    return 100.0 * float(np.sqrt(np.mean((A_true - np.asarray(A_hat)) ** 2)))


def sad_degrees(M, E_hat):
    """eq. SAD: mean over endmembers of the spectral angle in degrees,
    columns paired as given."""
    M = np.asarray(M, dtype=np.float64)
    E_hat = np.asarray(E_hat, dtype=np.float64)
    c = np.sum(M * E_hat, axis=0) / (np.linalg.norm(M, axis=0) * np.linalg.norm(E_hat, axis=0))
    return float(np.mean(np.degrees(np.arccos(np.clip(c, -1.0, 1.0)))))


def match_endmembers(M, E_hat):
    """Pairing of estimated with reference endmembers before scoring.  The
    paper does not say how the columns are paired (Section "Experimental
    setup", eq. SAD); the reading taken is the pairing of least total
    spectral angle, found here by trying every one of the p! pairings
    (p <= 9).  Returns perm with E_hat[:, perm[i]] paired to M[:, i]."""
    M = np.asarray(M, dtype=np.float64)
    E_hat = np.asarray(E_hat, dtype=np.float64)
    p = M.shape[1]
    if p > 9:
        raise ValueError("exhaustive pairing is limited to p <= 9")
    import itertools
    ang = np.zeros((p, p))                   # angle between M[:, i] and E_hat[:, j]
    for i in range(p):
        for j in range(p):
            c = np.dot(M[:, i], E_hat[:, j]) / (np.linalg.norm(M[:, i]) * np.linalg.norm(E_hat[:, j]))
            ang[i, j] = np.degrees(np.arccos(np.clip(c, -1.0, 1.0)))
    perms = np.array(list(itertools.permutations(range(p))))
    cost = ang[np.arange(p)[None, :], perms].sum(axis=1)
    return [int(v) for v in perms[int(np.argmin(cost))]]


def score(M, A, E_hat, A_hat):
    """Global abundance RMSE (eq. RMSE) and SAD (eq. SAD) of an estimate
    after pairing its endmembers with the reference ones."""
    perm = match_endmembers(M, E_hat)
    E_hat = np.asarray(E_hat, dtype=np.float64)[:, perm]
    A_hat = np.asarray(A_hat, dtype=np.float64)[perm, :]
    return dict(rmse=rmse_abundance(A, A_hat), sad=sad_degrees(M, E_hat), perm=perm)
