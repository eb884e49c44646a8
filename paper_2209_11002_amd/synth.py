"""Seeded synthetic hyperspectral scenes (linear mixing model).

This module holds no step of the unmixing method: it only draws inputs.  It is
the one module that both the float64 oracle's tests and the HIP library's
tests and benchmark consume, so that both sides see identical data.

The scenes follow the linear mixing model X = M A + noise of the paper's
Section "Model formulation" (eq. LMM), with the shapes of the paper's real
scenes (Samson, Jasper Ridge, Urban; Section "Datasets"), which are not
available here and are replaced by these draws:

* endmembers: p spectra over L bands, each a clipped sum of three Gaussians
  (centre U[0, L), width U[L/40, L/8], amplitude U[0.3, 1]); redrawn while two
  endmembers are closer than 5 degrees in spectral angle;
* abundances: Dirichlet(alpha) per pixel, optionally capped at a maximum
  abundance (rejection) or spatially smoothed (Gaussian filter of each
  abundance map on the image grid, then the per-pixel contrast restored by a
  softmax of the standardised maps, see smooth_abundances);
* noise: i.i.d. Gaussian, either a fixed sigma or a target SNR in dB.

X is returned as float32 (the stored data), before any normalisation.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Scene:
    X: np.ndarray          # L x N float32, raw (not normalised)
    M: np.ndarray          # L x p float64 endmembers
    A: np.ndarray          # p x N float64 abundances
    shape: tuple = ()      # image grid (rows, cols) if any
    meta: dict = field(default_factory=dict)


def _angle_deg(u, v):
    c = float(u @ v / (np.linalg.norm(u) * np.linalg.norm(v)))
    return float(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))


def endmembers(rng, L, p, min_angle_deg=5.0):
    lam = np.arange(L, dtype=np.float64)
    for _ in range(1000):
        M = np.zeros((L, p))
        for k in range(p):
            c = rng.uniform(0.0, L, size=3)
            w = rng.uniform(L / 40.0, L / 8.0, size=3)
            a = rng.uniform(0.3, 1.0, size=3)
            M[:, k] = np.clip(np.sum(a[None, :] * np.exp(-(lam[:, None] - c[None, :]) ** 2
                                                          / (2.0 * w[None, :] ** 2)), axis=1), 0.0, 1.0)
        ok = all(_angle_deg(M[:, i], M[:, j]) >= min_angle_deg
                 for i in range(p) for j in range(i + 1, p))
        if ok and np.all(np.linalg.norm(M, axis=0) > 0):
            return M
    raise RuntimeError("could not draw well-separated endmembers")


def dirichlet(rng, alpha, p, N, max_abundance=None):
    """Dirichlet(alpha) columns via normalised Gamma draws; with
    max_abundance, columns whose largest entry exceeds it are redrawn."""
    A = rng.gamma(alpha, 1.0, size=(p, N))
    A /= A.sum(axis=0, keepdims=True)
    if max_abundance is not None:
        bad = A.max(axis=0) > max_abundance
        while np.any(bad):
            n = int(bad.sum())
            R = rng.gamma(alpha, 1.0, size=(p, n))
            R /= R.sum(axis=0, keepdims=True)
            A[:, bad] = R
            bad = A.max(axis=0) > max_abundance
    return A


SMOOTH_CONTRAST = 3.0


def smooth_abundances(A, shape, sigma_px, contrast=SMOOTH_CONTRAST):
    """Spatially smooth abundance maps from per-pixel Dirichlet draws A (p x N
    on the image grid `shape`): each map is Gaussian-filtered (sigma_px,
    reflecting boundary).  Filtering independent per-pixel draws averages
    every pixel towards the uniform mixture (at sigma = 4 px each pixel
    averages about 200 draws, so all abundances end within about 1e-2 of 1/p
    and the scene is nearly rank one), so the per-pixel contrast is restored
    afterwards: every filtered map is standardised over the image and the
    abundances of a pixel are the softmax over endmembers of `contrast` times
    its standardised values (contrast 3 gives a mean largest abundance of
    about one half at p = 12)."""
    from scipy.ndimage import gaussian_filter
    p = A.shape[0]
    S = np.empty_like(A)
    for k in range(p):
        S[k] = gaussian_filter(A[k].reshape(shape), sigma=sigma_px, mode="reflect").ravel()
    Z = (S - S.mean(axis=1, keepdims=True)) / S.std(axis=1, keepdims=True)
    Z = contrast * Z
    Z -= Z.max(axis=0, keepdims=True)
    W = np.exp(Z)
    return W / W.sum(axis=0, keepdims=True)


def scene(seed, L, N, p, alpha=1.0, sigma=0.01, snr_db=None, max_abundance=None,
          shape=None, smooth_sigma_px=None, pure_pixels=False):
    """One synthetic scene.  pure_pixels=True places one pure pixel per
    endmember at columns 0..p-1 (used for the exact-recovery checks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = endmembers(rng, L, p)
    A = dirichlet(rng, alpha, p, N, max_abundance)
    if smooth_sigma_px is not None:
        A = smooth_abundances(A, shape, smooth_sigma_px)
    if pure_pixels:
        A[:, :p] = np.eye(p)
    Y = M @ A
    if snr_db is not None:
        var = float(np.sum(Y * Y)) / (L * N * 10.0 ** (snr_db / 10.0))
        noise = rng.normal(0.0, np.sqrt(var), size=Y.shape)
    elif sigma > 0:
        noise = rng.normal(0.0, sigma, size=Y.shape)
    else:
        noise = 0.0
    X = (Y + noise).astype(np.float32)
    return Scene(X=X, M=M, A=A, shape=shape or (), meta=dict(seed=seed, L=L, N=N, p=p, alpha=alpha,
                                                             sigma=sigma, snr_db=snr_db))


# ---------------------------------------------------------------------------
# Workload recipes.  Each returns the scene plus the run setup.
# ---------------------------------------------------------------------------
GAMMA_GRID5 = (0.25, 0.5, 1.0, 2.0, 4.0)   # the middle five values of the paper's gamma set


def samson_like(seed=1):
    """Plain single run: L=156, N=95x95, p=3, Dirichlet(1), sigma 0.01,
    200 outer iterations, gamma 1, run seed 0."""
    s = scene(seed, 156, 95 * 95, 3, alpha=1.0, sigma=0.01, shape=(95, 95))
    return s, dict(T=200, K1=5, K2=5, gammas=[1.0], seeds=[0])


def jasper_like(seed=2):
    """Single run with the gradient check: L=198, N=100x100, p=4,
    Dirichlet(0.5) capped at 0.8 (no pure pixels), sigma 0.01, T=100."""
    s = scene(seed, 198, 100 * 100, 4, alpha=0.5, sigma=0.01, max_abundance=0.8, shape=(100, 100))
    return s, dict(T=100, K1=5, K2=5, gammas=[1.0], seeds=[0])


def urban_ensemble(seed=3, n_seeds=10):
    """Batched ensemble: L=162, N=307x307, p=6, Dirichlet(0.7), sigma 0.02,
    M = n_seeds x 5 gammas; run m uses seed m // 5 and gamma GAMMA_GRID5[m % 5]."""
    s = scene(seed, 162, 307 * 307, 6, alpha=0.7, sigma=0.02, shape=(307, 307))
    seeds = [m // 5 for m in range(5 * n_seeds)]
    gammas = [GAMMA_GRID5[m % 5] for m in range(5 * n_seeds)]
    return s, dict(T=100, K1=5, K2=5, gammas=gammas, seeds=seeds)


def ragged_images(n_images=64, base_seed=1000):
    """Ragged batch: image j draws N in [4096, 65536], p in [3, 8] and L in
    [156, 224] from seed base_seed + j; Dirichlet(1), sigma 0.01."""
    out = []
    for j in range(n_images):
        r = np.random.Generator(np.random.PCG64(base_seed + j))
        N = int(r.integers(4096, 65536, endpoint=True))
        p = int(r.integers(3, 8, endpoint=True))
        L = int(r.integers(156, 224, endpoint=True))
        out.append(scene(base_seed + j, L, N, p, alpha=1.0, sigma=0.01))
    return out, dict(T=100, K1=5, K2=5, gammas=[1.0], seeds=[0])


def large_smooth(seed=5, n_seeds=4):
    """Large scene: L=224, N=512x614, p=12, spatially smooth Dirichlet(1)
    (Gaussian filter sigma 4 px, contrast restored), SNR 30 dB,
    M = n_seeds x 5 gammas."""
    s = scene(seed, 224, 512 * 614, 12, alpha=1.0, snr_db=30.0, shape=(512, 614), smooth_sigma_px=4.0)
    seeds = [m // 5 for m in range(5 * n_seeds)]
    gammas = [GAMMA_GRID5[m % 5] for m in range(5 * n_seeds)]
    return s, dict(T=100, K1=5, K2=5, gammas=gammas, seeds=seeds)


def small_case(seed=11, L=40, N=333, p=3, alpha=1.0, sigma=0.01):
    """A small scene for quick parity checks (several 64-pixel tiles and a ragged tail)."""
    return scene(seed, L, N, p, alpha=alpha, sigma=sigma)
