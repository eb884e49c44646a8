"""Abundance estimation with given endmembers (eq. update_A with E fixed,
through edaa_abundances) against the float64 oracle's abundances()."""
import sys

import numpy as np
import pytest
import torch

from oracle import edaa as O
from paper_2209_11002_amd import synth

gpu = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2209_11002_amd import api as A
    return A


@gpu
@pytest.mark.parametrize("L,N,p,gamma", [(40, 333, 3, 1.0), (156, 1000, 6, 0.5), (224, 700, 12, 2.0)])
def test_abundances_vs_oracle(api, L, N, p, gamma):
    _say(f"abundances L={L} N={N} p={p} gamma={gamma} T=20")
    s = synth.small_case(seed=70 + p, L=L, N=N, p=min(p, 8))
    Xn, _ = O.normalize_pixels(s.X)
    X32 = Xn.astype(np.float32)
    # endmembers: the scene's spectra (p > 8: plus pixels of the scene), unit norm, float32
    rng = np.random.default_rng(p)
    E = np.concatenate([s.M, X32[:, rng.choice(N, max(0, p - s.M.shape[1]), replace=False)]], axis=1)[:, :p]
    E = (E / np.linalg.norm(E, axis=0)).astype(np.float32)
    r = api.abundances(torch.from_numpy(X32).cuda(), torch.from_numpy(E).cuda(), T=20, K1=5, gamma=gamma)
    ref = O.abundances(X32.astype(np.float64), E.astype(np.float64), T=20, K1=5, gamma=gamma)
    rel = np.max(np.abs(r["loss"] - ref["loss"]) / ref["loss"])
    A_err = np.max(np.abs(r["A"].cpu().numpy() - ref["A"]))
    _say(f"loss rel {rel:.2e}  A {A_err:.2e}  eta1 rel {abs(r['eta1'] / ref['eta1'] - 1):.2e}")
    assert r["eta1"] == pytest.approx(ref["eta1"], rel=1e-5)
    assert rel <= 1e-5 and A_err <= 1e-4
    A = r["A"].cpu().numpy().astype(np.float64)
    assert np.all(A >= 0) and np.max(np.abs(A.sum(axis=0) - 1)) < 1e-5


@gpu
def test_abundances_bf16_X_and_resume(api):
    """bf16 X (the oracle runs on the same bf16 values), and resuming from
    the A and eta1 of a first call equals one longer call."""
    s = synth.small_case(seed=77, L=60, N=450, p=4)
    Xn, _ = O.normalize_pixels(s.X)
    X16 = torch.from_numpy(Xn.astype(np.float32)).to(torch.bfloat16)
    X64 = X16.to(torch.float64).numpy()
    E = (s.M / np.linalg.norm(s.M, axis=0)).astype(np.float32)
    Eg = torch.from_numpy(E).cuda()
    r = api.abundances(X16.cuda(), Eg, T=12, K1=5, gamma=1.0)
    ref = O.abundances(X64, E.astype(np.float64), T=12, K1=5, gamma=1.0)
    rel = np.max(np.abs(r["loss"] - ref["loss"]) / ref["loss"])
    _say(f"bf16 abundances: loss rel {rel:.2e}")
    assert rel <= 1e-5 and np.max(np.abs(r["A"].cpu().numpy() - ref["A"])) <= 1e-4
    r1 = api.abundances(X16.cuda(), Eg, T=6, K1=5, gamma=1.0)
    r2 = api.abundances(X16.cuda(), Eg, T=6, K1=5, A0=r1["A"], eta1=r1["eta1"])
    assert np.max(np.abs(r2["loss"] - r["loss"][6:]) / r["loss"][6:]) <= 1e-6
    assert np.max(np.abs(r2["A"].cpu().numpy() - r["A"].cpu().numpy())) <= 1e-6
