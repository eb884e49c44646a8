"""GPU: the launch-shape autotuner records a shape that later calls of the
same class use, and results with the tuned shapes still match the oracle and
single fits."""
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


def _prep(seed, L, N, p):
    s = synth.small_case(seed=seed, L=L, N=N, p=p)
    Xn, _ = O.normalize_pixels(s.X)
    return torch.from_numpy(Xn.astype(np.float32)).cuda().contiguous(), Xn.astype(np.float32).astype(np.float64)


@gpu
def test_autotune_ensemble_shape_is_used(api):
    L, N, p, M = 60, 3000, 4, 6
    Xg, X = _prep(81, L, N, p)
    best, us = api.autotune(Xg, p, M)
    _say(f"tuned {best}, {us:.1f} us per outer iteration")
    assert us > 0
    plan = api.plan(L, N, p, M)
    assert plan["source"] == "tuned"
    assert (plan["runs_per_chunk"], plan["pixel_groups"]) == (best["runs_per_chunk"], best["pixel_groups"])
    seeds, gammas = list(range(M)), [0.5, 1.0] * (M // 2)
    r = api.ensemble(Xg, p, seeds, gammas, T=5)
    ref = O.ensemble(X, p, seeds, gammas, T=5)
    for m, rr in enumerate(ref["runs"]):
        assert np.max(np.abs(r["loss"][m] - rr["loss"]) / rr["loss"]) < 1e-4, m


@gpu
def test_autotune_bf16_class_is_its_own(api):
    """bf16 X is its own tuning class (its passes are the bf16 matrix-core
    kernels): tuning it leaves the float32 class of the same shape at its
    default, and the tuned bf16 ensemble still matches the oracle run on the
    bf16 values."""
    L, N, p, M = 52, 2500, 5, 5
    Xg, _ = _prep(83, L, N, p)
    X16 = Xg.to(torch.bfloat16)
    X64 = X16.double().cpu().numpy()
    best, us = api.autotune(X16, p, M)
    _say(f"bf16 tuned {best}, {us:.1f} us per outer iteration")
    assert api.plan(L, N, p, M, x_dtype=torch.bfloat16)["source"] == "tuned"
    assert api.plan(L, N, p, M)["source"] == "default"
    seeds, gammas = list(range(M)), [0.5, 1.0, 2.0, 0.5, 1.0]
    r = api.ensemble(X16, p, seeds, gammas, T=5)
    ref = O.ensemble(X64, p, seeds, gammas, T=5)
    for m, rr in enumerate(ref["runs"]):
        assert np.max(np.abs(r["loss"][m] - rr["loss"]) / rr["loss"]) < 1e-4, m


@gpu
def test_autotune_ragged_item_size_is_used(api):
    shapes = [(40, 3000, 3), (57, 5000, 6), (31, 700, 4), (80, 9000, 8)]
    imgs = [_prep(90 + k, L, N, p)[0] for k, (L, N, p) in enumerate(shapes)]
    ps = [p for _, _, p in shapes]
    seeds, gammas = [1, 2, 3, 4], [1.0, 0.5, 2.0, 1.0]
    tpi, us = api.autotune_ragged(imgs, ps, seeds, gammas)
    _say(f"tuned tiles per item {tpi}, {us:.1f} us per outer iteration")
    assert tpi in (1, 2, 4, 8, 16, 32, 64, 128) and us > 0
    rr = api.fit_ragged(imgs, ps, seeds, gammas, T=5)
    for k, ((L, N, p), r) in enumerate(zip(shapes, rr)):
        ntiles = (N + 63) // 64
        assert r["pixel_groups"] == (ntiles + tpi - 1) // tpi, k
        one = api.fit(imgs[k], p, T=5, gamma=gammas[k], seed=seeds[k], pixel_groups=r["pixel_groups"],
                      f32_mfma=True)
        assert torch.equal(r["A"], one["A"]) and np.array_equal(r["loss"], one["loss"]), k
