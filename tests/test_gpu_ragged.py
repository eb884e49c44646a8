"""Ragged batch (single runs on images of different L, N, p, advanced
together): every image must give exactly what a single-image fit with the
same number of pixel groups gives (the persistent kernel and the
launch-per-kernel path run the same kernel bodies on the same geometry, with
the same order of every sum), and agree with the float64 oracle to the float32
tolerances."""
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


# (L, N, p): three images share p = 4, tails of 1..63 pixels, p from 1 to
# 16, fewer pixels than one tile, and L > 256 (more row blocks per wave)
SHAPES = [(40, 333, 4), (57, 1000, 3), (31, 64, 1), (64, 777, 4), (20, 130, 16), (156, 2500, 6), (300, 50, 4)]


def _images(dtype=torch.float32):
    out = []
    for k, (L, N, p) in enumerate(SHAPES):
        s = synth.small_case(seed=100 + k, L=L, N=N, p=min(p, 8))
        Xn, _ = O.normalize_pixels(s.X)
        Xt = torch.from_numpy(Xn.astype(np.float32)).to(dtype)
        out.append((Xt.cuda().contiguous(), Xt.to(torch.float64).numpy(), p))
    return out


def _check_equal_to_single(api, imgs, rr, T, gammas, seeds):
    for k, ((Xg, _, p), r) in enumerate(zip(imgs, rr)):
        # the ragged passes run on the float32 matrix cores
        single = api.fit(Xg, p, T=T, gamma=gammas[k], seed=seeds[k], pixel_groups=r["pixel_groups"],
                         f32_mfma=True)
        assert torch.equal(r["A"], single["A"]), k
        assert torch.equal(r["B"], single["B"]), k
        assert torch.equal(r["E"], single["E"]), k
        assert np.array_equal(r["loss"], single["loss"]), k


@gpu
def test_ragged_equals_single_image_fits(api):
    """Images with p <= 9 run in the persistent kernel, the p = 16 image with
    one launch per kernel."""
    _say("ragged vs single fits:", SHAPES)
    imgs = _images()
    seeds = [11 * k + 1 for k in range(len(imgs))]
    gammas = [0.5, 1.0, 2.0, 1.0, 0.25, 1.0, 4.0]
    rr = api.fit_ragged([x for x, _, _ in imgs], [p for _, _, p in imgs], seeds, gammas, T=12)
    _check_equal_to_single(api, imgs, rr, 12, gammas, seeds)


@gpu
@pytest.mark.parametrize("tiles_per_item", [1, 3, 8])
def test_ragged_persistent_many_images(api, tiles_per_item):
    """Sixteen images of p in [1, 9] and up to 12 000 pixels in the persistent
    kernel (work items of 1, 3 or 8 tiles), against single fits."""
    rng = np.random.default_rng(77)
    imgs, shapes = [], []
    for k in range(16):
        L, N, p = int(rng.integers(20, 120)), int(rng.integers(60, 12000)), int(rng.integers(1, 10))
        s = synth.small_case(seed=300 + k, L=L, N=N, p=min(p, 8))
        Xn, _ = O.normalize_pixels(s.X)
        Xt = torch.from_numpy(Xn.astype(np.float32))
        imgs.append((Xt.cuda().contiguous(), None, p))
        shapes.append((L, N, p))
    _say(f"ragged persistent, tiles per item {tiles_per_item}: {shapes}")
    seeds = list(range(16))
    gammas = [(0.25, 1.0, 4.0)[k % 3] for k in range(16)]
    rr = api.fit_ragged([x for x, _, _ in imgs], [p for _, _, p in imgs], seeds, gammas, T=6,
                        tiles_per_item=tiles_per_item)
    _check_equal_to_single(api, imgs, rr, 6, gammas, seeds)


@gpu
def test_ragged_persistent_equals_grouped(api):
    """The persistent kernel and the launch-per-kernel path give identical
    results for the same pixel groups."""
    _say("ragged persistent vs grouped")
    imgs = _images()
    args = ([x for x, _, _ in imgs], [p for _, _, p in imgs], list(range(len(imgs))), [1.0] * len(imgs))
    rp = api.fit_ragged(*args, T=7)
    rg = api.fit_ragged(*args, T=7, grouped=True, pixel_groups=[r["pixel_groups"] for r in rp])
    for k in range(len(imgs)):
        assert torch.equal(rp[k]["A"], rg[k]["A"]) and torch.equal(rp[k]["B"], rg[k]["B"]), k
        assert np.array_equal(rp[k]["loss"], rg[k]["loss"]), k


@gpu
def test_ragged_vs_oracle(api):
    _say("ragged vs oracle T=8")
    imgs = _images()
    seeds = list(range(len(imgs)))
    gammas = [1.0] * len(imgs)
    rr = api.fit_ragged([x for x, _, _ in imgs], [p for _, _, p in imgs], seeds, gammas, T=8)
    for k, ((_, X, p), r) in enumerate(zip(imgs, rr)):
        ref = O.edaa_fit(X, p, T=8, gamma=1.0, seed=seeds[k])
        rel = np.max(np.abs(r["loss"] - ref["loss"]) / ref["loss"])
        A_err = np.max(np.abs(r["A"].cpu().numpy() - ref["A"]))
        NB_err = X.shape[1] * np.max(np.abs(r["B"].cpu().numpy() - ref["B"]))
        _say(f"image {k} {SHAPES[k]}: loss rel {rel:.2e} A {A_err:.2e} N*B {NB_err:.2e}")
        assert rel <= 1e-4 and A_err <= 1e-3 and NB_err <= 1e-2, k


@gpu
def test_ragged_graph_replay(api):
    _say("ragged graph replay x3")
    imgs = _images()
    args = ([x for x, _, _ in imgs], [p for _, _, p in imgs], list(range(len(imgs))), [1.0] * len(imgs))
    eager = api.fit_ragged(*args, T=6)
    for rep in range(3):
        rg = api.fit_ragged(*args, T=6, graph=True)
        torch.cuda.synchronize()
        for k in range(len(imgs)):
            assert torch.equal(rg[k]["A"], eager[k]["A"]) and torch.equal(rg[k]["B"], eager[k]["B"]), (rep, k)
            assert np.array_equal(rg[k]["loss"], eager[k]["loss"]), (rep, k)
        _ = (imgs[0][0] * 2.0).sum().item()      # eager work between replays
