"""GPU: the entry point that allocates nothing (edaa_fit_noalloc) against
edaa_fit on the same inputs: two calls in a row on one context, the second
on a smaller problem, must reproduce edaa_fit's outputs (same kernels, same
launch shape and order of operations, so bit-identical), leave the device's
free memory unchanged, and refuse what it cannot hold."""
import sys

import numpy as np
import pytest
import torch

from oracle import edaa as O
from paper_2209_11002_amd import _lib as L_
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
    return torch.from_numpy(Xn.astype(np.float32)).cuda().contiguous()


@gpu
def test_noalloc_matches_fit_twice_then_smaller(api):
    dev = torch.device("cuda:0")
    api.set_graph_cache(dev, 16)           # creates this stream's context (and looks up the scratch array)
    for (seed, L, N, p, T, gamma) in ((71, 60, 1000, 4, 8, 2.0), (72, 40, 333, 3, 5, 0.5)):
        _say(f"noalloc vs fit L={L} N={N} p={p} T={T}")
        X = _prep(seed, L, N, p)
        ref = api.fit(X, p, T=T, gamma=gamma, seed=seed)
        out = dict(A=torch.full((p, N), np.nan, device=dev), B=torch.full((N, p), np.nan, device=dev),
                   E=torch.full((L, p), np.nan, device=dev),
                   loss=torch.full((T + 1,), np.nan, dtype=torch.float64, device=dev),
                   eta=torch.full((2,), np.nan, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info(dev)
        api.fit_noalloc(X, p, out, T=T, gamma=gamma, seed=seed)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info(dev)
        assert free1 == free0, (free0, free1)
        assert torch.equal(out["A"], ref["A"]) and torch.equal(out["B"], ref["B"]) and torch.equal(out["E"], ref["E"])
        assert np.array_equal(out["loss"].cpu().numpy(), ref["loss"])
        assert np.array_equal(out["eta"].cpu().numpy(), [ref["eta1"], ref["eta2"]])


@gpu
def test_noalloc_matches_fit_bf16(api):
    """The same with bf16 X (the bf16 matrix-core passes)."""
    dev = torch.device("cuda:0")
    L, N, p, T, seed = 50, 700, 5, 6, 73
    _say(f"noalloc vs fit, bf16 X, L={L} N={N} p={p} T={T}")
    X = _prep(seed, L, N, p).to(torch.bfloat16)
    ref = api.fit(X, p, T=T, gamma=1.0, seed=seed)
    out = dict(A=torch.full((p, N), np.nan, device=dev), B=torch.full((N, p), np.nan, device=dev),
               E=torch.full((L, p), np.nan, device=dev),
               loss=torch.full((T + 1,), np.nan, dtype=torch.float64, device=dev))
    api.fit_noalloc(X, p, out, T=T, gamma=1.0, seed=seed)
    torch.cuda.synchronize()
    assert torch.equal(out["A"], ref["A"]) and torch.equal(out["B"], ref["B"]) and torch.equal(out["E"], ref["E"])
    assert np.array_equal(out["loss"].cpu().numpy(), ref["loss"])


@gpu
def test_noalloc_refuses_what_it_cannot_hold(api):
    dev = torch.device("cuda:0")
    X = torch.zeros((448, 8), device=dev)
    P = L_.default_params()
    lib = L_.load()
    ctx = api._ctx(dev)
    # 448 x 600000 pixels need more than the 256 MiB scratch array: refused before anything is enqueued
    st = lib.edaa_fit_noalloc(ctx, api._ptr(X), 448, 600000, 4, P, 0, None, None,
                              api._ptr(X), api._ptr(X), None, None, None)
    assert st == L_.EDAA_EUNSUPPORTED
    assert b"scratch" in lib.edaa_last_error()
    P.flags = L_.EDAA_FLAG_GRAPH
    st = lib.edaa_fit_noalloc(ctx, api._ptr(X), 448, 8, 4, P, 0, None, None,
                              api._ptr(X), api._ptr(X), None, None, None)
    assert st == L_.EDAA_EINVAL
