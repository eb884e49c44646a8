"""Edge shapes and the BF16 row at the large scene's (L, p).

BF16 storage: the oracle runs on exactly the bf16 values the GPU reads, so
the float32 arithmetic is gated at the float32 tolerances; the effect of the
bf16 rounding itself (against the same runs on the float32 X) is reported
and only loosely bounded, since it is a property of the data, not of the
kernels."""
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


def _prep(X, dtype=torch.float32):
    Xn, _ = O.normalize_pixels(X)
    Xt = torch.from_numpy(Xn.astype(np.float32)).to(dtype)
    return Xt.cuda().contiguous(), Xt.to(torch.float64).numpy()


def _np(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


@gpu
def test_bf16_large_scene_shape_vs_oracle(api):
    """L = 224, p = 12, spatially smooth Dirichlet(1) abundances at SNR 30 dB
    (the large scene's recipe) on a 32 x 64 crop; M = 4 runs, T = 10."""
    s = synth.scene(5, 224, 32 * 64, 12, alpha=1.0, snr_db=30.0, shape=(32, 64), smooth_sigma_px=4.0)
    _say("bf16 X L=224 N=2048 p=12 M=4 T=10")
    X16g, X16 = _prep(s.X, torch.bfloat16)
    X32g, X32 = _prep(s.X, torch.float32)
    seeds, gammas = [0, 0, 1, 1], [0.5, 2.0, 1.0, 4.0]
    r16 = api.ensemble(X16g, 12, seeds, gammas, T=10)
    r32 = api.ensemble(X32g, 12, seeds, gammas, T=10)
    N = X16.shape[1]
    for m in range(4):
        ref = O.edaa_fit(X16, 12, T=10, gamma=gammas[m], seed=seeds[m])
        rel = np.max(np.abs(r16["loss"][m] - ref["loss"]) / ref["loss"])
        A_err = np.max(np.abs(_np(r16["A"][m]) - ref["A"]))
        NB_err = N * np.max(np.abs(_np(r16["B"][m]) - ref["B"]))
        q = np.max(np.abs(r16["loss"][m] - r32["loss"][m]) / r32["loss"][m])
        _say(f"run {m}: bf16 vs oracle on the bf16 X: loss {rel:.2e} A {A_err:.2e} N*B {NB_err:.2e}; "
             f"bf16 vs float32 X: loss {q:.2e}")
        assert rel <= 1e-4 and A_err <= 1e-3 and NB_err <= 1e-2
        assert q <= 5e-2


@gpu
@pytest.mark.parametrize("L,N,p,M,T", [
    (1, 100, 2, 1, 6),       # a single band
    (30, 50, 3, 10, 6),      # fewer pixels than one tile, 20 runs per chunk
    (25, 200, 3, 21, 5),     # the last chunk holds a single run
    (17, 64, 6, 9, 5),       # exactly one tile, two chunks (8 + 1 runs)
])
def test_edge_shapes_vs_oracle(api, L, N, p, M, T):
    _say(f"edge shape L={L} N={N} p={p} M={M} T={T}")
    s = synth.small_case(seed=40 + L, L=L, N=N, p=min(p, max(1, L)))
    Xg, X = _prep(s.X)
    seeds = [m // 2 for m in range(M)]
    gammas = [(0.5, 2.0)[m % 2] for m in range(M)]
    r = api.ensemble(Xg, p, seeds, gammas, T=T)
    # objectives near zero (L = 1: every normalised pixel is 1 and X B A
    # reproduces it exactly) are compared against a floor of 1e-7 x
    # 1/2 ||X||^2, the float32 resolution of the objective
    floor = 1e-7 * 0.5 * float(np.sum(X * X))
    for m in sorted({0, M // 2, M - 1}):
        ref = O.edaa_fit(X, p, T=T, gamma=gammas[m], seed=seeds[m])
        rel = np.max(np.abs(r["loss"][m] - ref["loss"]) / np.maximum(ref["loss"], floor))
        A_err = np.max(np.abs(_np(r["A"][m]) - ref["A"]))
        NB_err = N * np.max(np.abs(_np(r["B"][m]) - ref["B"]))
        _say(f"run {m}: loss {rel:.2e} A {A_err:.2e} N*B {NB_err:.2e}")
        assert rel <= 1e-4 and A_err <= 1e-3 and NB_err <= 1e-2
        A = _np(r["A"][m])
        B = _np(r["B"][m])
        assert np.max(np.abs(A.sum(axis=0) - 1)) < 1e-5 and np.max(np.abs(B.sum(axis=0) - 1)) < 1e-5


@gpu
def test_ragged_bf16_equals_single_fits(api):
    _say("ragged bf16: 3 images vs single fits")
    shapes = [(40, 333, 4), (64, 700, 5), (31, 129, 4)]
    imgs = []
    for k, (L, N, p) in enumerate(shapes):
        s = synth.small_case(seed=60 + k, L=L, N=N, p=p)
        imgs.append((_prep(s.X, torch.bfloat16)[0], p))
    rr = api.fit_ragged([x for x, _ in imgs], [p for _, p in imgs], [1, 2, 3], [1.0, 0.5, 2.0], T=8)
    for k, ((Xg, p), r) in enumerate(zip(imgs, rr)):
        # the ragged kernels run bf16 X on the float32 matrix cores
        one = api.fit(Xg, p, T=8, gamma=[1.0, 0.5, 2.0][k], seed=k + 1, pixel_groups=r["pixel_groups"],
                      bf16_widen=True)
        assert torch.equal(r["A"], one["A"]) and torch.equal(r["B"], one["B"]), k
        assert np.array_equal(r["loss"], one["loss"]), k


@gpu
@pytest.mark.parametrize("L,N,p,M,T", [
    (64, 900, 5, 1, 8),      # one run: one column block, k blocks split between wave pairs
    (162, 1000, 6, 10, 6),   # 8 runs per chunk (three column blocks), L not a multiple of 32
    (224, 2048, 12, 4, 6),   # the large scene's (L, p): four runs per chunk
    (256, 700, 16, 2, 5),    # the largest L of the bf16 matrix path, two column blocks
    (1, 100, 2, 1, 6),       # a single band: one k block of 32 with 31 zero bands
    (30, 50, 3, 10, 5),      # fewer pixels than one tile, 20 runs per chunk (four column blocks)
    (120, 800, 4, 4, 5),     # four runs per chunk, A-steps of a run spread over lane pairs
    (96, 500, 9, 4, 5),      # four runs per chunk at p = 9
    (224, 3000, 12, 1, 5),   # one run at the large scene's (L, p): A-steps over lane quads
])
def test_bf16_matrix_path_vs_oracle(api, L, N, p, M, T):
    """bf16 X on the bf16 matrix cores (the default for bf16 X: both passes
    up to p = 12 and L = 256, the B-pass above p = 12) against the oracle run
    on the same bf16 values, at the float32 gates; and against the
    float32-matrix-core path (bf16_widen), which computes the same products
    in float32: the two must agree to float32 rounding but not be identical
    (a check that the bf16 path ran)."""
    _say(f"bf16 matrix path L={L} N={N} p={p} M={M} T={T}")
    # L = 1 checks the 31 zero bands of the k block on the all-positive
    # single-band scene of test_edge_shapes_vs_oracle (seed 41).  With mixed
    # signs (seed 71: pixels normalise to +-1) the objective falls from 24 to
    # 1.9 in six iterations and plain float32 arithmetic already moves it by
    # 4.6e-5 there, growing tenfold per iteration: no float32 gate holds.
    s = synth.small_case(seed=41 if L == 1 else 70 + L, L=L, N=N, p=min(p, max(1, L)))
    Xg, X = _prep(s.X, torch.bfloat16)
    seeds = [m // 2 for m in range(M)]
    gammas = [(0.5, 1.0)[m % 2] for m in range(M)]
    r = api.ensemble(Xg, p, seeds, gammas, T=T) if M > 1 else None
    if M == 1:
        one = api.fit(Xg, p, T=T, gamma=gammas[0], seed=seeds[0])
        wide = api.fit(Xg, p, T=T, gamma=gammas[0], seed=seeds[0], bf16_widen=True)
        r = dict(loss=one["loss"][None], A=one["A"][None], B=one["B"][None])
        rw = dict(loss=wide["loss"][None])
    else:
        rw = api.ensemble(Xg, p, seeds, gammas, T=T, bf16_widen=True)
    floor = 1e-7 * 0.5 * float(np.sum(X * X))
    for m in sorted({0, M // 2, M - 1}):
        ref = O.edaa_fit(X, p, T=T, gamma=gammas[m], seed=seeds[m])
        rel = np.max(np.abs(r["loss"][m] - ref["loss"]) / np.maximum(ref["loss"], floor))
        A_err = np.max(np.abs(_np(r["A"][m]) - ref["A"]))
        NB_err = N * np.max(np.abs(_np(r["B"][m]) - ref["B"]))
        dw = np.max(np.abs(r["loss"][m] - rw["loss"][m]) / np.maximum(rw["loss"][m], floor))
        _say(f"run {m}: vs oracle loss {rel:.2e} A {A_err:.2e} N*B {NB_err:.2e}; vs float32 matrix path {dw:.2e}")
        assert rel <= 1e-4 and A_err <= 1e-3 and NB_err <= 1e-2
        assert dw <= 1e-4
    if L > 1:
        assert not np.array_equal(r["loss"], rw["loss"])


@gpu
@pytest.mark.parametrize("L,N,p,M,T", [
    (64, 900, 5, 1, 8),      # one run, one column block: the float32 matrix-core passes serve
    (162, 1000, 6, 10, 6),   # 8 runs per chunk: three column blocks, k blocks split, L not a multiple of 32
    (64, 900, 5, 4, 6),      # 4 runs per chunk: two column blocks, k blocks split
    (224, 2048, 12, 4, 6),   # three column blocks without room for the second projection buffer
    (256, 700, 16, 2, 5),    # the largest L of the path, two column blocks
    (1, 100, 2, 10, 6),      # a single band: one k block of 32 with 31 zero bands
    (30, 50, 3, 10, 5),      # fewer pixels than one tile, 20 runs per chunk (four column blocks)
    (156, 2500, 3, 8, 6),    # two column blocks at p = 3
    (300, 600, 4, 8, 5),     # L > 256: the float32 matrix-core passes serve
])
def test_f32_split_path_vs_oracle(api, L, N, p, M, T):
    """float32 X runs its B-pass (and, up to p = 6, its A-pass) on the bf16
    matrix cores with both operands in three bf16 terms when a chunk has at
    least two column blocks and L <= 256 (plan()'s bf16_passes says which):
    against the oracle at the float32 gates, and against the float32
    matrix-core passes (f32_mfma), which must agree to float32 rounding and
    differ exactly when the plan names a bf16 pass (a check of which
    kernels ran)."""
    _say(f"float32 split path L={L} N={N} p={p} M={M} T={T}")
    s = synth.small_case(seed=41 if L == 1 else 90 + L, L=L, N=N, p=min(p, max(1, L)))
    Xg, X = _prep(s.X)
    seeds = [m // 2 for m in range(M)]
    gammas = [(0.5, 1.0)[m % 2] for m in range(M)]
    passes = api.plan(L, N, p, M)["bf16_passes"]
    assert api.plan(L, N, p, M, f32_mfma=True)["bf16_passes"] == 0
    if M == 1:
        one = api.fit(Xg, p, T=T, gamma=gammas[0], seed=seeds[0])
        ref32 = api.fit(Xg, p, T=T, gamma=gammas[0], seed=seeds[0], f32_mfma=True)
        r = dict(loss=one["loss"][None], A=one["A"][None], B=one["B"][None])
        rw = dict(loss=ref32["loss"][None], A=ref32["A"][None])
    else:
        r = api.ensemble(Xg, p, seeds, gammas, T=T)
        rw = api.ensemble(Xg, p, seeds, gammas, T=T, f32_mfma=True)
    floor = 1e-7 * 0.5 * float(np.sum(X * X))
    for m in sorted({0, M // 2, M - 1}):
        ref = O.edaa_fit(X, p, T=T, gamma=gammas[m], seed=seeds[m])
        rel = np.max(np.abs(r["loss"][m] - ref["loss"]) / np.maximum(ref["loss"], floor))
        A_err = np.max(np.abs(_np(r["A"][m]) - ref["A"]))
        NB_err = N * np.max(np.abs(_np(r["B"][m]) - ref["B"]))
        dw = np.max(np.abs(r["loss"][m] - rw["loss"][m]) / np.maximum(rw["loss"][m], floor))
        _say(f"run {m} (bf16 passes {passes}): vs oracle loss {rel:.2e} A {A_err:.2e} N*B {NB_err:.2e}; "
             f"vs float32 matrix path {dw:.2e}")
        assert rel <= 1e-4 and A_err <= 1e-3 and NB_err <= 1e-2
        assert dw <= 1e-4
    same = np.array_equal(r["loss"], rw["loss"]) and torch.equal(r["A"], rw["A"])
    assert same == (passes == 0)
