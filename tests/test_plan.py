"""CPU checks of the launch-shape logic (edaa_plan, a host-only call): every
shape the library would launch has pass kernels whose accumulators cover all
L bands and whose LDS fits, explicit requests are honoured or refused with
EDAA_EUNSUPPORTED, and stacked-run chunks stay available at large L."""
import itertools

import pytest

from paper_2209_11002_amd import _lib as L_
from paper_2209_11002_amd import api

# compiled runs per chunk, largest first (as the library lists them)
def _choices(p):
    if p > 8:
        return [4, 2, 1]
    rmax = 8 if p > 5 else 12 if p == 5 else 16 if p == 4 else 20
    return [rmax] + ([8] if rmax > 8 else []) + [4, 1]


def _band_capacity(p, R):
    """Bands the accumulators of a chunk of R runs hold: 16-band row blocks,
    8 per wave-quarter for chunks of at most two 16-column blocks, else 4."""
    col_blocks = (p * R + 15) // 16
    return 4 * 16 * (8 if col_blocks <= 2 else 4)


def test_default_shapes_cover_every_band():
    for L, p, M in itertools.product((1, 16, 100, 162, 224, 256, 257, 272, 285, 300, 352, 400, 448),
                                     range(1, 17), (1, 2, 4, 5, 8, 13, 50, 100)):
        N = 4096
        try:
            pl = api.plan(L, N, p, M)
        except L_.EdaaError as e:
            assert e.status == L_.EDAA_EUNSUPPORTED, (L, p, M)
            continue
        R = pl["runs_per_chunk"]
        assert R in _choices(p), (L, p, M, R)
        assert L <= _band_capacity(p, R), (L, p, M, R)
        assert pl["chunks"] == -(-M // R)
        assert 1 <= pl["pixel_groups"] <= N // 64
        if M == 1:
            assert R == 1


@pytest.mark.parametrize("L,p,M", [(300, 4, 4), (300, 1, 6), (285, 4, 50), (280, 6, 8), (300, 12, 4)])
def test_large_L_keeps_stacked_runs(L, p, M):
    """Above 256 bands a chunk of at most two column blocks still stacks
    runs (an APEX-shaped L=285, p=4, M=50 ensemble no longer drops to one run
    per chunk)."""
    pl = api.plan(L, 13542, p, M)
    assert pl["runs_per_chunk"] > 1
    assert L <= _band_capacity(p, pl["runs_per_chunk"])


def test_requests_are_honoured_or_refused():
    assert api.plan(162, 94249, 6, 50, runs_per_chunk=4)["runs_per_chunk"] == 4
    assert api.plan(162, 94249, 6, 50, runs_per_chunk=4)["source"] == "requested"
    assert api.plan(162, 94249, 6, 50, pixel_groups=40)["pixel_groups"] == 40
    assert api.plan(162, 1000, 6, 50, pixel_groups=400)["pixel_groups"] == 16     # capped at the tile count
    for R in (3, 5, 16):                       # not compiled for p = 6
        with pytest.raises(L_.EdaaError) as e:
            api.plan(162, 94249, 6, 50, runs_per_chunk=R)
        assert e.value.status == L_.EDAA_EUNSUPPORTED
    with pytest.raises(L_.EdaaError) as e:     # three column blocks hold 256 bands only
        api.plan(300, 1000, 6, 8, runs_per_chunk=8)
    assert e.value.status == L_.EDAA_EUNSUPPORTED
    with pytest.raises(L_.EdaaError) as e:
        api.plan(162, 1000, 6, 8, runs_per_chunk=-1)
    assert e.value.status == L_.EDAA_EINVAL
    with pytest.raises(L_.EdaaError) as e:
        api.plan(500, 1000, 6, 8)
    assert e.value.status == L_.EDAA_EINVAL


def test_every_compiled_chunk_size_is_plannable_at_small_L():
    for p in range(1, 17):
        for R in _choices(p):
            assert api.plan(64, 2000, p, 2 * R, runs_per_chunk=R)["runs_per_chunk"] == R


def test_tuned_shapes_are_read_from_the_cache_file(tmp_path):
    """A class recorded in the file that EDAA_TUNE_CACHE names (format of
    edaa_autotune's records: tag, class, runs per chunk, pixel groups,
    microseconds; later lines win) sets the launch shape of that class only."""
    import json
    import os
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    # Urban-shaped ensemble class: L=162, p=6, M=50, float32 X, ceil(log2(1473 tiles)) = 11
    cache.write_text("edaa-tune-v1 ens:162:6:50:0:11 8 100 2000.0\n"
                     "edaa-tune-v1 ens:162:6:50:0:11 4 40 1900.0\n"
                     "edaa-tune-v1 ens:162:6:50:0:10 8 7 100.0\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import json; from paper_2209_11002_amd import api; "
            "print(json.dumps([api.plan(162, 94249, 6, 50), api.plan(162, 94249, 6, 49), api.plan(162, 40000, 6, 50),"
            " api.plan(162, 94249, 6, 50, runs_per_chunk=8)]))")
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, check=True,
                         env=dict(os.environ, EDAA_TUNE_CACHE=str(cache)))
    tuned, other_m, other_n, requested = json.loads(out.stdout.strip().splitlines()[-1])
    assert (tuned["source"], tuned["runs_per_chunk"], tuned["pixel_groups"]) == ("tuned", 4, 40)
    assert other_m["source"] == "default"                      # another M is another class
    assert (other_n["source"], other_n["runs_per_chunk"], other_n["pixel_groups"]) == ("tuned", 8, 7)
    assert requested["source"] == "requested" and requested["runs_per_chunk"] == 8


def test_bf16_matrix_passes_policy():
    """Which passes run on the bf16 matrix cores.  float32 X: the B-pass
    (operands in three bf16 terms) when a chunk has at least two 16-column
    blocks and L <= 256, the A-pass too up to p = 6 and three column blocks;
    single runs (one column block) keep the float32 matrix-core passes, as
    does EDAA_FLAG_F32_MFMA.  bf16 X: both passes up to p = 12 and L = 256
    (the B-pass above p = 12), none with EDAA_FLAG_BF16_WIDEN."""
    import torch
    bf = torch.bfloat16
    for L, N, p, M, want in [(162, 94249, 6, 50, 3), (162, 94249, 6, 1, 0), (224, 314368, 12, 20, 1),
                             (224, 314368, 12, 1, 0), (64, 900, 5, 4, 3), (30, 50, 3, 10, 1), (256, 700, 16, 2, 1),
                             (257, 700, 4, 8, 0), (300, 600, 4, 8, 0)]:
        pl = api.plan(L, N, p, M)
        assert pl["bf16_passes"] == want, (L, N, p, M, pl)
        assert api.plan(L, N, p, M, f32_mfma=True)["bf16_passes"] == 0
    for L, N, p, M, want in [(162, 94249, 6, 1, 3), (224, 314368, 12, 20, 3), (256, 700, 16, 2, 1),
                             (257, 700, 4, 8, 0)]:
        assert api.plan(L, N, p, M, x_dtype=bf)["bf16_passes"] == want, (L, N, p, M)
        assert api.plan(L, N, p, M, x_dtype=bf, bf16_widen=True)["bf16_passes"] == 0
