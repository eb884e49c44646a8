"""Writes large_fp64_ref.npz: float64 oracle results (Algorithm 1, K1 = K2 = 5,
the step-size rule of eq. eta0A / eq. eta0B) on the large smooth synthetic
scene (L=224, N=512x614, p=12, the 20-run ensemble of synth.large_smooth),
for stating the error of the GPU paths (float32 X and bf16 X) against
float64 at full size:

  * every run at T = 10: objective trace, E = X B, and A, B at a fixed sample
    of 256 pixels;
  * runs 0 (seed 0, gamma 0.25) and 4 (seed 0, gamma 4) at T = 100: the same.

The input is the oracle's pixel normalisation of the scene rounded to float32
(the float32 data the GPU receives).  Calls only oracle/ and the seeded scene
generator.  Takes about an hour on 8 cores.  With --float32 it writes
large_fp32_ref.npz instead: the objective traces of the same runs with the
oracle's steps in float32 (the drift of plain float32 arithmetic).

    python tests/golden/make_large_reference.py [--float32]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import edaa as O  # noqa: E402
from paper_2209_11002_amd import synth  # noqa: E402

T_ALL, T_LONG, LONG_RUNS, N_SAMPLE = 10, 100, (0, 4), 256


def sample_pixels(N):
    return np.sort(np.random.default_rng(2209).choice(N, size=N_SAMPLE, replace=False))


def main():
    scene, cfg = synth.large_smooth()
    Xn, _ = O.normalize_pixels(scene.X)
    X = Xn.astype(np.float32).astype(np.float64)
    del scene, Xn
    L, N = X.shape
    p = 12
    idx = sample_pixels(N)
    seeds, gammas = cfg["seeds"], cfg["gammas"]
    M = len(seeds)
    out = dict(idx=idx, seeds=np.array(seeds), gammas=np.array(gammas), long_runs=np.array(LONG_RUNS),
               loss10=np.zeros((M, T_ALL + 1)), E10=np.zeros((M, L, p)), A10=np.zeros((M, p, N_SAMPLE)),
               B10=np.zeros((M, N_SAMPLE, p)), eta=np.zeros((M, 2)),
               loss100=np.zeros((len(LONG_RUNS), T_LONG + 1)), E100=np.zeros((len(LONG_RUNS), L, p)),
               A100=np.zeros((len(LONG_RUNS), p, N_SAMPLE)), B100=np.zeros((len(LONG_RUNS), N_SAMPLE, p)))
    for m in range(M):
        t0 = time.time()
        keep = {}

        def cb(t, A, B, keep=keep):
            if t == T_ALL:
                keep["A"], keep["B"] = A[:, idx].copy(), B[idx, :].copy()
                keep["E"] = X @ B
        T = T_LONG if m in LONG_RUNS else T_ALL
        r = O.edaa_fit(X, p, T=T, K1=cfg["K1"], K2=cfg["K2"], gamma=gammas[m], seed=seeds[m], callback=cb)
        out["loss10"][m] = r["loss"][:T_ALL + 1]
        out["E10"][m], out["A10"][m], out["B10"][m] = keep["E"], keep["A"], keep["B"]
        out["eta"][m] = (r["eta1"], r["eta2"])
        if m in LONG_RUNS:
            k = LONG_RUNS.index(m)
            out["loss100"][k] = r["loss"]
            out["E100"][k], out["A100"][k], out["B100"][k] = r["E"], r["A"][:, idx], r["B"][idx, :]
        print(f"run {m} (seed {seeds[m]}, gamma {gammas[m]}) T={T}: loss[T] {r['loss'][-1]:.10g} "
              f"({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "large_fp64_ref.npz"), **out)


def main_f32():
    """large_fp32_ref.npz: the objective traces of the same runs with the
    oracle's steps in float32 (how far plain float32 arithmetic lands from
    float64 on this scene): loss10 [20, 11] and, for runs 0 and 4,
    loss100 [2, 101]."""
    scene, cfg = synth.large_smooth()
    Xn, _ = O.normalize_pixels(scene.X)
    X = Xn.astype(np.float32).astype(np.float64)
    del scene, Xn
    seeds, gammas = cfg["seeds"], cfg["gammas"]
    M = len(seeds)
    loss10 = np.zeros((M, T_ALL + 1))
    loss100 = np.zeros((len(LONG_RUNS), T_LONG + 1))
    for m in range(M):
        t0 = time.time()
        T = T_LONG if m in LONG_RUNS else T_ALL
        r = O.edaa_fit(X, 12, T=T, K1=cfg["K1"], K2=cfg["K2"], gamma=gammas[m], seed=seeds[m], dtype=np.float32)
        loss10[m] = r["loss"][:T_ALL + 1]
        if m in LONG_RUNS:
            loss100[LONG_RUNS.index(m)] = r["loss"]
        print(f"float32 run {m}: loss[T] {r['loss'][-1]:.10g} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "large_fp32_ref.npz"), loss10=loss10, loss100=loss100)


if __name__ == "__main__":
    if "--float32" in sys.argv:
        main_f32()
    else:
        main()
