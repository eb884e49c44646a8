"""Writes urban_fp64_traces.txt: the float64 oracle's objective trace
(Algorithm 1, T = 100, K1 = K2 = 5) on the Urban-shaped synthetic scene for
two runs of the benchmark ensemble (seed 0 with gamma 0.25 and gamma 4, the
step-size rule of eq. eta0A / eta0B).  The input is the oracle's pixel
normalisation rounded to float32, exactly what the GPU tests hand the
library.  Calls only oracle/ and the seeded scene generator.

    python tests/golden/make_urban_traces.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import edaa as O  # noqa: E402
from paper_2209_11002_amd import synth  # noqa: E402

RUNS = ((0, 0.25), (0, 4.0))   # (seed, gamma)


def main():
    scene, cfg = synth.urban_ensemble()
    Xn, _ = O.normalize_pixels(scene.X)
    X = Xn.astype(np.float32).astype(np.float64)
    cols = []
    for seed, gamma in RUNS:
        r = O.edaa_fit(X, 6, T=cfg["T"], K1=cfg["K1"], K2=cfg["K2"], gamma=gamma, seed=seed)
        cols.append(r["loss"])
        print(f"seed {seed} gamma {gamma}: loss[0] {r['loss'][0]:.10g} loss[T] {r['loss'][-1]:.10g}", flush=True)
    out = os.path.join(HERE, "urban_fp64_traces.txt")
    header = ("float64 oracle objective trace, Urban-shaped scene (L=162, N=307x307, p=6), T=100, K1=K2=5;\n"
              "columns: t, seed 0 gamma 0.25, seed 0 gamma 4; written by make_urban_traces.py")
    np.savetxt(out, np.column_stack([np.arange(len(cols[0])), *cols]), fmt=["%d", "%.17g", "%.17g"], header=header)


if __name__ == "__main__":
    main()
