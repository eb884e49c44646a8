"""Writes jasper_full_ref.npz: the float64 oracle on the full Jasper-Ridge-
shaped scene (L=198, N=100x100, p=4, Dirichlet(0.5) capped at 0.8, sigma
0.01; one run, seed 0, gamma 1, T=100, K1=K2=5, Algorithm 1 with the step
rule of eq. eta0A / eq. eta0B), and how far plain float32 arithmetic lands
from it: the oracle's own steps in float32 with the pixels in 8 orders (a
permutation of the pixels is an exact symmetry of Algorithm 1, so each order
is an equally valid float32 evaluation).  The input is the oracle's pixel
normalisation rounded to float32, as the GPU tests hand it to the library.
Calls only oracle/ and the seeded scene generator.

Arrays: loss (T+1, float64), A (p x N) and NB (N x p, N times B) rounded to
float32 (far below the 1e-3 / 1e-2 gates they serve);
f32_loss_max / f32_loss_med (T+1: largest / median relative deviation of the
objective at each t over the 8 orders); f32_A_max, f32_NB_max (largest
absolute deviation of A and N B over the orders).

    python tests/golden/make_jasper_reference.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import edaa as O  # noqa: E402
from paper_2209_11002_amd import synth  # noqa: E402

N_ORDERS = 8
P = 4


def data():
    s, cfg = synth.jasper_like()
    Xn, _ = O.normalize_pixels(s.X)
    return Xn.astype(np.float32).astype(np.float64), cfg


def main():
    X, cfg = data()
    N = X.shape[1]
    ref = O.edaa_fit(X, P, T=cfg["T"], K1=cfg["K1"], K2=cfg["K2"], gamma=1.0, seed=0)
    B0 = O.init_B_from_seed(0, N, P)
    dl, da, db = [], [], []
    for k in range(N_ORDERS):
        perm = np.random.default_rng(k).permutation(N)
        inv = np.argsort(perm)
        r = O.edaa_fit(X[:, perm], P, T=cfg["T"], K1=cfg["K1"], K2=cfg["K2"], seed=0, B0=B0[perm],
                       eta=(ref["eta1"], ref["eta2"]), dtype=np.float32)
        dl.append(np.abs(r["loss"] - ref["loss"]) / ref["loss"])
        da.append(np.max(np.abs(r["A"].astype(np.float64)[:, inv] - ref["A"])))
        db.append(N * np.max(np.abs(r["B"].astype(np.float64)[inv] - ref["B"])))
        print(f"order {k}: loss max {dl[-1].max():.3e}, A {da[-1]:.3e}, N B {db[-1]:.3e}", flush=True)
    dl = np.array(dl)
    np.savez_compressed(os.path.join(HERE, "jasper_full_ref.npz"), loss=ref["loss"], A=ref["A"].astype(np.float32),
                        NB=(N * ref["B"]).astype(np.float32),
                        f32_loss_max=dl.max(axis=0), f32_loss_med=np.median(dl, axis=0),
                        f32_A_max=np.max(da), f32_NB_max=np.max(db))


if __name__ == "__main__":
    main()
