"""Writes hundred_fp32_envelope.txt: for each run of the 100-run ensemble of
tests/test_gpu_ensemble.py (L=40, N=333, p=3 small scene, seed 90; run m has
seed m and gamma drawn from the paper's set S by numpy's default_rng(2209);
T = 10, K1 = K2 = 5), how far plain float32 arithmetic lands from the float64
oracle: the oracle's own steps run in float32 on the same data with the pixels
in 8 different orders (a permutation of the pixels is an exact symmetry of
Algorithm 1, so every order is an equally valid float32 evaluation and the
float64 result does not depend on it).  Columns: run, gamma, then the median
and the maximum over the 8 orders of (a) the largest relative deviation of the
objective trace, (b) the relative deviation of the l1 fit, (c) the absolute
deviation of the coherence.  Calls only oracle/ and the seeded generator.

    python tests/golden/make_hundred_envelope.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import edaa as O  # noqa: E402
from paper_2209_11002_amd import synth  # noqa: E402

N_ORDERS = 8


def case():
    s = synth.small_case(seed=90, L=40, N=333, p=3)
    Xn, _ = O.normalize_pixels(s.X)
    X = Xn.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(2209)
    gammas = [float(g) for g in rng.choice(O.GAMMA_SET, size=100)]
    return X, gammas


def main():
    X, gammas = case()
    N = X.shape[1]
    rows = []
    for m in range(100):
        ref = O.edaa_fit(X, 3, T=10, gamma=gammas[m], seed=m)
        fit_ref, mu_ref = O.fit_l1(X, ref["E"], ref["A"]), O.coherence(ref["E"])
        B0 = O.init_B_from_seed(m, N, 3)
        dl, df, dm = [], [], []
        for k in range(N_ORDERS):
            perm = np.random.default_rng(k).permutation(N)
            Xp = X[:, perm]
            r = O.edaa_fit(Xp, 3, T=10, seed=m, B0=B0[perm], eta=(ref["eta1"], ref["eta2"]), dtype=np.float32)
            dl.append(np.max(np.abs(r["loss"] - ref["loss"]) / ref["loss"]))
            E, A = r["E"].astype(np.float64), r["A"].astype(np.float64)
            df.append(abs(O.fit_l1(Xp, E, A) - fit_ref) / fit_ref)
            dm.append(abs(O.coherence(E) - mu_ref))
        rows.append([m, gammas[m], np.median(dl), np.max(dl), np.median(df), np.max(df), np.median(dm), np.max(dm)])
    header = ("float32 arithmetic vs the float64 oracle, 100-run ensemble (L=40, N=333, p=3, T=10), "
              f"{N_ORDERS} pixel orders; written by make_hundred_envelope.py\n"
              "run gamma loss_med loss_max fit_med fit_max mu_med mu_max")
    np.savetxt(os.path.join(HERE, "hundred_fp32_envelope.txt"), np.array(rows),
               fmt=["%d", "%.6g"] + ["%.4e"] * 6, header=header)


if __name__ == "__main__":
    main()
