"""Synthetic ablation of EDAA's hyper-parameters, scored with the paper's metrics.

The paper's ablation study (Section "Ablation study", and the detailed
tables of the supplementary material) varies, with the model selection of
Algorithm 2 on top:
  (a) the inner iterations K1 = K2 = K at a fixed budget of 1000 updates,
      T = 500 / K outer iterations (K in {1, 5, 10, 20, 50}), with M = 100 runs;
  (b) the outer iterations T with K1 = K2 = 5;
  (c) the number of runs M with K1 = K2 = 5 and T = 100,
and scores the selected model by the global abundance RMSE (eq. RMSE) and
the endmember spectral angle distance SAD (eq. SAD) against the ground
truth.  The paper's data sets are not available, so the scenes here are
synthetic analogues with known endmembers and abundances; each run draws
its step multiplier gamma uniformly from the set S of the step-size rule
(Section "Implementation details"), as the paper does.

The paper does not say how estimated endmembers are paired with the
reference ones before scoring; here they are paired by the assignment of
least total spectral angle (exhaustive over the p! pairings up to p = 8,
the Hungarian method above).

Every EDAA iteration runs in the library's kernels (``api.ensemble``); this
module only draws the run parameters and scores the selected model.
"""
import itertools
import json
import sys
import time

import numpy as np
import torch

from . import api, synth

# The set S of step multipliers gamma (Section "Implementation details").
GAMMA_SET = (0.125, 0.25, 0.5, 1.0, 2.0, 4.0, 8.0)
K_BUDGET = (1, 5, 10, 20, 50)        # (a): T = 500 / K
T_SWEEP = (100, 75, 50)              # (b)
M_SWEEP = (10, 20, 50, 100)          # (c)


def spectral_angles(M_ref, E):
    """Angle in degrees between every reference column i and estimated
    column j (the summand of eq. SAD), as a [p][p] float64 array."""
    M_ref = torch.as_tensor(M_ref, dtype=torch.float64)
    E = torch.as_tensor(E, dtype=torch.float64).to(M_ref.device)
    c = (M_ref.T @ E) / torch.outer(torch.linalg.norm(M_ref, dim=0), torch.linalg.norm(E, dim=0))
    return torch.rad2deg(torch.arccos(torch.clamp(c, -1.0, 1.0))).cpu().numpy()


def match_endmembers(M_ref, E):
    """perm with E[:, perm[i]] paired to M_ref[:, i], minimising the total
    spectral angle."""
    ang = spectral_angles(M_ref, E)
    p = ang.shape[0]
    if p <= 8:
        perms = np.array(list(itertools.permutations(range(p))))
        cost = ang[np.arange(p)[None, :], perms].sum(axis=1)
        return [int(v) for v in perms[int(np.argmin(cost))]]
    from scipy.optimize import linear_sum_assignment
    rows, cols = linear_sum_assignment(ang)
    perm = [0] * p
    for r, c in zip(rows, cols):
        perm[int(r)] = int(c)
    return perm


def rmse(A_ref, A):
    """eq. RMSE: 100 sqrt(sum_ij (A_ij - A^_ij)^2 / (p N)), in percent."""
    A_ref = torch.as_tensor(A_ref, dtype=torch.float64)
    A = torch.as_tensor(A, dtype=torch.float64).to(A_ref.device)
    return float(100.0 * torch.sqrt(torch.mean((A_ref - A) ** 2)))


def sad(M_ref, E):
    """eq. SAD: mean over the p endmembers of the spectral angle, in degrees
    (columns paired as given)."""
    return float(np.mean(np.diag(spectral_angles(M_ref, E))))


def normalised_abundances(M_ref, A_ref):
    """The reference abundances restated for l2-normalised pixels: a noise-free
    pixel x = M a normalises to x / ||x|| = sum_j c_j m_j / ||m_j|| with c_j =
    a_j ||m_j|| / ||M a||, a point on the ray of the simplex combination
    a^_j = a_j ||m_j|| / sum_k a_k ||m_k|| of the normalised endmembers.
    Abundances on the simplex fitted to normalised data estimate a^, not a
    (they coincide when the endmembers have equal norms)."""
    M_ref = torch.as_tensor(M_ref, dtype=torch.float64)
    A_ref = torch.as_tensor(A_ref, dtype=torch.float64).to(M_ref.device)
    W = A_ref * torch.linalg.norm(M_ref, dim=0)[:, None]
    return W / W.sum(dim=0, keepdim=True)


def score(M_ref, A_ref, E, A):
    """RMSE and SAD of an estimate (E [L][p], A [p][N]) after pairing its
    endmembers with the reference ones; rmse_normalised scores the same
    abundances against normalised_abundances."""
    perm = match_endmembers(M_ref, E)
    E = torch.as_tensor(E)[:, perm]
    A = torch.as_tensor(A)[perm, :]
    return dict(rmse=rmse(A_ref, A), rmse_normalised=rmse(normalised_abundances(M_ref, A_ref), A),
                sad=sad(M_ref, E), perm=perm)


def draw_runs(M, gamma_seed=0):
    """Seeds 0..M-1 and one gamma per run drawn uniformly from S."""
    rng = np.random.default_rng(gamma_seed)
    return list(range(M)), [float(g) for g in rng.choice(GAMMA_SET, size=M)]


def run_config(X, scene, p, K, T, M, gamma_seed=0, graph=True):
    """One ensemble of M runs (K1 = K2 = K, T outer iterations) on the
    normalised image X (device, [L][N]); returns the selected model's
    scores, its run index and the ensemble's wall time."""
    seeds, gammas = draw_runs(M, gamma_seed)
    torch.cuda.synchronize(X.device)
    t0 = time.perf_counter()
    r = api.ensemble(X, p, seeds, gammas, T=T, K1=K, K2=K, graph=graph)
    torch.cuda.synchronize(X.device)
    dt = time.perf_counter() - t0
    sel = int(r["selected"])
    out = score(scene.M, scene.A, r["E"][sel].double(), r["A"][sel].double())
    out.update(K=K, T=T, M=M, selected=sel, gamma=gammas[sel], seconds=dt,
               loss=float(r["loss"][sel][-1]))
    return out


def sweeps(X, scene, p, k_budget=K_BUDGET, t_sweep=T_SWEEP, m_sweep=M_SWEEP, m_budget=100, k_default=5,
           t_default=100, gamma_seed=0):
    """The three sweeps (a), (b), (c) on one scene; a list of result dicts
    tagged with their sweep."""
    res = []
    for K in k_budget:
        res.append(dict(sweep="a", **run_config(X, scene, p, K, 500 // K, m_budget, gamma_seed)))
    for T in t_sweep:
        res.append(dict(sweep="b", **run_config(X, scene, p, k_default, T, m_budget, gamma_seed)))
    for M in m_sweep:
        res.append(dict(sweep="c", **run_config(X, scene, p, k_default, t_default, M, gamma_seed)))
    return res


SCENES = {
    "samson": synth.samson_like,
    "jasper": synth.jasper_like,
    "urban6": lambda: synth.urban_ensemble(n_seeds=1),
}


def main(argv=None):
    """python -m paper_2209_11002_amd.ablation [scene ...]: one JSON line per
    configuration (scene, sweep, K, T, M, rmse, sad, selected run, seconds)."""
    names = (argv if argv is not None else sys.argv[1:]) or list(SCENES)
    for name in names:
        sc, _ = SCENES[name]()
        p = sc.M.shape[1]
        X = api.normalize_pixels(torch.from_numpy(sc.X).cuda())
        # as in the paper's experiments, EDAA sees the l2-normalised pixels
        # and is scored against the scene's own ground truth (SAD does not
        # depend on the scale of the endmembers); rmse_normalised scores
        # against that ground truth restated for normalised pixels
        for row in sweeps(X, sc, p):
            print(json.dumps(dict(scene=name, **row)), flush=True)


if __name__ == "__main__":
    main()
