"""GPU checks of the autograd path: the fused loss, its hand-written backward
(checked against the float64 oracle gradient and against central finite
differences on a 32-pixel crop of the Jasper-Ridge-shaped scene), and the
mirror steps that consume the gradients."""
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


def _simplex(rng, d, n):
    Z = rng.gamma(1.0, 1.0, size=(d, n)) + 1e-3
    return Z / Z.sum(axis=0, keepdims=True)


def _case(L, N, p, seed=0):
    s = synth.small_case(seed=seed, L=L, N=N, p=min(p, 8))
    Xn, _ = O.normalize_pixels(s.X)
    X32 = Xn.astype(np.float32)
    rng = np.random.default_rng(seed)
    A = _simplex(rng, p, N).astype(np.float32)
    B = _simplex(rng, N, p).astype(np.float32)
    return X32, A, B


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _elementwise(a, b, tol=1e-5):
    """Every entry within tol of the gradient's largest entry plus tol of its
    own size (a Frobenius-norm gate alone would let one entry be off by up to
    sqrt(size) times more)."""
    d = np.abs(a - b)
    bound = tol * np.max(np.abs(b)) + tol * np.abs(b)
    worst = float(np.max(d / bound))
    _say(f"element-wise: worst entry at {worst:.3f} of its bound")
    return worst <= 1.0


@gpu
@pytest.mark.parametrize("L,N,p", [(40, 333, 3), (198, 1000, 4), (300, 70, 16)])
def test_loss_and_gradients_vs_oracle(api, L, N, p):
    _say(f"loss/grad L={L} N={N} p={p}")
    X, A, B = _case(L, N, p)
    Xg, Ag, Bg = (torch.from_numpy(a).cuda() for a in (X, A, B))
    X64, A64, B64 = X.astype(np.float64), A.astype(np.float64), B.astype(np.float64)
    f = api.loss_fwd(Xg, Ag, Bg).item()
    assert f == pytest.approx(O.loss(X64, A64, B64), rel=1e-5)
    go = torch.tensor(0.75, device="cuda")
    gA, gB = api.loss_bwd(Xg, Ag, Bg, go)
    gA_ref, gB_ref = 0.75 * O.grad_A(X64, A64, B64), 0.75 * O.grad_B(X64, A64, B64)
    assert _rel(gA.cpu().numpy(), gA_ref) < 1e-5
    assert _rel(gB.cpu().numpy(), gB_ref) < 1e-5
    assert _elementwise(gA.cpu().numpy(), gA_ref)
    assert _elementwise(gB.cpu().numpy(), gB_ref)


@gpu
def test_autograd_function_fd_on_jasper_crop(api):
    """Backward of ReconLoss on the 32-pixel crop (pixels 0..31) of the
    Jasper-Ridge-shaped scene, at uniform init and at a point reached after 10
    outer iterations, against central finite differences of the float64
    objective (exact for a quadratic along one coordinate) over all 256
    entries of A and B."""
    s, _ = synth.jasper_like()
    Xn, _ = O.normalize_pixels(s.X)
    Xc = Xn[:, :32].astype(np.float32)
    X64 = Xc.astype(np.float64)
    p = 4
    r10 = O.edaa_fit(X64, p, T=10, gamma=1.0, seed=0)
    points = [(O.init_A(p, 32), O.init_B_from_seed(0, 32, p)), (r10["A"], r10["B"])]
    for k, (A64, B64) in enumerate(points):
        _say(f"FD crop point {k}")
        A32, B32 = A64.astype(np.float32), B64.astype(np.float32)
        A64, B64 = A32.astype(np.float64), B32.astype(np.float64)
        Xg = torch.from_numpy(Xc).cuda()
        Ag = torch.from_numpy(A32).cuda().requires_grad_(True)
        Bg = torch.from_numpy(B32).cuda().requires_grad_(True)
        loss = api.ReconLoss.apply(Xg, Ag, Bg)
        loss.backward()
        h = 1e-6

        def fd(Z, which):
            G = np.zeros_like(Z)
            for idx in np.ndindex(Z.shape):
                Zp, Zm = Z.copy(), Z.copy()
                Zp[idx] += h
                Zm[idx] -= h
                if which == "A":
                    G[idx] = (O.loss(X64, Zp, B64) - O.loss(X64, Zm, B64)) / (2 * h)
                else:
                    G[idx] = (O.loss(X64, A64, Zp) - O.loss(X64, A64, Zm)) / (2 * h)
            return G

        fdA, fdB = fd(A64, "A"), fd(B64, "B")
        assert _rel(Ag.grad.cpu().numpy(), fdA) < 1e-5
        assert _rel(Bg.grad.cpu().numpy(), fdB) < 1e-5
        assert _rel(Ag.grad.cpu().numpy(), O.grad_A(X64, A64, B64)) < 1e-5
        assert _rel(Bg.grad.cpu().numpy(), O.grad_B(X64, A64, B64)) < 1e-5
        assert _elementwise(Ag.grad.cpu().numpy(), fdA)
        assert _elementwise(Bg.grad.cpu().numpy(), fdB)


@gpu
def test_mirror_steps_vs_oracle(api):
    _say("mirror steps")
    X, A, B = _case(40, 500, 5, seed=3)
    rng = np.random.default_rng(1)
    gA = rng.normal(size=A.shape).astype(np.float32)
    gB = rng.normal(size=B.shape).astype(np.float32) * 50
    Ag, Bg = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    api.mirror_step_A(Ag, torch.from_numpy(gA).cuda(), 0.3)
    api.mirror_step_B(Bg, torch.from_numpy(gB).cuda(), 0.05)
    refA = O.mirror_step(A.astype(np.float64), gA.astype(np.float64), 0.3)
    refB = O.mirror_step(B.astype(np.float64), gB.astype(np.float64), 0.05)
    assert np.max(np.abs(Ag.cpu().numpy() - refA)) < 1e-6
    assert np.max(np.abs(Bg.cpu().numpy() - refB) / refB.max()) < 1e-5


@gpu
def test_modular_path_reproduces_fused_iteration(api):
    """K1 mirror steps on A with ReconLoss gradients, then K2 on B, reproduce
    one outer iteration of the fused path (eq. update_A / eq. update_B)."""
    _say("modular vs fused one outer iteration")
    s = synth.small_case(seed=41, L=30, N=256, p=3)
    Xn, _ = O.normalize_pixels(s.X)
    Xg = torch.from_numpy(Xn.astype(np.float32)).cuda()
    r0 = api.fit(Xg, 3, T=0, seed=4)
    A = r0["A"].clone()
    B = r0["B"].clone()
    e1, e2 = r0["eta1"], r0["eta2"]
    for _ in range(5):
        A.requires_grad_(True)
        loss = api.ReconLoss.apply(Xg, A, B)
        gA, = torch.autograd.grad(loss, A)
        A = api.mirror_step_A(A.detach(), gA, e1)
    for _ in range(5):
        B.requires_grad_(True)
        loss = api.ReconLoss.apply(Xg, A, B)
        gB, = torch.autograd.grad(loss, B)
        B = api.mirror_step_B(B.detach(), gB, e2)
    r1 = api.fit(Xg, 3, T=1, seed=4)
    assert torch.max(torch.abs(A - r1["A"])).item() < 1e-5
    assert 256 * torch.max(torch.abs(B - r1["B"])).item() < 1e-4
