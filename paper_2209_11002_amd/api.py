"""Python binding of the EDAA library (arXiv 2209.11002) for PyTorch-ROCm.

Argument marshalling only: every step of the method runs in the HIP kernels
of libedaa.so.  PyTorch provides device memory (tensors) and the stream (the
current torch stream of the tensor's device).  Layouts follow include/edaa.h:
X [L][N], A [p][N], B [N][p], E [L][p]; ensembles stack runs first.
"""
import ctypes
from ctypes import byref, c_double, c_int, c_uint64

import numpy as np
import torch

from . import _lib as L_
from ._lib import EdaaError, check  # noqa: F401  (re-exported)

_contexts = {}


def _ctx(device):
    """One library context per (device, torch stream)."""
    dev = torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(idx)
    key = (idx, stream.cuda_stream)
    c = _contexts.get(key)
    if c is None:
        lib = L_.load()
        h = ctypes.c_void_p()
        check(lib.edaa_create(byref(h), idx, ctypes.c_void_p(stream.cuda_stream)))
        c = h
        _contexts[key] = c
    return c


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _x_dtype(X):
    if X.dtype == torch.float32:
        return L_.EDAA_X_F32
    if X.dtype == torch.bfloat16:
        return L_.EDAA_X_BF16
    raise TypeError(f"X must be float32 or bfloat16, got {X.dtype}")


def _check_x(X):
    if not (isinstance(X, torch.Tensor) and X.dim() == 2 and X.is_contiguous()):
        raise ValueError("X must be a contiguous 2-D [L, N] tensor")
    _x_dtype(X)
    if not X.is_cuda:
        raise ValueError("X must be a GPU tensor")
    return X.shape[0], X.shape[1]


def _check_f32(name, t, shape, device):
    """t must be a contiguous float32 tensor of exactly `shape` on `device`
    (the kernels read and write it through a raw pointer with that layout)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")


def _check_dense_operands(X, A, B):
    """Operands of the objective and its gradients: X [L, N] float32 (these
    kernels read float32 X only), A [p, N] and B [N, p] float32, all
    contiguous and on X's device."""
    if not (isinstance(X, torch.Tensor) and X.dim() == 2 and X.is_contiguous()):
        raise ValueError("X must be a contiguous 2-D [L, N] tensor")
    if X.dtype != torch.float32:
        raise TypeError(f"X must be float32 for the objective and its gradients, got {X.dtype}")
    Lb, N = X.shape
    if not (isinstance(A, torch.Tensor) and A.dim() == 2):
        raise ValueError("A must be a 2-D [p, N] tensor")
    p = A.shape[0]
    _check_f32("A", A, (p, N), X.device)
    _check_f32("B", B, (N, p), X.device)
    if not X.is_cuda:
        raise ValueError("X must be a GPU tensor")
    return Lb, N, p


def _params(T, K1, K2, gamma, eta, init_scale, threshold, x_dtype, coherence, graph, time_passes=False,
            runs_per_chunk=0, pixel_groups=0, bf16_widen=False, f32_mfma=False):
    P = L_.default_params()
    P.runs_per_chunk, P.pixel_groups = int(runs_per_chunk), int(pixel_groups)
    P.T, P.K1, P.K2 = int(T), int(K1), int(K2)
    P.gamma = float(gamma)
    if eta is not None:
        P.eta1, P.eta2 = float(eta[0]), float(eta[1])
    P.init_scale = float(init_scale)
    P.select_threshold = float(threshold)
    P.x_dtype = x_dtype
    P.coherence_mode = {"cosine": L_.EDAA_COHERENCE_COSINE, "raw": L_.EDAA_COHERENCE_RAW}[coherence]
    P.flags = (L_.EDAA_FLAG_GRAPH if graph else 0) | (L_.EDAA_FLAG_TIME_PASSES if time_passes else 0)
    if bf16_widen:
        P.flags |= L_.EDAA_FLAG_BF16_WIDEN
    if f32_mfma:
        P.flags |= L_.EDAA_FLAG_F32_MFMA
    return P


def normalize_pixels(X, out_dtype=torch.float32, count_zero=False):
    """eq. normalization on the GPU: every pixel (column) of X [L, N] float32
    divided by its l2 norm; returns a new tensor of dtype out_dtype
    (float32 or bfloat16) and, with count_zero, the number of zero pixels."""
    Lb, N = _check_x(X)
    if X.dtype != torch.float32:
        raise TypeError("normalize_pixels takes float32 input")
    out = torch.empty((Lb, N), dtype=out_dtype, device=X.device)
    od = L_.EDAA_X_BF16 if out_dtype == torch.bfloat16 else L_.EDAA_X_F32
    nz = c_int(0)
    check(L_.load().edaa_normalize_pixels(_ctx(X.device), _ptr(X), _ptr(out), Lb, N, od,
                                          byref(nz) if count_zero else None))
    return (out, nz.value) if count_zero else out


def fit(X, p, T=100, K1=5, K2=5, gamma=1.0, seed=0, A0=None, B0=None, eta=None,
        init_scale=0.1, graph=False, time_passes=False, pixel_groups=0, out=None, bf16_widen=False,
        f32_mfma=False):
    """One run of Algorithm 1 on l2-normalised X [L, N] (float32 or bfloat16,
    on the GPU).  Returns a dict: A [p, N], B [N, p], E [L, p] (tensors),
    loss (numpy, T+1), eta1, eta2.  out: optional dict of preallocated
    A [p, N], B [N, p], E [L, p] float32 tensors to write into.
    bf16_widen: bf16 X runs the passes on the float32 matrix cores
    (EDAA_FLAG_BF16_WIDEN) instead of the bf16 ones.  f32_mfma: float32 X
    runs the B-pass on the float32 matrix cores (EDAA_FLAG_F32_MFMA) instead
    of the bf16 ones with three-term operands."""
    Lb, N = _check_x(X)
    dev = X.device
    if out is None:
        A = torch.empty((p, N), dtype=torch.float32, device=dev)
        B = torch.empty((N, p), dtype=torch.float32, device=dev)
        E = torch.empty((Lb, p), dtype=torch.float32, device=dev)
    else:
        for k, shp in (("A", (p, N)), ("B", (N, p)), ("E", (Lb, p))):
            if k not in out:
                raise ValueError(f"out must hold '{k}'")
            _check_f32(f"out['{k}']", out[k], shp, dev)
        A, B, E = out["A"], out["B"], out["E"]
    for name, t, shp in (("A0", A0, (p, N)), ("B0", B0, (N, p))):
        if t is not None:
            _check_f32(name, t, shp, dev)
    trace = (c_double * (T + 1))()
    eta_out = (c_double * 2)()
    P = _params(T, K1, K2, gamma, eta, init_scale, 1.05, _x_dtype(X), "cosine", graph, time_passes,
                pixel_groups=pixel_groups, bf16_widen=bf16_widen, f32_mfma=f32_mfma)
    lib = L_.load()
    st = lib.edaa_fit(_ctx(dev), _ptr(X), Lb, N, p, byref(P), c_uint64(seed), _ptr(A0), _ptr(B0),
                      _ptr(A), _ptr(B), _ptr(E), trace, eta_out)
    if st not in (L_.EDAA_OK, L_.EDAA_ENUMERIC):
        check(st)
    return dict(A=A, B=B, E=E, loss=np.array(trace[:]), eta1=eta_out[0], eta2=eta_out[1],
                status=st, launches=lib.edaa_last_launch_count(_ctx(dev)))


def fit_noalloc(X, p, out, T=100, K1=5, K2=5, gamma=1.0, seed=0, A0=None, B0=None, eta=None, init_scale=0.1):
    """fit() through the entry point that allocates nothing (edaa_fit_noalloc):
    every output is a preallocated GPU tensor in `out` -- A [p, N], B [N, p],
    E [L, p] float32, loss [T+1] and eta [2] float64 -- and nothing is
    synchronised or copied to the host.  Returns `out`."""
    Lb, N = _check_x(X)
    dev = X.device
    for k, shp in (("A", (p, N)), ("B", (N, p)), ("E", (Lb, p))):
        if k not in out:
            raise ValueError(f"out must hold '{k}'")
        _check_f32(f"out['{k}']", out[k], shp, dev)
    for k, n in (("loss", T + 1), ("eta", 2)):
        t = out.get(k)
        if t is not None and not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_contiguous()
                                  and tuple(t.shape) == (n,) and t.device == dev):
            raise ValueError(f"out['{k}'] must be a contiguous float64 tensor of shape ({n},) on {dev}")
    for name, t, shp in (("A0", A0, (p, N)), ("B0", B0, (N, p))):
        if t is not None:
            _check_f32(name, t, shp, dev)
    P = _params(T, K1, K2, gamma, eta, init_scale, 1.05, _x_dtype(X), "cosine", False)
    check(L_.load().edaa_fit_noalloc(_ctx(dev), _ptr(X), Lb, N, p, byref(P), c_uint64(seed), _ptr(A0), _ptr(B0),
                                     _ptr(out["A"]), _ptr(out["B"]), _ptr(out["E"]), _ptr(out.get("loss")),
                                     _ptr(out.get("eta"))))
    return out


def abundances(X, E, T=100, K1=5, gamma=1.0, A0=None, eta1=None, graph=False):
    """Abundances for given endmembers E [L, p] (float32, GPU): T outer
    iterations of K1 entropic A-steps (eq. update_A with E fixed) on
    l2-normalised X [L, N].  Returns a dict: A [p, N] (tensor), loss (numpy,
    T+1), eta1."""
    Lb, N = _check_x(X)
    if not (isinstance(E, torch.Tensor) and E.dim() == 2):
        raise ValueError("E must be a 2-D [L, p] tensor")
    p = E.shape[1]
    _check_f32("E", E, (Lb, p), X.device)
    if A0 is not None:
        _check_f32("A0", A0, (p, N), X.device)
    A = torch.empty((p, N), dtype=torch.float32, device=X.device)
    trace = (c_double * (T + 1))()
    eta_out = (c_double * 2)()
    P = _params(T, K1, 0, gamma, None if eta1 is None else (eta1, 1.0), 0.1, 1.05, _x_dtype(X), "cosine", graph)
    st = L_.load().edaa_abundances(_ctx(X.device), _ptr(X), Lb, N, p, byref(P), _ptr(E), _ptr(A0), _ptr(A),
                                   trace, eta_out)
    if st not in (L_.EDAA_OK, L_.EDAA_ENUMERIC):
        check(st)
    return dict(A=A, loss=np.array(trace[:]), eta1=eta_out[0], status=st)


def ensemble(X, p, seeds, gammas, T=100, K1=5, K2=5, coherence="cosine", threshold=1.05,
             init_scale=0.1, graph=False, out=None, time_passes=False, runs_per_chunk=0, pixel_groups=0,
             bf16_widen=False, f32_mfma=False):
    """M runs of Algorithm 1 advanced together plus Algorithm 2.  Returns a
    dict with A [M, p, N], B [M, N, p], E [M, L, p] (tensors), loss [M, T+1],
    fit [M], mu [M], status [M] (numpy) and the selected run index.
    runs_per_chunk / pixel_groups pin the launch shape (0: tuned or
    default; see plan()); bf16_widen, f32_mfma as for fit()."""
    Lb, N = _check_x(X)
    M = len(seeds)
    if len(gammas) != M:
        raise ValueError("seeds and gammas must have the same length")
    dev = X.device
    if out is None:
        out = dict(A=torch.empty((M, p, N), dtype=torch.float32, device=dev),
                   B=torch.empty((M, N, p), dtype=torch.float32, device=dev),
                   E=torch.empty((M, Lb, p), dtype=torch.float32, device=dev))
    else:
        for k, shp in (("A", (M, p, N)), ("B", (M, N, p)), ("E", (M, Lb, p))):
            if k not in out:
                raise ValueError(f"out must hold '{k}'")
            _check_f32(f"out['{k}']", out[k], shp, dev)
    sd = (c_uint64 * M)(*[int(s) for s in seeds])
    gm = (c_double * M)(*[float(g) for g in gammas])
    loss = np.zeros((M, T + 1))
    fitv = np.zeros(M)
    mu = np.zeros(M)
    status = np.zeros(M, dtype=np.int32)
    sel = c_int(-1)
    P = _params(T, K1, K2, 1.0, None, init_scale, threshold, _x_dtype(X), coherence, graph, time_passes,
                runs_per_chunk, pixel_groups, bf16_widen, f32_mfma)
    lib = L_.load()
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(c_double))  # noqa: E731
    st = lib.edaa_ensemble(_ctx(dev), _ptr(X), Lb, N, p, byref(P), M, sd, gm,
                           _ptr(out["A"]), _ptr(out["B"]), _ptr(out["E"]),
                           dp(loss), dp(fitv), dp(mu), status.ctypes.data_as(ctypes.POINTER(c_int)), byref(sel))
    if st not in (L_.EDAA_OK, L_.EDAA_ENUMERIC):
        check(st)
    return dict(A=out["A"], B=out["B"], E=out["E"], loss=loss, fit=fitv, mu=mu, status=status,
                selected=sel.value, launches=lib.edaa_last_launch_count(_ctx(dev)))


def _ragged_descs(images, ps, seeds, gammas, T, pixel_groups=None):
    """Descriptors, output tensors and host traces of a ragged batch."""
    n = len(images)
    if n < 1 or len(ps) != n or len(seeds) != n or len(gammas) != n:
        raise ValueError("images, ps, seeds and gammas must be non-empty and of equal length")
    if pixel_groups is not None and len(pixel_groups) != n:
        raise ValueError("pixel_groups must have one entry per image")
    dt, dev0 = images[0].dtype, images[0].device
    for k, X in enumerate(images):
        if not isinstance(X, torch.Tensor):
            raise TypeError(f"image {k} must be a tensor")
        if X.dtype != dt or X.device != dev0:
            raise ValueError(f"image {k}: every image must share the dtype and device of image 0 "
                             f"({dt}, {dev0}), got ({X.dtype}, {X.device})")
    descs = (L_.EdaaImageDesc * n)()
    outs, traces = [], []
    for k, X in enumerate(images):
        Lb, N = _check_x(X)
        p = int(ps[k])
        o = dict(A=torch.empty((p, N), dtype=torch.float32, device=X.device),
                 B=torch.empty((N, p), dtype=torch.float32, device=X.device),
                 E=torch.empty((Lb, p), dtype=torch.float32, device=X.device))
        tr = (c_double * (T + 1))()
        d = descs[k]
        d.X, d.L, d.N, d.p = X.data_ptr(), Lb, N, p
        d.seed, d.gamma = int(seeds[k]), float(gammas[k])
        d.A, d.B, d.E = o["A"].data_ptr(), o["B"].data_ptr(), o["E"].data_ptr()
        d.loss_trace = tr
        d.pixel_groups = int(pixel_groups[k]) if pixel_groups is not None else 0
        outs.append(o)
        traces.append(tr)
    return descs, outs, traces


def fit_ragged(images, ps, seeds, gammas, T=100, K1=5, K2=5, init_scale=0.1, graph=False, grouped=False,
               tiles_per_item=0, pixel_groups=None):
    """Independent runs of Algorithm 1 on images of different (L, N, p), all
    advanced together: images with p <= 9 in one persistent launch (work
    items of `tiles_per_item` 64-pixel tiles, 0 for the tuned or default
    size), the others (every image with grouped=True) one launch per kernel
    and group of equal p.  images: list of l2-normalised [L_k, N_k] GPU
    tensors (one dtype); pixel_groups: optional per-image item counts.
    Returns a list of dicts with A, B, E (tensors), loss (numpy) and the
    pixel_groups used (a single fit with that many pixel groups gives the
    same results)."""
    descs, outs, traces = _ragged_descs(images, ps, seeds, gammas, T, pixel_groups)
    P = _params(T, K1, K2, 1.0, None, init_scale, 1.05, _x_dtype(images[0]), "cosine", graph)
    P.tiles_per_item = int(tiles_per_item)
    if grouped:
        P.flags |= L_.EDAA_FLAG_RAGGED_GROUPED
    check(L_.load().edaa_fit_ragged(_ctx(images[0].device), len(images), descs, byref(P)))
    for k, (o, tr) in enumerate(zip(outs, traces)):
        o["loss"] = np.array(tr[:])
        o["pixel_groups"] = descs[k].pixel_groups
    return outs


def autotune(X, p, M=1, K1=5, K2=5, gamma=1.0):
    """Time the candidate launch shapes of an M-run problem on X (see
    edaa_autotune) and record the fastest for its class.  Returns the plan
    dict (as plan()) and the microseconds per outer iteration."""
    Lb, N = _check_x(X)
    P = _params(1, K1, K2, gamma, None, 0.1, 1.05, _x_dtype(X), "cosine", False)
    best = L_.EdaaLaunchPlan()
    us = c_double(0.0)
    check(L_.load().edaa_autotune(_ctx(X.device), _ptr(X), Lb, N, int(p), int(M), byref(P), byref(best), byref(us)))
    return dict(runs_per_chunk=best.runs_per_chunk, chunks=best.chunks, pixel_groups=best.pixel_groups,
                double_buffer=best.double_buffer, source="tuned", bf16_passes=best.bf16_passes), us.value


def autotune_ragged(images, ps, seeds, gammas, K1=5, K2=5):
    """Time the persistent kernel's work-item sizes on a ragged batch (see
    edaa_autotune_ragged) and record the fastest for its class.  Returns
    (tiles per item, microseconds per outer iteration)."""
    descs, _, _ = _ragged_descs(images, ps, seeds, gammas, 1)
    P = _params(1, K1, K2, 1.0, None, 0.1, 1.05, _x_dtype(images[0]), "cosine", False)
    tpi = c_int(0)
    us = c_double(0.0)
    check(L_.load().edaa_autotune_ragged(_ctx(images[0].device), len(images), descs, byref(P), byref(tpi),
                                         byref(us)))
    return tpi.value, us.value


def plan(L, N, p, M=1, runs_per_chunk=0, pixel_groups=0, x_dtype=torch.float32, bf16_widen=False,
         f32_mfma=False):
    """Launch shape that fit (M = 1) or ensemble (M runs) would use: a dict
    with runs_per_chunk, chunks, pixel_groups, double_buffer, source
    ('default', 'tuned' or 'requested') and bf16_passes (bit 0: the B-pass,
    bit 1: the A-pass on the bf16 matrix cores).  Host only."""
    P = _params(1, 1, 1, 1.0, None, 0.1, 1.05, L_.EDAA_X_BF16 if x_dtype == torch.bfloat16 else L_.EDAA_X_F32,
                "cosine", False, runs_per_chunk=runs_per_chunk, pixel_groups=pixel_groups, bf16_widen=bf16_widen,
                f32_mfma=f32_mfma)
    out = L_.EdaaLaunchPlan()
    check(L_.load().edaa_plan(int(L), int(N), int(p), int(M), byref(P), byref(out)))
    return dict(runs_per_chunk=out.runs_per_chunk, chunks=out.chunks, pixel_groups=out.pixel_groups,
                double_buffer=out.double_buffer, bf16_passes=out.bf16_passes,
                source={L_.EDAA_PLAN_DEFAULT: "default", L_.EDAA_PLAN_TUNED: "tuned",
                        L_.EDAA_PLAN_REQUESTED: "requested"}[out.source])


def set_graph_cache(device, n):
    """Capacity of the captured-graph cache of this device's current-stream
    context (default 16)."""
    check(L_.load().edaa_set_graph_cache(_ctx(device), int(n)))


def pass_times(device, kind):
    """(launch count, summed milliseconds) of the A-pass (kind 0), B-pass (1)
    or closing pass (2) kernels of the last fit/ensemble call made with
    time_passes=True on this device's current stream."""
    n = c_int(0)
    ms = c_double(0.0)
    check(L_.load().edaa_pass_times(_ctx(device), int(kind), byref(n), byref(ms)))
    return n.value, ms.value


def loss_fwd(X, A, B):
    """1/2 ||X - X B A||_F^2 as a 0-d float32 GPU tensor."""
    Lb, N, p = _check_dense_operands(X, A, B)
    out = torch.empty((), dtype=torch.float32, device=X.device)
    check(L_.load().edaa_loss_fwd(_ctx(X.device), _ptr(X), _ptr(A), _ptr(B), Lb, N, p, _ptr(out)))
    return out


def loss_bwd(X, A, B, grad_out):
    """(dA, dB) of grad_out * 1/2 ||X - X B A||^2; grad_out is a 0-d GPU tensor."""
    Lb, N, p = _check_dense_operands(X, A, B)
    gA = torch.empty_like(A)
    gB = torch.empty_like(B)
    go = grad_out.detach().to(device=X.device, dtype=torch.float32).reshape(()).contiguous()
    check(L_.load().edaa_loss_bwd(_ctx(X.device), _ptr(X), _ptr(A), _ptr(B), Lb, N, p, _ptr(go),
                                  _ptr(gA), _ptr(gB)))
    return gA, gB


def mirror_step_A(A, gA, eta):
    """In place: every column of A [p, N] <- softmax(log a - eta gA)."""
    if not (isinstance(A, torch.Tensor) and A.dim() == 2):
        raise ValueError("A must be a 2-D [p, N] tensor")
    p, N = A.shape
    _check_f32("A", A, (p, N), A.device)
    _check_f32("gA", gA, (p, N), A.device)
    if not A.is_cuda:
        raise ValueError("A must be a GPU tensor")
    check(L_.load().edaa_mirror_step_A(_ctx(A.device), _ptr(A), _ptr(gA), p, N, float(eta)))
    return A


def mirror_step_B(B, gB, eta):
    """In place: every column of B [N, p] <- softmax over N of (log b - eta gB)."""
    if not (isinstance(B, torch.Tensor) and B.dim() == 2):
        raise ValueError("B must be a 2-D [N, p] tensor")
    N, p = B.shape
    _check_f32("B", B, (N, p), B.device)
    _check_f32("gB", gB, (N, p), B.device)
    if not B.is_cuda:
        raise ValueError("B must be a GPU tensor")
    check(L_.load().edaa_mirror_step_B(_ctx(B.device), _ptr(B), _ptr(gB), N, p, float(eta)))
    return B


class ReconLoss(torch.autograd.Function):
    """f(A, B) = 1/2 ||X - X B A||_F^2 with the library's hand-written backward
    (dA = (XB)^T (XBA - X), dB = X^T (XBA - X) A^T).  X carries no gradient."""

    @staticmethod
    def forward(ctx, X, A, B):
        A = A.contiguous()
        B = B.contiguous()
        ctx.save_for_backward(X, A, B)
        return loss_fwd(X, A, B)

    @staticmethod
    def backward(ctx, grad_out):
        X, A, B = ctx.saved_tensors
        gA, gB = loss_bwd(X, A, B, grad_out)
        return None, gA, gB


def select(fit, mu, threshold=1.05):
    """Algorithm 2 selection via the library's host function edaa_select."""
    f = np.ascontiguousarray(fit, dtype=np.float64)
    m = np.ascontiguousarray(mu, dtype=np.float64)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(c_double))  # noqa: E731
    return int(L_.load().edaa_select(dp(f), dp(m), len(f), float(threshold)))
