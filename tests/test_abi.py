"""CPU checks of the C ABI: the built library loads, exports every function
include/edaa.h declares, its host-only logic (defaults, selection, argument
checks) behaves as documented.  No GPU computation is started here."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

from oracle import edaa as O
from paper_2209_11002_amd import _lib as L_

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "edaa.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(edaa_[a-z_A-Z0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return L_.load()


def test_header_declarations_are_bound():
    names = _declared_functions()
    assert len(names) >= 14
    assert set(names) == set(L_.SIGNATURES), set(names) ^ set(L_.SIGNATURES)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = os.popen(f"nm -D --defined-only {L_.LIB_PATH}").read()
    exported = set(re.findall(r" T (edaa_\w+)", out))
    assert set(_declared_functions()) <= exported


def test_struct_layouts_match_header():
    # edaa_params: 3 ints, 5 doubles, 6 ints (with natural alignment)
    assert ctypes.sizeof(L_.EdaaParams) == 3 * 4 + 4 + 5 * 8 + 6 * 4
    assert L_.EdaaParams.gamma.offset == 16
    assert ctypes.sizeof(L_.EdaaImageDesc) == 8 + 4 * 3 + 4 + 8 + 8 + 8 * 4 + 8


def test_default_params_are_the_papers(lib):
    p = L_.default_params()
    assert (p.T, p.K1, p.K2) == (O.DEFAULT_T, O.DEFAULT_K1, O.DEFAULT_K2)
    assert p.init_scale == O.INIT_SCALE and p.select_threshold == O.SELECT_THRESHOLD
    assert p.gamma in O.GAMMA_SET and p.eta1 == 0.0 and p.eta2 == 0.0
    assert p.x_dtype == L_.EDAA_X_F32 and p.coherence_mode == L_.EDAA_COHERENCE_COSINE and p.flags == 0


def _select(lib, fit, mu, thr=1.05):
    f = np.ascontiguousarray(fit, dtype=np.float64)
    m = np.ascontiguousarray(mu, dtype=np.float64)
    P = ctypes.POINTER(ctypes.c_double)
    return lib.edaa_select(f.ctypes.data_as(P), m.ctypes.data_as(P), len(f), thr)


@pytest.mark.parametrize("fit,mu,thr", [
    ([1.0], [0.5], 1.05),
    ([1.0, 1.05, 1.2], [0.9, 0.1, 0.0], 1.05),
    ([1.0, 1.0500001, 1.2], [0.9, 0.1, 0.0], 1.05),
    ([2.0, 2.0, 2.0], [0.3, 0.3, 0.3], 1.05),
    ([np.nan, 1.0, np.inf], [0.0, 0.4, 0.0], 1.05),
    ([np.nan, np.inf], [0.0, 0.0], 1.05),
    ([1.0, 1.0], [np.nan, 0.7], 1.05),
    ([5.0, 1.0, 1.04], [0.1, 0.5, 0.4], 1.05),
    ([1.0, 1.3, 1.2], [0.9, 0.1, 0.2], 1.25),
])
def test_select_matches_algorithm_2(lib, fit, mu, thr):
    assert _select(lib, fit, mu, thr) == O.select(fit, mu, thr)


def test_select_random_cases(lib):
    rng = np.random.default_rng(0)
    for _ in range(200):
        M = int(rng.integers(1, 12))
        fit = rng.uniform(1.0, 1.2, size=M)
        fit[rng.random(M) < 0.1] = np.inf
        mu = np.round(rng.uniform(0, 1, size=M), 1)      # frequent ties
        assert _select(lib, fit, mu) == O.select(fit, mu)


def test_select_degenerate_arguments(lib):
    assert lib.edaa_select(None, None, 3, 1.05) == -1
    f = np.ones(2)
    P = ctypes.POINTER(ctypes.c_double)
    assert lib.edaa_select(f.ctypes.data_as(P), f.ctypes.data_as(P), 0, 1.05) == -1


def test_null_context_is_rejected(lib):
    p = L_.default_params()
    st = lib.edaa_fit(None, None, 10, 10, 3, ctypes.byref(p), 0, None, None, None, None, None, None, None)
    assert st == L_.EDAA_EINVAL
    assert b"context" in lib.edaa_last_error()
    assert lib.edaa_mirror_step_A(None, None, None, 3, 10, 0.1) == L_.EDAA_EINVAL
    lib.edaa_destroy(None)                      # no-op
    assert lib.edaa_last_launch_count(None) == -1


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device error path")
def test_create_without_device(lib):
    h = ctypes.c_void_p()
    st = lib.edaa_create(ctypes.byref(h), 0, None)
    assert st == L_.EDAA_EDEVICE
    assert lib.edaa_last_error() == b"no HIP device available"
    assert h.value is None


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(L_, "_lib", None)
    monkeypatch.setattr(L_, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        L_.load()
