"""Pins of the oracle's counter-based generator (oracle/philox.py).

Philox4x64-10 is checked against NumPy's independent implementation
(numpy.random.Philox), which advances its 256-bit counter by one *before*
producing each block of four words: the block it emits first for counter c is
Philox(c + 1, key).
"""
import numpy as np
import pytest

from oracle.philox import philox4x64_10, uniform_u


def _numpy_block(ctr, key):
    c = np.array(ctr, dtype=np.uint64).copy()
    # numpy pre-increments the counter (with carry); undo that.
    for w in range(4):
        if c[w] != 0:
            c[w] -= np.uint64(1)
            break
        c[w] = np.uint64(0xFFFFFFFFFFFFFFFF)
    bg = np.random.Philox(counter=c, key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((0, 1, 0, 0), (5, 7)),                       # exercises the carry path in numpy
    ((123456789, 3, 0, 0), (42, 0)),
    ((2**64 - 1, 2**63, 17, 2**40), (2**64 - 1, 2**64 - 2)),
    ((9024, 1, 0, 0), (9, 0)),
])
def test_philox_matches_numpy(ctr, key):
    ref = _numpy_block(ctr, key)
    out = philox4x64_10(tuple(np.uint64(c) for c in ctr), tuple(np.uint64(k) for k in key))
    assert [int(x) for x in out] == [int(x) for x in ref]


def test_philox_vectorised_matches_scalar():
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2**63, size=(4, 64), dtype=np.uint64)
    k = rng.integers(0, 2**63, size=(2, 64), dtype=np.uint64)
    vec = philox4x64_10(tuple(c), tuple(k))
    for n in range(0, 64, 7):
        ref = _numpy_block(c[:, n], k[:, n])
        assert [int(v[n]) for v in vec] == [int(x) for x in ref]


def test_uniform_u_layout_and_range():
    N, p, seed = 1000, 6, 3
    U = uniform_u(seed, N, p)
    assert U.shape == (N, p)
    assert np.all(U >= 0.0) and np.all(U < 1.0)
    # 24-bit grid: exactly representable in float32
    assert np.all(U * 2**24 == np.floor(U * 2**24))
    assert np.array_equal(U.astype(np.float32).astype(np.float64), U)
    # element (i, j) is word j % 4 of block (i, j // 4)
    for i, j in [(0, 0), (5, 3), (999, 4), (17, 5)]:
        words = _numpy_block((i, j // 4, 0, 0), (seed, 0))
        assert U[i, j] == float(int(words[j % 4]) >> 40) * 2.0**-24
    # a prefix of pixels does not depend on N; seeds differ
    assert np.array_equal(uniform_u(seed, 10, p), U[:10])
    assert not np.array_equal(uniform_u(seed + 1, N, p), U)
    # crude uniformity
    assert abs(U.mean() - 0.5) < 0.02 and abs(U.var() - 1 / 12) < 0.01
