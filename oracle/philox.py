"""Philox4x64-10 counter-based generator, written from its published definition.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this module.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11 (the Philox-4x64 S-box: two 64x64->128
multiplies per round, Weyl key schedule, 10 rounds).

The EDAA paper draws the entries of the initial pixel-weight matrix from
U[0,1] (Section "Implementation details", paragraph "Initialization", eq.
initB0) without naming a generator.  Both sides of this project (this oracle
and the HIP library) implement the same counter-based generator from the
publication above so that the draw is a pure function of (seed, pixel,
column) and can be compared bit for bit:

    block(i, j)  = Philox4x64-10(counter=(i, j // 4, 0, 0), key=(seed, 0))
    r            = block(i, j)[j % 4]                       (a 64-bit word)
    u[i, j]      = (r >> 40) * 2**-24                       (24-bit uniform in [0,1))

The 24-bit mantissa makes u exactly representable in float32, so a float32
device path and this float64 oracle start from identical values.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    cross = (ll >> _S32) + (hl & _LO32) + lh          # < 3 * 2**32, no wrap
    hi = hh + (hl >> _S32) + (cross >> _S32)
    lo = (cross << _S32) | (ll & _LO32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Apply 10 Philox-4x64 rounds.

    ctr: four uint64 arrays (broadcastable), key: two uint64 arrays.
    Returns a tuple of four uint64 arrays.
    """
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
        k0, k1 = (np.asarray(k, dtype=np.uint64) for k in key)
        for rnd in range(10):
            if rnd > 0:                       # Weyl key schedule between rounds
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mulhilo64(M0, c0)
            hi1, lo1 = _mulhilo64(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform_u(seed, N, p):
    """u[i, j] in [0, 1), shape (N, p), float64, per the mapping in the module
    docstring.  Pixel index i runs over the columns of X, j over endmembers."""
    i = np.arange(N, dtype=np.uint64)[:, None]
    j = np.arange(p, dtype=np.uint64)[None, :]
    zero = np.zeros_like(i * j)
    words = philox4x64_10((i + zero, j // np.uint64(4) + zero, zero, zero),
                          (np.uint64(seed) + zero, zero))
    words = np.stack(words, axis=0)                        # (4, N, p)
    sel = (j % np.uint64(4)).astype(np.int64) + np.zeros((N, 1), dtype=np.int64)
    r = np.take_along_axis(words, sel[None, :, :], axis=0)[0]
    return (r >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
