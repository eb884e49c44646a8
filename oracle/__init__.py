"""Float64 CPU oracle for EDAA (arXiv 2209.11002).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
HIP library is checked against.  Only tests/, the smoke check in
__graft_entry__ and the CPU-baseline leg of bench.py may import it.  It shares
no code with the library: neither imports the other, and the only thing both
sides consume is the seeded synthetic input generator, which holds none of the
method's arithmetic.

Functions whose result is pinned only by the oracle itself ("parity
unpinned"): the long-horizon trajectory of edaa_fit on mixed data, and the
selected run when fit/coherence margins fall below float32 rounding.
"""
from . import philox, edaa  # noqa: F401
