"""MI355X (gfx950) implementation of the hot path of Entropic Descent
Archetypal Analysis (arXiv 2209.11002): HIP kernels behind a C ABI
(include/edaa.h, libedaa.so) with a thin PyTorch binding.

Importing the package loads nothing; `paper_2209_11002_amd.api` loads the
library on first use and raises if it has not been built.
"""
__all__ = ["api", "synth", "build"]
