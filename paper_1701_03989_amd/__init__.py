"""Adaptive s-step conjugate gradient (arXiv 1701.03989) on AMD MI355X.

The solver and its per-stage kernels live in ``libsscg.so`` (hand-written HIP
for gfx950 behind the C ABI declared in ``include/sscg.h``).  ``sscg`` is the
thin ctypes binding; ``problems`` holds the seeded synthetic input generators.
Importing this package loads nothing; ``sscg`` loads the library on first use
and raises if it has not been built.
"""
