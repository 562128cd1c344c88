"""CPU oracle of classical and s-step CG (arXiv 1701.03989), FP64 and exact.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference the HIP
path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the product package
(``paper_1701_03989_amd``) never imports, links or runs anything here, and this
package imports nothing from it.

Modules
  arith     FP64 with correctly rounded reductions, and exact rationals
  sstep     Algorithms 2, 3, 4 (fixed, scheduled and adaptive s-step CG)
  cg        Algorithm 1 (classical CG)
  kappa     condition numbers of sub-Gram matrices (Jacobi eigenvalues)
  spectral  Chebyshev interval: Gershgorin bound and Lanczos Ritz values
  native    loader of crsum.c, the correctly rounded summation helper

Parity status: every function is pinned by a test in tests/test_oracle_*.py
(exact-arithmetic identities, closed forms, library cross-checks, the paper's
error bounds); the s_k schedules of the paper's own matrices cannot be pinned
(those matrices are not available) -- see the design notes.
"""
