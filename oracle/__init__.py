"""FP64 CPU oracle for the shifted-Laplace rational-filter (SLRF) eigensolver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the GPU
path: the only common module is ``pencils`` (seeded input generation).

Plain, slow, obviously-correct float64 implementations, each citing the part of
the paper it follows (Wang, Meerbergen, Vandebril, An, Mo, "A shifted Laplace
rational filter for large-scale eigenvalue problems", arXiv:2503.21618):

  poles.py     SLRF pole/weight design (Section 3.1, the rational filter of
               eq. (rational filter) and the delta-weighted least-squares
               problem), separation factor (Definition 3.1), quadrature-rule
               filters on a circle (Section 3.2).
  filter.py    The scalar filter Phi(lambda) (Section 3, the rational function
               filter) and filter application U = sum_j 2 Re(w_j Y_j) with
               exact direct solves (Algorithm 1, steps "Solve"/"Compute U";
               the conjugate-pair reduction of Section 3).
  krylov.py    Right-preconditioned BiCGStab (van der Vorst 1992, the inner
               solver of Sections 2 and 4.2) and COCG (van der Vorst and
               Melissen 1990) for the shifted systems; preconditioners of the
               shifted operator: point Jacobi, ILU(0), 3x3 node-block Jacobi
               and the multicolour symmetric Gauss-Seidel / SOR (greedy
               colouring of the node graph).
  inertia.py   Eigenvalue counts below gamma by Sylvester's law of inertia.
  dense.py     All eigenpairs of a tiny pencil (Cholesky reduction).
  subspace.py  Algorithm 1 (rational filter subspace iteration) with exact
               solves, B-orthonormalisation, Rayleigh-Ritz and the relative
               residual of Algorithm 1 / Section 4.2.
  banded.py    Banded Cholesky of A and block-elimination inertia counts for
               the large structured-grid pencils.
  shift_invert.py  Eigenpairs in (0, gamma] of the large pencils by
               shift-invert subspace iteration (Algorithm 1 with the filter
               1/lambda, the Ericsson-Ruhe method of Section 1).

Parity status: every function is pinned by tests under ``tests/test_oracle_*``
against closed forms, invariants or brute force, except the numerical pole
values of the SLRF optimiser, which the paper never prints (its pole figures
are not reproduced in the text): those are "parity unpinned" and are checked
only through the invariants the paper states (filter real on the real axis,
scale invariance in gamma, separation factor growing with N and falling with
alpha, sharper slope for beta = 0.01).
"""
