"""Oracle: a plain, slow, FP64 CPU implementation of the odd-even Wilson-clover path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, calls or links
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code, constants or helpers with the HIP library; the
two meet only through the seeded inputs of ``paper_2407_08092_amd.synth``.

Modules
  dirac     Wilson-clover D (Sect. 2.3), odd-even split (Sect. 2.4.5, eq. 1),
            Schur complement (eq. 3), prepare / reconstruct (eq. 2), dense and
            sparse assemblies, explicit adjoint.
  solvers   Richardson (Alg. 4), power iteration for |lambda_max| (Sect. 2.4.4),
            restarted GMRES (Alg. 2), flexible variant with a Richardson
            preconditioner.
  gradient  torch-CPU complex128 re-expression of L = |D_S(U) phi|^2 for an
            autograd gradient, su(3) projection, central finite differences.

Every function is pinned by the CPU tests (tests/test_oracle_*.py) against
closed forms, invariants and brute force; see the pin list in each docstring.
"""
