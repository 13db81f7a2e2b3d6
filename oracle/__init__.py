"""CPU oracle for the anelastic ADER-DG update with clustered rate-2 LTS.

TEST INFRASTRUCTURE ONLY.  A plain, slow FP64 NumPy implementation of what the
GPU path computes, written from the paper (Breuer & Heinecke, "Next-Generation
Local Time Stepping for the ADER-DG Finite Element Method", arXiv 2202.10313).
Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the product path never does, and it shares no code with the HIP
library (only the seeded input generators in ``synth`` serve both).

It is written in *quadrature form*: volume and face integrals are evaluated at
physical quadrature points and the neighbour's polynomial is evaluated at the
same physical face points through its own reference map.  There are no
precomputed flux matrices, no orientation bookkeeping and no factored
relaxation frequencies; in exact arithmetic this equals the factored modal
kernels of Sec. III (ADER-DG Finite Element Method) (all integrands are polynomials and the rules are exact).

Modules:
  poly     Dubiner orthonormal bases built as exact monomial polynomials
  quad     collapsed Gauss-Legendre rules on the unit tetrahedron / triangle
  mesh     face adjacency and affine geometry
  physics  Jacobians, anelastic coupling, eigenvector-based Riemann solver
  lts      CFL steps, rate-2 clustering, normalisation, lambda search
  solver   time kernel, volume and surface kernels, LTS buffers and schedule,
           point sources, receivers

Parity status per function is recorded in each module header; every function
listed there is pinned by a test in tests/test_oracle_*.py.
"""
from .solver import Oracle  # noqa: F401
