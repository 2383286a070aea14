"""Plain FP64 CPU oracle for the BDF2 all-at-once Riesz fractional diffusion solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the GPU smoke check and the benchmark's
CPU-baseline leg may import this package.  The product library never calls it, and it
shares no code, tables or constants with the HIP path.

Everything here is numpy / scipy in float64 (complex128), written to be checked by
eye against the paper (Gu, Zhao, Zhao, Carpentieri, Huang, "A note on parallel
preconditioning for the all-at-once solution of Riesz fractional diffusion
equations", arXiv:2003.07020).  Each function cites the section / equation it
follows.  Where the printed text is garbled or silent, the reading taken is stated
in the function's docstring.

Modules
  weights    fractional centred-difference weights, eq. (2.4), Lemma 2.1
  allatonce  Toeplitz block, BDF2 scheme eq. (1.2), all-at-once system eq. (2.10)-(2.12)
  precond    alpha-circulant preconditioner, Section 3.1 and 3.2, tau/DST variant eq. (3.9)
  krylov     flexible GMRES with right preconditioning (Section 4 solver settings)
  twod       2D model eq. (4.1), Kronecker-sum Jacobian eq. (4.2), tau approximation eq. (4.5)
  mlp        the learned initial-guess network (forward, chain-rule gradients, Adam, sine basis)

Parity status: every function is pinned by a test in tests/test_oracle_*.py against a
closed form, an invariant, a brute-force computation or a value printed in the paper.
"""
from . import weights, allatonce, precond, krylov, twod, mlp  # noqa: F401
