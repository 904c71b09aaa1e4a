"""CPU oracle for the SplitSolve hot path — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct complex128 NumPy/SciPy code.  Only the test-suite, the smoke check
and the benchmark's CPU-baseline leg may import it; the product library never does, and this package
imports nothing from the product library (it shares no code, header, table or helper with it).

Contents (each function cites the passage of the paper it follows):

* ``selfenergy``: lead blocks, plain Sancho-Rubio decimation of the lead's surface Green's function
  (Sec. 3A, the "standard iterative decimation technique"), the independent mode route through the
  lead's quadratic eigenproblem (Sec. 3A, Eq. (bound) with nearest-cell coupling), quadratic residual
  and retardedness checks.
* ``linalg``: dense assembly and brute-force solves, block-Thomas elimination of a block-tridiagonal
  system (the definition of T^{-1} b restricted to the block structure).
* ``transport``: the whole hot path by definition — first/last block columns Q of A^{-1}
  (Sec. 3B, Step 1), G^R corner blocks and psi from a direct solve of T = A - Sigma (Sec. 2B,
  Eq. (negf)/(wf)), the SMW quantities R, z (Sec. 3B, Eq. (x)) and the Caroli transmission.
* ``bands``: open-channel count from the lead band structure (independent physics pin).
* ``observables``: orbital density and bond current from psi and their energy integral (Sec. 2B: the
  charge and current densities follow from c(E) once Eq. (wf) is solved over the (E, k) grid).
* ``warmstart``: Newton's method on the self-energy's fixed-point equation with the Stein correction by
  the Kronecker system or Smith's doubling, and the float64 forward/backward passes and Adam update of
  the multilayer perceptron that predicts the starting iterate.

Parity is pinned for every function here by the ``-m "not gpu"`` tests (closed forms, brute force,
invariants, band counting).  No function is "parity unpinned".
"""
from . import bands, linalg, observables, selfenergy, transport, warmstart  # noqa: F401
