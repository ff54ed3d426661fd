"""CPU FP64 oracle for the per-interval Jones-chain gain solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test suite, the package smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path.

It is a plain, slow, obviously correct restatement of the paper's method
(Kenyon et al., "Africanus II. QuartiCal", Section 2 and Algorithm 1):

* ``jones``   - Jones matrices, vectorisation, permutation, chain products
                (eq. gvec, eq. jones, eq. jonesconj, eq. permutation,
                eq. joneschain, eq. jonesfactor)
* ``solver``  - model/residual (eq. baselinemodel, eq. baselineresidual),
                Jacobian blocks (eq. g_derivative_di/dd), AllJones JHJ/JHr
                (eq. jhj_entry_simplified, eq. jhr_entry_simplified), the
                parameterised delay case (eq. jhj_case2, eq. jhwr_case2),
                block solve and update (eq. update), Algorithm 1, chains
* ``outputs`` - residual / corrupted model / corrected data (Section 4.4)
* ``dense``   - the explicit augmented Jacobian (eq. jacobian) on tiny
                problems by finite-difference Wirtinger derivatives; used
                only to pin the fast forms above
* ``delay_init`` - Fourier-peak delay initial estimate (Section 4.3)
* ``warmstart`` - interval feature pass and the two-layer MLP (forward,
                backward, Adam) used by the learned warm start

All floating point is FP64 / complex128.  Inputs in complex64 are upcast
exactly.  Flagged samples are selected out (never multiplied by zero), so
non-finite payloads under flags have no effect.
"""
from . import jones, solver, outputs, dense, delay_init, warmstart  # noqa: F401
