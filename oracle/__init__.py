"""CPU FP64 oracle for the sparsity-discovering exact GP (test infrastructure).

This package is the reference that the GPU library is checked against.  It is
plain, slow, dense NumPy/LAPACK code in float64 that follows the paper's
definitions directly:

* ``oracle.kernel``     -- the compact core of Section 2.2 (eq:kstat) and a
                           Wendland core, the bump functions (eq:bump), the
                           sparsity-discovering kernel (eq:bump_kernel, plus a
                           SUM combine), the stored-entry predicate, dense K.
* ``oracle.gp``         -- log marginal likelihood (eqn:log_likelihood) by
                           Cholesky, its analytic gradient, the posterior
                           (eq:pred_distr).
* ``oracle.estimators`` -- counter-based Rademacher probes (SplitMix64),
                           stochastic Lanczos quadrature, Hutchinson traces,
                           the randomised Taylor-series log-det cited in
                           Section 2.5.
* ``oracle.sparsity``   -- the sparsity bound (eq:sparsity_estimate) and the
                           constrained / augmented objectives of Section 2.4.

It shares no code with the GPU path and imports nothing from it.  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import
it; the product path never calls it.

Parity status: every function here is pinned by tests in ``tests/`` against
closed forms, multi-precision evaluations of the paper's literal formulas,
brute force on tiny inputs, or invariants.  None is "parity unpinned".
"""

from . import kernel, gp, estimators, sparsity  # noqa: F401

__all__ = ["kernel", "gp", "estimators", "sparsity"]
