"""The 100,000-point 3-D configuration: points uniform in [0,1)^3, Wendland
core for ~100 core neighbours per row, 8 x 4 bump functions with radii
U(0.03, 0.06), SUM combine, y = 5 Gaussian bumps + N(0, 0.01^2), noise
variance 1e-4; CG rtol 1e-10 with the low-rank preconditioner and the
factored operator; SLQ with 30 Rademacher probes.

* The log-det with the quadrature truncated at 50 Lanczos steps stays within
  3 standard errors of the one on every CG step (its truncation bias is
  small against the estimator's spread), and the gradient does not depend
  on the cap (the trace term uses the CG solves).
* The adjoint gradient of sigma2, the core radius, one bump's (a, beta, r,
  c_0) and the noise variance against central differences of the GPU LML
  with common random numbers (same probes at h +- step, step 1e-4 of the
  value): both estimate the same derivative with independent stochastic
  errors of the size of the estimator's standard error, so a component
  passes within 4 SE, with SE the spread of the adjoint estimate over six
  probe seeds (plus 1e-6 relative for rounding and the difference quotient).
  The differences use the quadrature on every CG step: a 50-step cap adds a
  truncation bias whose dependence on h the adjoint does not see (measured
  here: 32 SE on the noise variance)."""
import numpy as np
import pytest

from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_c2_slq_and_gradient_vs_central_differences():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.uniform3d_100k()
    n, nh = w.x.shape[0], len(w.h)
    gu.log("C2 n=%d nh=%d" % (n, nh))
    x, y = gu.dev(w.x), gu.dev(w.y)
    c = gu.ctx()

    def est(seed, m):
        return sd.estimator(probes=30, seed=seed, lanczos_steps=m, cg_rtol=1e-10, cg_max_iter=20000,
                            precond=sd.PRECOND_LOWRANK, operator_form=sd.OPERATOR_FACTORED)

    v50, g50, i50 = c.lml_grad(w.desc, x, y, w.h, est(1, 50))
    v0, g0, i0 = c.lml_grad(w.desc, x, y, w.h, est(1, 0))
    gu.log("  nnz/row %.1f cg iters %d; logdet 50 steps %.10g all %.10g (se %.4g)" %
           (i0.nnz / n, i0.cg_iters, i50.logdet, i0.logdet, i0.logdet_stderr))
    assert i0.cg_relres_max <= 1e-10
    assert abs(i50.logdet - i0.logdet) <= 3.0 * i0.logdet_stderr
    assert np.array_equal(g50, g0)
    idx = [0, 1, 2, 3, 4, 5, nh - 1]
    gs = [g0[idx]]
    for seed in range(2, 7):
        gs.append(c.lml_grad(w.desc, x, y, w.h, est(seed, 0))[1][idx])
    se = np.std(np.array(gs), axis=0, ddof=1)
    e = est(1, 0)
    for j, k in enumerate(idx):
        step = 1e-4 * max(abs(w.h[k]), 1e-2)
        hp, hm = w.h.copy(), w.h.copy()
        hp[k] += step
        hm[k] -= step
        vp, _ = c.lml(w.desc, x, y, hp, e)
        vm, _ = c.lml(w.desc, x, y, hm, e)
        fd = (vp - vm) / (2.0 * step)
        gu.log("  h[%d] adjoint %.8g fd %.8g se %.3g (%.2f se)" % (k, g0[k], fd, se[j], abs(g0[k] - fd) / se[j]))
        assert abs(g0[k] - fd) <= 4.0 * se[j] + 1e-6 * abs(fd)
