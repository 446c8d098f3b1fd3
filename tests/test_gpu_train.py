"""Differential-evolution training over the batched device path."""
import numpy as np
import pytest

from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_train_de_improves_and_reports_consistent_fitness():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(800, 2, 2, 2, 17, per_row=15.0, noise_var=1e-2)
    gu.log("train_de n=%d" % w.x.shape[0])
    nh = len(w.h)
    lo, hi = w.h.copy(), w.h.copy()
    lo[1], hi[1] = 0.5 * w.h[1], 1.5 * w.h[1]        # core radius
    lo[0], hi[0] = 0.2, 3.0                          # sigma2
    lo[-1], hi[-1] = 1e-4, 0.1                       # noise variance
    rng = np.random.default_rng(4)
    B = 6
    H0 = np.tile(w.h, (B, 1))
    for k in (0, 1, nh - 1):
        H0[:, k] = lo[k] + (hi[k] - lo[k]) * rng.random(B)
    est = sd.estimator(probes=8, seed=2, cg_rtol=1e-11, cg_max_iter=5000)
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    H, fit, hist = c.train_de(w.desc, x, y, H0, lo, hi, est, generations=4, F=0.7, CR=0.9, seed=9)
    gu.log("  history %s" % hist)
    assert np.all(np.diff(hist) >= 0.0)
    assert np.isfinite(fit).all()
    assert (H >= lo).all() and (H <= hi).all()
    # fixed components untouched
    free = np.zeros(nh, bool)
    free[[0, 1, nh - 1]] = True
    assert np.array_equal(H[:, ~free], H0[:, ~free])
    # reported fitness is the LML of the returned vectors
    for m in range(B):
        v, _, _ = c.lml_grad(w.desc, x, y, H[m], est)
        assert abs(v - fit[m]) <= 1e-8 * abs(v)
