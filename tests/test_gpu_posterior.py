"""GPU posterior (eq:pred_distr) parity against the dense oracle."""
import numpy as np
import pytest

from oracle import gp
from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("core,combine,dim", [(1, 1, 2), (1, 0, 2), (0, 1, 3), (0, 0, 3), (0, 1, 4)])
def test_posterior_matches_oracle(core, combine, dim):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(1500, dim, 3, 2, 13, core=core, combine=combine, per_row=15.0)
    rng = np.random.default_rng(1)
    x0 = np.concatenate([
        rng.random((150, dim)),                   # interior
        w.x[:10],                                 # on training points
        rng.random((5, dim)) * 1.4 - 0.2,         # partly outside the box
        np.full((1, dim), 7.0),                   # far away
    ])
    gu.log("posterior core=%d combine=%d dim=%d n0=%d" % (core, combine, dim, len(x0)))
    c = gu.ctx()
    est = sd.estimator(probes=1, cg_rtol=1e-13, cg_max_iter=20000)
    m, v = c.posterior_mean_var(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, gu.dev(x0), est)
    m0, v0 = gp.posterior_mean_var(w.desc, w.h, w.x, w.y, x0)
    m, v = m.cpu().numpy(), v.cpu().numpy()
    ms = np.abs(m0).max()
    assert np.allclose(m, m0, rtol=1e-8, atol=1e-10 * ms), np.abs(m - m0).max()
    vs = np.abs(v0).max()
    assert np.allclose(v, v0, rtol=1e-7, atol=1e-9 * vs), np.abs(v - v0).max()
    assert m[-1] == 0.0


def test_posterior_many_test_points_chunks():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(800, 2, 2, 2, 2, per_row=10.0)
    x0 = np.random.default_rng(5).random((200, 2))   # 4 chunks of <= 64, ragged tail
    gu.log("posterior chunks n0=200")
    c = gu.ctx()
    est = sd.estimator(probes=1, cg_rtol=1e-13, cg_max_iter=20000)
    m, v = c.posterior_mean_var(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, gu.dev(x0), est)
    m0, v0 = gp.posterior_mean_var(w.desc, w.h, w.x, w.y, x0)
    assert np.allclose(m.cpu().numpy(), m0, rtol=1e-8, atol=1e-10)
    assert np.allclose(v.cpu().numpy(), v0, rtol=1e-7, atol=1e-10)
