"""Gradient of the GPU LML against central finite differences of the GPU LML
itself (exact mode: identity probes, CG to 1e-13, so ln L is a smooth
deterministic function of h), and the torch.autograd path against the plain
call.  Components cover every hyperparameter kind: sigma2, the core radius,
bump height, shape, radius and centre, and the noise variance."""
import numpy as np
import pytest

from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _components(desc):
    """Indices of sigma2, r_core, (a, beta, r, c_0) of bump (0, 0) and of the
    last bump, and noise_var."""
    nh = desc.n_hyper
    first = wl.hyper_index(desc, 0, 0)
    last = wl.hyper_index(desc, desc.n1 - 1, desc.n2 - 1)
    idx = [0, 1, first, first + 1, first + 2, first + 3, last, last + 2, last + 3 + desc.dim - 1, nh - 1]
    return sorted(set(idx))


@pytest.mark.parametrize("combine,dim", [(1, 2), (0, 2), (1, 3)], ids=["sum-2d", "product-2d", "sum-3d"])
def test_gradient_matches_central_differences(combine, dim):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(700, dim, 2, 2, 31 + dim, combine=combine, per_row=14.0, noise_var=1e-2)
    gu.log("finite differences combine=%d dim=%d n=%d" % (combine, dim, w.x.shape[0]))
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    est = sd.exact_estimator(cg_rtol=1e-13)
    _, g, _ = c.lml_grad(w.desc, x, y, w.h, est)
    for k in _components(w.desc):
        step = 1e-4 * max(abs(w.h[k]), 1e-2)
        hp, hm = w.h.copy(), w.h.copy()
        hp[k] += step
        hm[k] -= step
        vp, _ = c.lml(w.desc, x, y, hp, est)
        vm, _ = c.lml(w.desc, x, y, hm, est)
        fd = (vp - vm) / (2 * step)
        gu.log("  h[%d]=%.6g grad %.10g fd %.10g" % (k, w.h[k], g[k], fd))
        assert abs(g[k] - fd) <= 2e-5 * abs(fd) + 1e-6 * np.abs(g).max(), k


def test_autograd_path_matches_plain_call():
    gu.need_gpu()
    import torch
    import paper_2205_09070_amd as sd
    w = wl.random_small(2000, 3, 2, 2, 8, per_row=15.0)
    gu.log("autograd path")
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    est = sd.estimator(probes=8, seed=3, cg_rtol=1e-11)
    v0, g0, _ = c.lml_grad(w.desc, x, y, w.h, est)
    h = torch.tensor(w.h, dtype=torch.float64, requires_grad=True)
    out = sd.lml(h, c, w.desc, x, y, est)
    (2.0 * out).backward()
    assert float(out.detach()) == v0
    assert np.array_equal(h.grad.numpy(), 2.0 * g0)
