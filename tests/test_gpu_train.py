"""Differential-evolution training over the batched device path
(sdgp_train_de), checked against the oracle.

The population is evaluated in exact mode (identity probes), so every
member's fitness is a deterministic function of its hyperparameters:

* objective LML: the final fitness of every member equals the dense
  Cholesky oracle's ln L of the returned vector (1e-6 relative);
* objective AUGMENTED (Section 2.4 eq:augmented): fitness = the oracle's
  augmented objective of (ln L, s(h)), with s(h) the oracle's sparsity bound
  (eq:sparsity_estimate) of the returned vector;
* objective CONSTRAINED (Section 2.4 eq:constrained): fitness = ln L when the
  oracle's s(h) is below the requirement, else -inf; the bump radii are
  searched over a range whose bound crosses the requirement, so both
  branches occur.
The best-fitness history never decreases, bounds hold, and fixed components
stay fixed."""
import numpy as np
import pytest

from oracle import gp
from oracle import sparsity as osp
from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _setup(seed_rng, free_radii):
    w = wl.random_small(700, 2, 2, 2, 17, per_row=15.0, noise_var=1e-2)
    nh = len(w.h)
    lo, hi = w.h.copy(), w.h.copy()
    lo[1], hi[1] = 0.5 * w.h[1], 1.5 * w.h[1]        # core radius
    lo[0], hi[0] = 0.2, 3.0                          # sigma2
    lo[-1], hi[-1] = 1e-3, 0.1                       # noise variance
    free = [0, 1, nh - 1]
    if free_radii:
        p = wl.unpack_hyper(w.desc, w.h)
        for i in range(w.desc.n1):
            for j in range(w.desc.n2):
                k = wl.hyper_index(w.desc, i, j) + 2   # the bump radius r_ij
                lo[k], hi[k] = 0.5 * p["r"][i, j], 2.0 * p["r"][i, j]
                free.append(k)
    rng = np.random.default_rng(seed_rng)
    B = 6
    H0 = np.tile(w.h, (B, 1))
    for k in free:
        H0[:, k] = lo[k] + (hi[k] - lo[k]) * rng.random(B)
    return w, lo, hi, H0, np.array(sorted(free))


@pytest.mark.parametrize("objective", ["lml", "augmented", "constrained"])
def test_train_de_matches_oracle(objective):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, lo, hi, H0, free = _setup(4, objective != "lml")
    obj = {"lml": sd.DE_LML, "augmented": sd.DE_AUGMENTED, "constrained": sd.DE_CONSTRAINED}[objective]
    # requirement: the median bound of the initial population, so that the
    # search meets feasible and infeasible vectors
    s_init = [osp.sparsity_bound(w.desc, h) for h in H0]
    req = float(np.median(s_init)) if objective == "constrained" else 1.0
    gu.log("train_de objective=%s n=%d requirement %.3g (initial bounds %s)" %
           (objective, w.x.shape[0], req, np.round(s_init, 4)))
    est = sd.exact_estimator()
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    H, fit, hist = c.train_de(w.desc, x, y, H0, lo, hi, est, generations=3, F=0.7, CR=0.9, seed=9,
                              objective=obj, requirement=req, domain_volume=1.0)
    gu.log("  history %s" % hist)
    assert np.all(np.diff(hist) >= 0.0)
    assert (H >= lo).all() and (H <= hi).all()
    fixed = np.ones(len(w.h), bool)
    fixed[free] = False
    assert np.array_equal(H[:, fixed], H0[:, fixed])
    n_feasible = 0
    for m in range(H.shape[0]):
        v0, _, _, _ = gp.lml(w.desc, H[m], w.x, w.y)
        s0 = osp.sparsity_bound(w.desc, H[m])
        if objective == "lml":
            want = v0
        elif objective == "augmented":
            want = osp.augmented_objective(v0, s0)
        else:
            want = v0 if osp.constrained_feasible(s0, req) else -np.inf
        gu.log("  member %d fitness %.15g oracle %.15g (s %.4g)" % (m, fit[m], want, s0))
        if np.isinf(want):
            assert fit[m] == want
        else:
            n_feasible += 1
            assert abs(fit[m] - want) <= gu.LML_REL * abs(want)
    assert n_feasible >= 1
    assert hist[-1] == np.max(fit)
