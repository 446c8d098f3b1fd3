"""Batched population evaluation (sdgp_lml_grad_batched).

* Exact mode (identity probes): every member against the dense Cholesky
  oracle, at the single-evaluation tolerances.
* Stochastic mode: every member against the single-evaluation entry point
  on the same probes.  The member with the largest core radius shares the
  single evaluation's cell grid, so its result is bitwise identical; the
  others are ordered on a coarser grid and agree to rounding.
* Graph replay of the CG iterations gives bitwise the non-graph result, on
  repeated calls with other stream work in between.
* A member with invalid hyperparameters fails alone: its status is
  INVALID_ARG with NaN outputs, and the other members' results are bitwise
  those of the batch without it."""
import numpy as np
import pytest

from oracle import gp
from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def population(n, dim, n1, n2, members, seed, combine=1, per_row=12.0):
    """Members differ in sigma2, core radius and bump heights; member 0 has
    the largest core radius."""
    w = wl.random_small(n, dim, n1, n2, seed, combine=combine, per_row=per_row, noise_var=1e-3)
    rng = np.random.default_rng(seed + 1000)
    H = np.tile(w.h, (members, 1))
    for m in range(members):
        p = wl.unpack_hyper(w.desc, w.h)
        s2 = 1.0 if m == 0 else rng.uniform(0.5, 1.5)
        rc = p["r_core"] * (1.0 if m == 0 else rng.uniform(0.6, 0.95))
        a = p["a"] * (1.0 if m == 0 else rng.uniform(0.3, 1.0, size=p["a"].shape))
        H[m] = wl.pack_hyper(w.desc, s2, rc, a, p["beta"], p["r"], p["c"], p["noise_var"])
    return w, H


@pytest.mark.parametrize("combine", [1, 0], ids=["sum", "product"])
def test_batched_exact_matches_oracle(combine):
    """Every member of a population (assembled together, every assembly
    phase one launch over all members) against the dense oracle."""
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, H = population(1200, 3, 2, 2, 3, 21, combine=combine)
    gu.log("batched exact B=%d n=%d combine=%d" % (H.shape[0], w.x.shape[0], combine))
    c = gu.ctx()
    v, g, st, infos = c.lml_grad_batched(w.desc, gu.dev(w.x), gu.dev(w.y), H, sd.exact_estimator())
    assert (st == sd.OK).all(), st
    for m in range(H.shape[0]):
        v0, g0 = gp.lml_grad(w.desc, H[m], w.x, w.y)
        gu.log("  member %d gpu %.15g oracle %.15g iters %d" % (m, v[m], v0, infos[m].cg_iters))
        assert abs(v[m] - v0) <= gu.LML_REL * abs(v0)
        assert gu.grad_close(g[m], g0).all()


@pytest.mark.parametrize("precond,operator", [
    (0, 0), (1, 0),
    pytest.param(1, 1, marks=pytest.mark.skip(
        reason="an earlier version of the batched factored-operator path met a device memory fault whose "
               "cause is not shown; the library rejects that combination and the case stays off the GPU")),
], ids=["plain", "lowrank", "factored"])
def test_batched_matches_single(precond, operator):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, H = population(4000, 3, 4, 2, 5, 7)
    gu.log("batched vs single precond=%d operator=%d" % (precond, operator))
    est = sd.estimator(probes=12, seed=77, cg_rtol=1e-11, cg_max_iter=5000, precond=precond,
                       operator_form=operator)
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    v, g, st, infos = c.lml_grad_batched(w.desc, x, y, H, est)
    assert (st == sd.OK).all(), st
    for m in range(H.shape[0]):
        v1, g1, i1 = c.lml_grad(w.desc, x, y, H[m], est)
        gu.log("  member %d batched %.15g single %.15g iters %d/%d" % (m, v[m], v1, infos[m].cg_iters,
                                                                        i1.cg_iters))
        assert infos[m].nnz == i1.nnz
        # candidate pairs: every stored pair is one; member 0 has the
        # largest core radius, so its cell grid is the population's
        assert i1.nnz <= i1.candidates <= w.x.shape[0] ** 2
        assert infos[m].nnz <= infos[m].candidates <= w.x.shape[0] ** 2
        if m == 0:
            assert infos[m].candidates == i1.candidates
        if m == 0:
            assert v[m] == v1
            assert np.array_equal(g[m], g1)
        else:
            assert abs(v[m] - v1) <= 1e-9 * abs(v1)
            assert gu.grad_close(g[m], g1, rel=1e-7).all()


def test_batched_factored_rejected():
    """Populations reject the factored operator with INVALID_ARG on the
    host, before any device work."""
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, H = population(300, 3, 2, 2, 2, 5)
    est = sd.estimator(probes=4, seed=1, cg_rtol=1e-10, cg_max_iter=100, precond=sd.PRECOND_LOWRANK,
                       operator_form=sd.OPERATOR_FACTORED)
    c = gu.ctx()
    with pytest.raises(sd.SdgpError) as e:
        c.lml_grad_batched(w.desc, gu.dev(w.x), gu.dev(w.y), H, est)
    assert e.value.status == sd.INVALID_ARG


def test_graph_replay_is_bitwise():
    gu.need_gpu()
    import torch
    import paper_2205_09070_amd as sd
    w, H = population(3000, 2, 3, 2, 4, 3)
    gu.log("graph replay bitwise")
    est = sd.estimator(probes=8, seed=5, cg_rtol=1e-11, cg_max_iter=5000, precond=1)
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    v0, g0, st0, _ = c.lml_grad_batched(w.desc, x, y, H, est)
    assert (st0 == sd.OK).all()
    c.set_option("graph", 1)
    junk = torch.randn(1 << 20, dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        junk.mul_(1.0001).add_(1.0)
        v1, g1, st1, _ = c.lml_grad_batched(w.desc, x, y, H, est)
        torch.cuda.synchronize()
        gu.log("  replay %d: %s" % (rep, v1))
        assert (st1 == sd.OK).all()
        assert np.array_equal(v1, v0)
        assert np.array_equal(g1, g0)
    # a single evaluation in graph mode too
    c.set_option("graph", 1)
    vs, gs, _ = c.lml_grad(w.desc, x, y, H[1], est)
    c.set_option("graph", 0)
    vn, gn, _ = c.lml_grad(w.desc, x, y, H[1], est)
    assert vs == vn and np.array_equal(gs, gn)


def test_invalid_member_fails_alone():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, H = population(2500, 2, 2, 2, 4, 11)
    gu.log("invalid member isolation")
    est = sd.estimator(probes=8, seed=9, cg_rtol=1e-11, cg_max_iter=5000)
    bad = H.copy()
    bad[2, 0] = -1.0                       # sigma2 < 0
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    v, g, st, _ = c.lml_grad_batched(w.desc, x, y, bad, est)
    assert st[2] == sd.INVALID_ARG
    assert np.isnan(v[2]) and np.isnan(g[2]).all()
    keep = [0, 1, 3]
    v1, g1, st1, _ = c.lml_grad_batched(w.desc, x, y, H[keep], est)
    assert (st[keep] == sd.OK).all() and (st1 == sd.OK).all()
    assert np.array_equal(v[keep], v1)
    assert np.array_equal(g[keep], g1)
