"""Block preconditioner (M = B + F F^T, 16-row schedule tiles) on the GPU
against the oracle's block-preconditioned estimator with the same tiles
(rebuilt on the CPU from the library's documented ordering) and the same
probes: log-det, LML and gradient to the single-evaluation tolerances; the
solve itself matches the unpreconditioned one; ragged last tiles (n not a
multiple of 16) and n1 = 0 are covered; the block preconditioner needs
fewer CG iterations than c I + F F^T."""
import numpy as np
import pytest

from oracle import estimators as es
from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu
from tests import sched_ref

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="block preconditioner switched off: its device path met a memory fault "
                                      "whose cause is not yet found (the option is rejected)")]


@pytest.mark.parametrize("dim,n1,n,factored", [(2, 3, 1203, True), (3, 5, 1200, True), (3, 12, 1211, False),
                                               (3, 0, 1000, True)],
                         ids=["2d-n1_3-factored", "3d-n1_5-factored", "3d-n1_12-assembled", "3d-n1_0"])
def test_block_estimators_match_oracle(dim, n1, n, factored):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(n, dim, n1, 2, 21 + n1, combine=1, per_row=14.0, noise_var=1e-3)
    gu.log("block preconditioner dim=%d n1=%d n=%d factored=%d" % (dim, n1, n, factored))
    P, seed = 12, 9090
    tiles = sched_ref.schedule_tiles(w.x, wl.unpack_hyper(w.desc, w.h)["r_core"])
    c = gu.ctx()
    est = sd.estimator(probes=P, seed=seed, cg_rtol=1e-12, cg_max_iter=5000, precond=sd.PRECOND_BLOCK,
                       operator_form=sd.OPERATOR_FACTORED if factored else sd.OPERATOR_ASSEMBLED)
    val, g, info = c.lml_grad(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, est)
    v0, g0, ld0, se0 = es.block_preconditioned_lml_grad(w.desc, w.h, w.x, w.y, seed, P, 400, tiles,
                                                        factored=factored)
    gu.log("  gpu logdet %.12g oracle %.12g (se %.3g), cg iters %d" % (info.logdet, ld0, se0, info.cg_iters))
    assert abs(info.logdet - ld0) <= 1e-7 * abs(ld0)
    assert abs(val - v0) <= 1e-7 * abs(v0)
    assert gu.grad_close(g, g0, rel=1e-6).all()
    # the solve itself does not depend on the preconditioner
    _, _, info2 = c.lml_grad(w.desc, gu.dev(w.x), gu.dev(w.y), w.h,
                             sd.estimator(probes=P, seed=seed, cg_rtol=1e-12, cg_max_iter=5000))
    assert abs(info.yKy - info2.yKy) <= 1e-9 * abs(info2.yKy)


def test_block_needs_fewer_iterations_than_lowrank():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.uniform_3d(20000, 40.0, 8, 4, seed=3)
    gu.log("block vs low-rank iterations n=20000")
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    base = dict(probes=8, seed=1, cg_rtol=1e-10, cg_max_iter=20000, operator_form=sd.OPERATOR_FACTORED)
    vb, gb, ib = c.lml_grad(w.desc, x, y, w.h, sd.estimator(precond=sd.PRECOND_BLOCK, **base))
    vl, gl, il = c.lml_grad(w.desc, x, y, w.h, sd.estimator(precond=sd.PRECOND_LOWRANK, **base))
    gu.log("  iterations block %d low-rank %d; logdet %.6f +- %.3g vs %.6f +- %.3g"
           % (ib.cg_iters, il.cg_iters, ib.logdet, ib.logdet_stderr, il.logdet, il.logdet_stderr))
    assert ib.cg_iters < il.cg_iters
    assert abs(ib.yKy - il.yKy) <= 1e-7 * abs(il.yKy)
    # both are unbiased estimates of the same log-det
    assert abs(ib.logdet - il.logdet) <= 5.0 * np.hypot(ib.logdet_stderr, il.logdet_stderr)


def test_block_rejected_without_sum_or_rademacher():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(300, 2, 2, 2, 1, combine=0, per_row=10.0)
    c = gu.ctx()
    with pytest.raises(sd.SdgpError) as e:
        c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, sd.estimator(probes=4, precond=sd.PRECOND_BLOCK))
    assert e.value.status == 1
    est = sd.exact_estimator()
    est.precond = sd.PRECOND_BLOCK
    with pytest.raises(sd.SdgpError):
        c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, est)
