"""GPU LML and gradient parity against the oracle.

Exact mode (identity probes, CG to 1e-13): LML within 1e-6 relative and
every gradient component within 1e-5 relative of the dense Cholesky oracle.
Stochastic mode (Rademacher probes shared through the SplitMix64 counter
generator): LML and gradient against the oracle's own SLQ + Hutchinson
estimator on the same probes."""
import numpy as np
import pytest

from oracle import estimators as es
from oracle import gp
from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

EXACT = [
    ("2d-kstat-product", lambda: wl.small_2d(2000, 0, core=1, combine=0)),
    ("2d-kstat-sum", lambda: wl.small_2d(2000, 0, core=1, combine=1)),
    ("2d-wendland-sum", lambda: wl.small_2d(2000, 0, core=0, combine=1)),
    ("2d-wendland-product", lambda: wl.small_2d(2000, 0, core=0, combine=0)),
    ("3d-sum", lambda: wl.random_small(1500, 3, 3, 2, 8, per_row=20.0)),
    ("4d-sum", lambda: wl.random_small(1200, 4, 2, 2, 6, per_row=15.0)),
]


@pytest.mark.parametrize("name,make", EXACT, ids=[c[0] for c in EXACT])
def test_exact_lml_and_gradient(name, make):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = make()
    gu.log("exact lml/grad %s n=%d" % (name, w.x.shape[0]))
    c = gu.ctx()
    val, g, info = c.lml_grad(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, sd.exact_estimator())
    v0, g0 = gp.lml_grad(w.desc, w.h, w.x, w.y)
    gu.log("  gpu %.15g oracle %.15g  cg iters %d relres %.2e" % (val, v0, info.cg_iters, info.cg_relres_max))
    assert abs(val - v0) <= gu.LML_REL * abs(v0)
    ok = gu.grad_close(g, g0)
    assert ok.all(), "grad mismatch at %s: gpu %s oracle %s" % (np.nonzero(~ok)[0], g[~ok], g0[~ok])


def test_exact_lml_only_matches():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.small_2d(2000, 0, core=1, combine=1)
    gu.log("exact lml only")
    c = gu.ctx()
    val, info = c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, sd.exact_estimator())
    v0, _, logdet0, yKy0 = gp.lml(w.desc, w.h, w.x, w.y)
    assert abs(info.logdet - logdet0) <= 1e-9 * abs(logdet0) + 1e-9
    assert abs(info.yKy - yKy0) <= 1e-9 * abs(yKy0)
    assert abs(val - v0) <= gu.LML_REL * abs(v0)


@pytest.mark.parametrize("combine", [0, 1])
def test_stochastic_estimators_match_oracle_estimators(combine):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(1500, 2, 2, 2, 3, combine=combine, per_row=12.0, noise_var=1e-3)
    gu.log("stochastic lml/grad combine=%d" % combine)
    P, seed = 16, 12345
    c = gu.ctx()
    est = sd.estimator(probes=P, seed=seed, cg_rtol=1e-12, cg_max_iter=5000)
    val, g, info = c.lml_grad(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, est)
    Z = es.rademacher(seed, w.x.shape[0], P)
    v0, g0, ld0, se0 = es.stochastic_lml_grad(w.desc, w.h, w.x, w.y, Z, 400)
    gu.log("  gpu logdet %.12g oracle SLQ %.12g (se %.3g)" % (info.logdet, ld0, se0))
    assert abs(info.logdet - ld0) <= 1e-7 * abs(ld0)
    assert abs(val - v0) <= 1e-7 * abs(v0)
    assert gu.grad_close(g, g0, rel=1e-6).all()


def test_stochastic_truncated_lanczos_matches_oracle_lanczos():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(1000, 3, 2, 2, 4, per_row=15.0, noise_var=1e-2)
    gu.log("truncated lanczos")
    P, seed, m = 8, 99, 30
    c = gu.ctx()
    est = sd.estimator(probes=P, seed=seed, lanczos_steps=m, cg_rtol=1e-12)
    _, info = c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, est)
    from oracle import kernel as kn
    A = kn.kernel_matrix(w.desc, w.h, w.x)
    Z = es.rademacher(seed, w.x.shape[0], P)
    ld0, _ = es.slq_logdet(A, Z, m)
    assert abs(info.logdet - ld0) <= 1e-6 * abs(ld0)


@pytest.mark.parametrize("per_row", [20.0, 300.0])
def test_spmm_matches_dense_product(per_row):
    """R = 1 (the SpMV; at 300 neighbours per row the rows span several
    128-entry steps of a 32-lane group) and wider right-hand sides."""
    gu.need_gpu()
    import torch
    w = wl.random_small(900, 2, 2, 2, 1, per_row=per_row)
    gu.log("spmm R in (1, 2, 5, 34, 64, 70), per_row %g" % per_row)
    c = gu.ctx()
    rp, col, val = c.kernel_assemble(w.desc, gu.dev(w.x), w.h)
    _, _, _, S = gu.csr_to_host(rp, col, val, w.x.shape[0])
    rng = np.random.default_rng(0)
    for R in (1, 2, 5, 34, 64, 70):
        X = rng.standard_normal((w.x.shape[0], R))
        Y = c.csr_spmm(rp, col, val, gu.dev(X if R > 1 else X[:, 0]))
        ref = S @ (X if R > 1 else X[:, 0])
        assert np.allclose(Y.cpu().numpy(), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    torch.cuda.synchronize()


def test_deterministic_bitwise():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(3000, 3, 4, 2, 5, per_row=20.0)
    gu.log("determinism")
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    est = sd.estimator(probes=8, seed=3)
    a = c.lml_grad(w.desc, x, y, w.h, est)
    b = c.lml_grad(w.desc, x, y, w.h, est)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1])


def test_not_spd_reported():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    # the printed compact core is not positive definite in 4-D: on the 8^4
    # lattice with radius 3.5 spacings K has 6 negative eigenvalues (min
    # -4.8e-4), and CG on Rademacher probes meets p^T A p <= 0
    g = np.arange(8) / 8.0
    x = np.stack(np.meshgrid(g, g, g, g, indexing="ij"), -1).reshape(-1, 4)
    desc = wl.KernelDesc(4, 0, 1, 1, 1)
    h = np.array([1.0, 3.5 / 8.0 + 1e-9, 0.0])
    gu.log("not-spd path")
    c = gu.ctx()
    with pytest.raises(sd.SdgpError) as e:
        c.lml(desc, gu.dev(x), gu.dev(np.ones(len(x))), h, sd.estimator(probes=4, cg_max_iter=3000))
    assert e.value.status in (3,)


def test_invalid_arguments_rejected():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(100, 2, 1, 1, 0)
    c = gu.ctx()
    bad = w.h.copy()
    bad[1] = -1.0
    with pytest.raises(sd.SdgpError) as e:
        c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), bad)
    assert e.value.status == 1
    bad = w.h.copy()
    bad[0] = np.nan
    with pytest.raises(sd.SdgpError):
        c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), bad)
    with pytest.raises(sd.SdgpError):
        c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, sd.estimator(probes=65))
    for name, value in (("union_spmm", 2), ("fw_mfma", -2), ("spmm_blocks", 12), ("no_such_option", 1)):
        with pytest.raises(sd.SdgpError) as e:
            c.set_option(name, value)
        assert e.value.status == 1


def test_not_converged_reported():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(800, 2, 1, 2, 2, per_row=15.0)
    c = gu.ctx()
    with pytest.raises(sd.SdgpError) as e:
        c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, sd.estimator(probes=2, cg_max_iter=1))
    assert e.value.status == 4


@pytest.mark.parametrize("dim,n1", [(2, 3), (3, 5), (3, 12)])
def test_preconditioned_estimators_match_oracle(dim, n1):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(1200, dim, n1, 2, 21, combine=1, per_row=14.0, noise_var=1e-3)
    gu.log("preconditioned lml/grad dim=%d n1=%d" % (dim, n1))
    P, seed = 12, 777
    c = gu.ctx()
    est = sd.estimator(probes=P, seed=seed, cg_rtol=1e-12, cg_max_iter=5000, precond=sd.PRECOND_LOWRANK)
    val, g, info = c.lml_grad(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, est)
    v0, g0, ld0, se0 = es.preconditioned_lml_grad(w.desc, w.h, w.x, w.y, seed, P, 400)
    gu.log("  gpu logdet %.12g oracle %.12g (se %.3g), cg iters %d" % (info.logdet, ld0, se0, info.cg_iters))
    assert abs(info.logdet - ld0) <= 1e-7 * abs(ld0)
    assert abs(val - v0) <= 1e-7 * abs(v0)
    assert gu.grad_close(g, g0, rel=1e-6).all()
    # the solve itself does not depend on the preconditioner
    _, _, info2 = c.lml_grad(w.desc, gu.dev(w.x), gu.dev(w.y), w.h,
                             sd.estimator(probes=P, seed=seed, cg_rtol=1e-12, cg_max_iter=5000))
    assert abs(info.yKy - info2.yKy) <= 1e-9 * abs(info2.yKy)


def test_preconditioner_rejected_for_product_and_identity():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(300, 2, 2, 2, 1, combine=0, per_row=10.0)
    c = gu.ctx()
    with pytest.raises(sd.SdgpError) as e:
        c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, sd.estimator(probes=4, precond=sd.PRECOND_LOWRANK))
    assert e.value.status == 1
    est = sd.exact_estimator()
    est.precond = sd.PRECOND_LOWRANK
    with pytest.raises(sd.SdgpError):
        c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, est)


def test_preconditioned_posterior_matches():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(900, 3, 4, 2, 2, combine=1, per_row=12.0)
    x0 = np.random.default_rng(2).random((70, 3))
    c = gu.ctx()
    est = sd.estimator(probes=1, cg_rtol=1e-13, cg_max_iter=20000, precond=sd.PRECOND_LOWRANK)
    m, v = c.posterior_mean_var(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, gu.dev(x0), est)
    m0, v0 = gp.posterior_mean_var(w.desc, w.h, w.x, w.y, x0)
    assert np.allclose(m.cpu().numpy(), m0, rtol=1e-8, atol=1e-10)
    assert np.allclose(v.cpu().numpy(), v0, rtol=1e-7, atol=1e-10)


# n1 = 16 and 32 fill the F^T Y kernel's template width (its unguarded,
# four-rows-at-a-time form); the others take its guarded form
@pytest.mark.parametrize("dim,n1", [(2, 3), (3, 12), (3, 16), (2, 32), (3, 40)])
def test_factored_operator_matches_oracle_and_assembled(dim, n1):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(1200, dim, n1, 2, 31, combine=1, per_row=14.0, noise_var=1e-3)
    gu.log("factored operator dim=%d n1=%d" % (dim, n1))
    P, seed = 12, 4242
    c = gu.ctx()
    base = dict(probes=P, seed=seed, cg_rtol=1e-12, cg_max_iter=5000, precond=sd.PRECOND_LOWRANK)
    vf, gf, inf_f = c.lml_grad(w.desc, gu.dev(w.x), gu.dev(w.y), w.h,
                               sd.estimator(operator_form=sd.OPERATOR_FACTORED, **base))
    va, ga, inf_a = c.lml_grad(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, sd.estimator(**base))
    v0, g0, ld0, _ = es.preconditioned_lml_grad(w.desc, w.h, w.x, w.y, seed, P, 400)
    gu.log("  factored %.12g assembled %.12g oracle %.12g; nnz %d vs %d" % (vf, va, v0, inf_f.nnz, inf_a.nnz))
    assert inf_f.nnz <= inf_a.nnz
    assert abs(vf - v0) <= 1e-7 * abs(v0)
    assert abs(vf - va) <= 1e-9 * abs(va)
    assert gu.grad_close(gf, g0, rel=1e-6).all()
    assert gu.grad_close(gf, ga, rel=1e-8).all()


@pytest.mark.parametrize("probes,operator,n", [(12, 1, 3001), (12, 0, 3001), (40, 1, 2999), (40, 0, 1203)],
                         ids=["1slab-factored", "1slab-assembled", "2slabs-factored", "2slabs-assembled"])
def test_union_spmm_matches_csr_spmm(probes, operator, n):
    """The CG SpMM over the 4-row union lists (union_spmm = 1; the default
    from 65536 points) agrees to rounding with the CSR SpMM (union_spmm = 0),
    with one and with two slabs of right-hand sides, on point counts that
    leave a ragged last group."""
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(n, 3, 6, 2, 50 + probes, per_row=18.0, noise_var=1e-3)
    gu.log("union spmm probes=%d operator=%d n=%d" % (probes, operator, n))
    est = sd.estimator(probes=probes, seed=9, cg_rtol=1e-11, cg_max_iter=5000, precond=1, operator_form=operator)
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    c.set_option("union_spmm", 1)
    v1, g1, i1 = c.lml_grad(w.desc, x, y, w.h, est)
    c.set_option("union_spmm", 0)
    v0, g0, i0 = c.lml_grad(w.desc, x, y, w.h, est)
    c.set_option("union_spmm", -1)
    gu.log("  union %.15g csr %.15g iters %d/%d" % (v1, v0, i1.cg_iters, i0.cg_iters))
    assert abs(i1.cg_iters - i0.cg_iters) <= 2
    assert abs(v1 - v0) <= 1e-10 * abs(v0)
    assert gu.grad_close(g1, g0, rel=1e-8).all()


def test_factored_operator_graph_replay_is_bitwise():
    """CG iterations replayed from a HIP graph (8 per graph) give bitwise the
    eager result with the factored operator, on repeated calls with other
    stream work in between."""
    gu.need_gpu()
    import torch
    import paper_2205_09070_amd as sd
    w = wl.random_small(3000, 3, 12, 2, 44, combine=1, per_row=14.0, noise_var=1e-3)
    gu.log("factored graph replay")
    est = sd.estimator(probes=12, seed=8, cg_rtol=1e-11, cg_max_iter=5000, precond=sd.PRECOND_LOWRANK,
                       operator_form=sd.OPERATOR_FACTORED)
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    v0, g0, i0 = c.lml_grad(w.desc, x, y, w.h, est)
    c.set_option("graph", 1)
    junk = torch.randn(1 << 20, dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        junk.mul_(1.0001).add_(1.0)
        v1, g1, i1 = c.lml_grad(w.desc, x, y, w.h, est)
        torch.cuda.synchronize()
        gu.log("  replay %d: %.15g iters %d" % (rep, v1, i1.cg_iters))
        assert v1 == v0 and np.array_equal(g1, g0)
        assert i1.cg_iters == i0.cg_iters
    c.set_option("graph", 0)


def test_factored_operator_requires_preconditioner():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(300, 2, 2, 2, 1, combine=1, per_row=10.0)
    c = gu.ctx()
    with pytest.raises(sd.SdgpError) as e:
        c.lml(w.desc, gu.dev(w.x), gu.dev(w.y), w.h,
              sd.estimator(probes=4, operator_form=sd.OPERATOR_FACTORED))
    assert e.value.status == 1


@pytest.mark.parametrize("terms", [1, 7, 60])
def test_taylor_logdet_matches_oracle_estimator(terms):
    gu.need_gpu()
    from oracle import kernel as kn
    w = wl.random_small(900, 2, 2, 2, 5, per_row=12.0, noise_var=0.3)
    gu.log("taylor logdet terms=%d" % terms)
    P, seed = 16, 99
    c = gu.ctx()
    ld, alpha = c.logdet_taylor(w.desc, gu.dev(w.x), w.h, probes=P, terms=terms, seed=seed)
    A = kn.kernel_matrix(w.desc, w.h, w.x)
    Z = es.rademacher(seed, w.x.shape[0], P)
    ld0, alpha0 = es.boutsidis_logdet(A, Z, terms)
    assert alpha == pytest.approx(alpha0, rel=1e-13)
    assert ld == pytest.approx(ld0, rel=1e-11, abs=1e-9)


@pytest.mark.parametrize("n1,operator", [(6, 1), (20, 1), (20, 0), (40, 1), (64, 1)],
                         ids=["n1=6-factored", "n1=20-factored", "n1=20-assembled", "n1=40-factored",
                              "n1=64-factored"])
def test_update_products_on_matrix_cores_match_broadcasts(n1, operator):
    """The F w products of the CG update kernels per 16-row tile on the
    matrix cores (fw_mfma = 1) agree to rounding with the per-row broadcast
    form (fw_mfma = 0)."""
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(3000, 3, n1, 2, 21, per_row=15.0, noise_var=1e-3)
    gu.log("fw_mfma n1=%d operator=%d" % (n1, operator))
    est = sd.estimator(probes=12, seed=6, cg_rtol=1e-11, cg_max_iter=5000, precond=1, operator_form=operator)
    c = gu.ctx()
    x, y = gu.dev(w.x), gu.dev(w.y)
    c.set_option("fw_mfma", 1)
    v1, g1, i1 = c.lml_grad(w.desc, x, y, w.h, est)
    c.set_option("fw_mfma", 0)
    v0, g0, i0 = c.lml_grad(w.desc, x, y, w.h, est)
    c.set_option("fw_mfma", -1)
    assert abs(i1.cg_iters - i0.cg_iters) <= 2
    assert abs(v1 - v0) <= 1e-10 * abs(v0)
    assert gu.grad_close(g1, g0, rel=1e-8).all()


_UNION_ORACLE = {}


def _union_oracle(P):
    """Oracle estimator (dense preconditioned SLQ + Hutchinson on the same
    probes) for the union-list parity cases, computed once per probe count."""
    if P not in _UNION_ORACLE:
        w = wl.random_small(3001, 3, 4, 2, 5, combine=1, per_row=20.0, noise_var=1e-2)
        _UNION_ORACLE[P] = (w, es.preconditioned_lml_grad(w.desc, w.h, w.x, w.y, 77, P, 300))
    return _UNION_ORACLE[P]


@pytest.mark.parametrize("probes", [16, 33], ids=["1slab", "2slabs"])
@pytest.mark.parametrize("operator", [1, 0], ids=["factored", "assembled"])
def test_union_spmm_matches_oracle(probes, operator):
    """The CG SpMM over the 4-row union lists (union_spmm = 1, the default
    from 65536 points), with the low-rank preconditioner, against the
    oracle's own preconditioned estimator on the same probes: 3001 points
    (750 full 4-row groups and a ragged one), 16 probes (one slab of
    right-hand-side columns) and 33 probes (two slabs); LML within 1e-7
    relative, every gradient component within 1e-6 relative (floor 1e-6 of
    the largest)."""
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, (v0, g0, ld0, se0) = _union_oracle(probes)
    gu.log("union spmm vs oracle probes=%d operator=%d n=%d" % (probes, operator, w.x.shape[0]))
    est = sd.estimator(probes=probes, seed=77, cg_rtol=1e-12, cg_max_iter=5000, precond=sd.PRECOND_LOWRANK,
                       operator_form=operator)
    c = gu.ctx()
    c.set_option("union_spmm", 1)
    v, g, info = c.lml_grad(w.desc, gu.dev(w.x), gu.dev(w.y), w.h, est)
    gu.log("  gpu %.15g oracle %.15g; logdet %.12g vs %.12g (se %.3g); cg iters %d" %
           (v, v0, info.logdet, ld0, se0, info.cg_iters))
    assert abs(info.logdet - ld0) <= 1e-7 * abs(ld0)
    assert abs(v - v0) <= 1e-7 * abs(v0)
    ok = gu.grad_close(g, g0, rel=1e-6)
    assert ok.all(), "grad mismatch at %s: gpu %s oracle %s" % (np.nonzero(~ok)[0], g[~ok], g0[~ok])


@pytest.mark.parametrize("operator", [0, 1], ids=["assembled", "factored"])
def test_probe_rtol_matches_oracle(operator):
    """probe_rtol: the probe columns stop at 1e-7 while y keeps cg_rtol 1e-12
    and, once every probe column has stopped, finishes alone with the
    column-0 kernels (from the union-list SpMM to the CSR one); the LML and
    the gradient still agree with the oracle's estimator on the same probes
    (LML 1e-7, gradient 1e-6 relative), y^T K^{-1} y with the all-tight run
    within 1e-10, and probe_rtol = cg_rtol is bitwise the default."""
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, (v0, g0, ld0, se0) = _union_oracle(33)
    c = gu.ctx()
    c.set_option("union_spmm", 1)
    x, y = gu.dev(w.x), gu.dev(w.y)
    base = dict(probes=33, seed=77, cg_rtol=1e-12, cg_max_iter=5000, precond=sd.PRECOND_LOWRANK,
                operator_form=operator)
    v1, g1, i1 = c.lml_grad(w.desc, x, y, w.h, sd.estimator(**base))
    assert c.get_option("last_y_tail") == 0
    v2, g2, i2 = c.lml_grad(w.desc, x, y, w.h, sd.estimator(probe_rtol=1e-7, **base))
    tail = c.get_option("last_y_tail")
    gu.log("probe_rtol 1e-7 operator=%d: iters %d (y %d, %d alone) against %d; lml %.15g tight %.15g oracle %.15g"
           % (operator, i2.cg_iters, i2.cg_iters_y, tail, i1.cg_iters, v2, v1, v0))
    assert tail > 0 and i2.cg_iters < i1.cg_iters
    assert abs(i2.yKy - i1.yKy) <= 1e-10 * abs(i1.yKy)
    assert abs(v2 - v0) <= 1e-7 * abs(v0)
    assert gu.grad_close(g2, g0, rel=1e-6).all()
    v3, g3, _ = c.lml_grad(w.desc, x, y, w.h, sd.estimator(probe_rtol=1e-12, **base))
    assert v3 == v1 and np.array_equal(g3, g1)
