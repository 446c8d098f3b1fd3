"""Edge cases of the LML path on the GPU, against the oracle.

* No points: every entry point rejects n = 0 with INVALID_ARG before any
  device work.
* Tiny and ragged point counts (1, 2, 7, 17, 33: below one 16-row tile, one
  tile plus a ragged tail, two tiles plus one row): exact mode (identity
  probes) against the dense Cholesky oracle, for both combines; the
  preconditioned estimator with the assembled and the factored operator
  against the oracle's own estimator on the same probes, with the CSR and
  with the union-list SpMM; and a population of one member against the
  single evaluation, bitwise (assembled operator; a population with the
  factored operator is rejected before any device work)."""
import numpy as np
import pytest

from oracle import estimators as es
from oracle import gp
from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

TINY = [1, 2, 7, 17, 33]


def _points(n, combine, seed):
    w = wl.random_small(max(n, 2), 2, 2, 2, seed, combine=combine, per_row=8.0, noise_var=1e-2)
    return w, w.x[:n].copy(), w.y[:n].copy()


def test_no_points_rejected():
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, x, y = _points(5, 1, 3)
    c = gu.ctx()
    x0, y0 = gu.dev(x)[:0], gu.dev(y)[:0]
    gu.log("n = 0 rejected")
    for call in (lambda: c.lml(w.desc, x0, y0, w.h),
                 lambda: c.lml_grad(w.desc, x0, y0, w.h),
                 lambda: c.kernel_assemble(w.desc, x0, w.h),
                 lambda: c.lml_grad_batched(w.desc, x0, y0, w.h[None, :])):
        with pytest.raises(sd.SdgpError) as e:
            call()
        assert e.value.status == 1


@pytest.mark.parametrize("combine", [0, 1], ids=["product", "sum"])
@pytest.mark.parametrize("n", TINY)
def test_tiny_exact_matches_oracle(n, combine):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, x, y = _points(n, combine, 40 + n)
    gu.log("tiny exact n=%d combine=%d" % (n, combine))
    c = gu.ctx()
    v, g, info = c.lml_grad(w.desc, gu.dev(x), gu.dev(y), w.h, sd.exact_estimator())
    v0, g0 = gp.lml_grad(w.desc, w.h, x, y)
    gu.log("  gpu %.15g oracle %.15g iters %d" % (v, v0, info.cg_iters))
    assert abs(v - v0) <= gu.LML_REL * abs(v0) + 1e-12
    assert gu.grad_close(g, g0).all()


@pytest.mark.parametrize("operator", [0, 1], ids=["assembled", "factored"])
@pytest.mark.parametrize("n", TINY)
def test_tiny_preconditioned_matches_oracle_estimator(n, operator):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w, x, y = _points(n, 1, 60 + n)
    P, seed = 4, 77
    gu.log("tiny preconditioned n=%d operator=%d" % (n, operator))
    c = gu.ctx()
    est = sd.estimator(probes=P, seed=seed, cg_rtol=1e-12, cg_max_iter=1000, precond=sd.PRECOND_LOWRANK,
                       operator_form=operator)
    v, g, info = c.lml_grad(w.desc, gu.dev(x), gu.dev(y), w.h, est)
    v0, g0, _, _ = es.preconditioned_lml_grad(w.desc, w.h, x, y, seed, P, 400)
    gu.log("  gpu %.15g oracle %.15g iters %d" % (v, v0, info.cg_iters))
    assert abs(v - v0) <= 1e-7 * abs(v0) + 1e-10
    assert gu.grad_close(g, g0, rel=1e-6).all()
    if operator == 0:
        vb, gb, st, infos = c.lml_grad_batched(w.desc, gu.dev(x), gu.dev(y), w.h[None, :], est)
        assert int(st[0]) == sd.OK
        assert vb[0] == v
        assert np.array_equal(gb[0], g)
    else:
        # populations reject the factored operator on the host, before any
        # device work (an earlier version of that path met a device fault
        # whose cause is not shown)
        with pytest.raises(sd.SdgpError) as e:
            c.lml_grad_batched(w.desc, gu.dev(x), gu.dev(y), w.h[None, :], est)
        assert e.value.status == sd.INVALID_ARG
    # the union-list SpMM (automatic only from 65536 points) on the same
    # tiny and ragged groups
    c.set_option("union_spmm", 1)
    vu, gu_, _ = c.lml_grad(w.desc, gu.dev(x), gu.dev(y), w.h, est)
    c.set_option("union_spmm", -1)
    assert abs(vu - v0) <= 1e-7 * abs(v0) + 1e-10
    assert gu.grad_close(gu_, g0, rel=1e-6).all()


def test_workspace_cap_gives_oom():
    """A context whose workspace_cap is below what the call needs fails with
    OOM before allocating past the cap, and works again once the cap is
    lifted (same result as a fresh context)."""
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    w = wl.random_small(3000, 3, 4, 2, 5, combine=1, per_row=20.0, noise_var=1e-2)
    est = sd.estimator(probes=8, seed=3, cg_rtol=1e-10, cg_max_iter=2000, precond=sd.PRECOND_LOWRANK)
    gu.log("workspace cap -> OOM")
    x, y = gu.dev(w.x), gu.dev(w.y)
    ref = gu.ctx()
    v0, g0, _ = ref.lml_grad(w.desc, x, y, w.h, est)
    c = gu.ctx()
    c.set_option("workspace_cap", 1 << 20)
    with pytest.raises(sd.SdgpError) as e:
        c.lml_grad(w.desc, x, y, w.h, est)
    assert e.value.status == sd.OOM
    assert "workspace_cap" in str(e.value)
    c.set_option("workspace_cap", 0)
    v1, g1, _ = c.lml_grad(w.desc, x, y, w.h, est)
    assert v1 == v0 and np.array_equal(g1, g0)
    with pytest.raises(sd.SdgpError):
        c.set_option("workspace_cap", -1)


def test_assemble_capacity_checked():
    """sdgp_kernel_assemble_sorted writes the caller's arrays directly: with
    too little capacity it returns CAPACITY, reports the count, writes
    row_ptr and leaves col / val / perm untouched; with enough it returns
    the oracle's matrix (in the returned order) and row_ptr ends at the
    count."""
    gu.need_gpu()
    import ctypes as C
    import torch
    import paper_2205_09070_amd as sd
    from paper_2205_09070_amd import _lib
    from oracle import kernel as okn
    w = wl.random_small(1500, 3, 4, 2, 8, combine=1, per_row=20.0, noise_var=1e-2)
    c = gu.ctx()
    x = gu.dev(w.x)
    n = w.x.shape[0]
    nnz = c.kernel_nnz(w.desc, x, w.h)
    gu.log("assemble capacity: n=%d nnz=%d" % (n, nnz))
    d = _lib.desc_of(w.desc)
    hh = np.ascontiguousarray(w.h, dtype=np.float64)
    dev = x.device
    for cap in (nnz - 1, nnz):
        row_ptr = torch.full((n + 1,), -7, dtype=torch.int64, device=dev)
        col = torch.full((nnz,), -5, dtype=torch.int32, device=dev)
        val = torch.full((nnz,), -3.0, dtype=torch.float64, device=dev)
        perm = torch.full((n,), -9, dtype=torch.int32, device=dev)
        out = C.c_int64(0)
        st = c.lib.sdgp_kernel_assemble_sorted(
            c.h, C.byref(d), C.c_void_p(x.data_ptr()), n, hh.ctypes.data_as(C.c_void_p), 1,
            C.c_void_p(row_ptr.data_ptr()), C.c_void_p(col.data_ptr()), C.c_void_p(val.data_ptr()),
            C.c_void_p(perm.data_ptr()), cap, C.byref(out))
        torch.cuda.synchronize()
        assert out.value == nnz
        if cap < nnz:
            assert st == sd.CAPACITY
            assert (col == -5).all() and (val == -3.0).all() and (perm == -9).all()
            assert int(row_ptr[n]) == nnz
            continue
        assert st == sd.OK
        rp = row_ptr.cpu().numpy()
        assert rp[0] == 0 and rp[-1] == nnz and (np.diff(rp) >= 1).all()
        p = perm.cpu().numpy()
        assert np.array_equal(np.sort(p), np.arange(n))
        ix = np.ix_(p, p)
        K = okn.kernel_matrix(w.desc, w.h, w.x)[ix]
        pat = okn.pattern(w.desc, w.h, w.x)[ix]
        bnd = okn.boundary_pairs(w.desc, w.h, w.x)[ix]
        cc, vv = col.cpu().numpy(), val.cpu().numpy()
        rows = np.repeat(np.arange(n), np.diff(rp))
        gpat = np.zeros((n, n), dtype=bool)
        gpat[rows, cc] = True
        assert not ((gpat != pat) & ~bnd).any()
        Kg = np.zeros((n, n))
        Kg[rows, cc] = vv
        both = gpat & pat
        assert gu.check_k_entries(Kg[both], K[both], np.abs(np.diag(K)).max()).all()
