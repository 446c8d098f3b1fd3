"""GPU assembly parity: the CSR pattern bit-exact against the oracle's
support predicate (boundary pairs excepted), stored values within 1e-13
relative (or 1e-15 of the largest diagonal), bitwise symmetry, canonical
column order."""
import numpy as np
import pytest

from oracle import kernel as kn
from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

CASES = [
    ("2d-kstat-product", lambda: wl.small_2d(2000, 0, core=1, combine=0)),
    ("2d-kstat-sum", lambda: wl.small_2d(2000, 0, core=1, combine=1)),
    ("2d-wendland-sum", lambda: wl.small_2d(2000, 0, core=0, combine=1)),
    ("2d-wendland-product", lambda: wl.small_2d(2000, 0, core=0, combine=0)),
    ("3d-sum", lambda: wl.random_small(3000, 3, 4, 3, 7, per_row=25.0)),
    ("3d-product", lambda: wl.random_small(3000, 3, 4, 3, 7, combine=0, per_row=25.0)),
    ("4d-sum", lambda: wl.random_small(2500, 4, 3, 2, 3, per_row=20.0)),
    ("1d-sum", lambda: wl.random_small(700, 1, 2, 2, 5, per_row=9.0)),
    ("3d-manybumps", lambda: wl.random_small(1500, 3, 40, 2, 9, per_row=15.0)),
    ("2d-nobumps", lambda: wl.random_small(800, 2, 0, 1, 2, per_row=10.0)),
]


def _oracle_csr(w, add_noise=True):
    K = kn.kernel_matrix(w.desc, w.h, w.x, add_noise=add_noise)
    pat = kn.pattern(w.desc, w.h, w.x)
    bnd = kn.boundary_pairs(w.desc, w.h, w.x)
    return K, pat, bnd


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_assemble_matches_oracle(name, make):
    gu.need_gpu()
    w = make()
    gu.log("assemble parity %s n=%d dim=%d n1=%d" % (name, w.x.shape[0], w.desc.dim, w.desc.n1))
    c = gu.ctx()
    x = gu.dev(w.x)
    n = w.x.shape[0]
    rp, col, val = c.kernel_assemble(w.desc, x, w.h, add_noise=True)
    rp, col, val, S = gu.csr_to_host(rp, col, val, n)
    K, pat, bnd = _oracle_csr(w)
    # canonical: ascending, unique columns; diagonal present
    for a in range(n):
        cs = col[rp[a]:rp[a + 1]]
        assert np.all(np.diff(cs) > 0), "row %d not ascending" % a
        assert a in set(cs.tolist())
    gpat = np.zeros((n, n), dtype=bool)
    rows = np.repeat(np.arange(n), np.diff(rp))
    gpat[rows, col] = True
    diff = (gpat != pat) & ~bnd
    assert not diff.any(), "pattern differs at %d pairs" % diff.sum()
    both = gpat & pat
    Kg = S.toarray()
    scale = np.abs(np.diag(K)).max()
    ok = gu.check_k_entries(Kg[both], K[both], scale)
    assert ok.all(), "values differ at %d entries (max err %g)" % ((~ok).sum(), np.abs(Kg[both] - K[both]).max())
    assert np.array_equal(Kg, Kg.T), "GPU K not bitwise symmetric"


def test_assemble_without_noise_and_sorted_order():
    gu.need_gpu()
    w = wl.random_small(1200, 3, 3, 2, 11, per_row=15.0)
    gu.log("assemble sorted order n=1200")
    c = gu.ctx()
    x = gu.dev(w.x)
    n = w.x.shape[0]
    rp, col, val = c.kernel_assemble(w.desc, x, w.h, add_noise=False)
    _, _, _, S = gu.csr_to_host(rp, col, val, n)
    rp2, col2, val2, perm = c.kernel_assemble(w.desc, x, w.h, add_noise=False, sorted_order=True)
    _, _, _, S2 = gu.csr_to_host(rp2, col2, val2, n)
    p = perm.cpu().numpy()
    assert np.array_equal(np.sort(p), np.arange(n))
    # sorted-order matrix is P K P^T with the same stored values
    Kp = S.toarray()[np.ix_(p, p)]
    assert np.array_equal(Kp, S2.toarray())
    K = kn.kernel_matrix(w.desc, w.h, w.x, add_noise=False)
    scale = np.abs(np.diag(K)).max()
    ok = gu.check_k_entries(S.toarray(), K, scale)
    assert ok.all()


@pytest.mark.parametrize("n", [1, 2, 3, 65, 129])
def test_assemble_tiny_and_ragged(n):
    gu.need_gpu()
    gu.log("assemble tiny n=%d" % n)
    w = wl.random_small(max(n, 2), 2, 1, 2, 17, per_row=30.0)
    x = w.x[:n]
    c = gu.ctx()
    rp, col, val = c.kernel_assemble(w.desc, gu.dev(x), w.h)
    _, _, _, S = gu.csr_to_host(rp, col, val, n)
    K = kn.kernel_matrix(w.desc, w.h, x)
    pat = kn.pattern(w.desc, w.h, x)
    gpat = S.toarray() != 0
    Kg = S.toarray()
    assert np.all(gu.check_k_entries(Kg, K, np.abs(np.diag(K)).max()))
    assert int(rp.cpu().numpy()[-1]) == int(pat.sum())
    del gpat


def test_assemble_duplicate_points_and_degenerate_axis():
    gu.need_gpu()
    gu.log("assemble duplicates / flat axis")
    rng = np.random.default_rng(4)
    base = rng.random((200, 3))
    x = np.concatenate([base, base[:50]])        # exact duplicates
    x[:, 2] = 0.5                                # zero extent on one axis
    desc = wl.KernelDesc(3, 2, 2, 0, 1)
    h = wl.pack_hyper(desc, 1.0, 0.08, np.full((2, 2), 0.7), np.ones((2, 2)),
                      np.full((2, 2), 0.15), rng.random((2, 2, 3)), 1e-4)
    c = gu.ctx()
    n = x.shape[0]
    rp, col, val = c.kernel_assemble(desc, gu.dev(x), h)
    _, _, _, S = gu.csr_to_host(rp, col, val, n)
    K = kn.kernel_matrix(desc, h, x)
    pat = kn.pattern(desc, h, x)
    bnd = kn.boundary_pairs(desc, h, x)
    gpat = np.zeros((n, n), dtype=bool)
    rpn = rp.cpu().numpy()
    gpat[np.repeat(np.arange(n), np.diff(rpn)), col.cpu().numpy()] = True
    assert not ((gpat != pat) & ~bnd).any()
    assert np.all(gu.check_k_entries(S.toarray(), K, np.abs(np.diag(K)).max()))


def test_assemble_rows_at_one_million_points_sampled():
    """Full-size (1,000,000 points in [0,1)^3, 16x4 bumps) assembly in the
    configuration the benchmark times: sampled rows compared one by one with
    the oracle's kernel row."""
    gu.need_gpu()
    w = wl.uniform3d_1m()
    gu.log("assemble sampled rows at n=%d" % w.x.shape[0])
    c = gu.ctx()
    x = gu.dev(w.x)
    rp, col, val = c.kernel_assemble(w.desc, x, w.h)
    rp = rp.cpu().numpy()
    n = w.x.shape[0]
    rng = np.random.default_rng(0)
    _, M = kn.bump_F(w.desc, w.h, w.x)
    in_bump = np.nonzero(M.any(axis=1))[0]
    rows = np.concatenate([rng.choice(n, 24, replace=False), rng.choice(in_bump, 8, replace=False), [0, n - 1]])
    p = kn.unpack(w.desc, w.h)
    for a in rows:
        lo, hi = rp[a], rp[a + 1]
        gc = col[lo:hi].cpu().numpy()
        gv = val[lo:hi].cpu().numpy()
        krow = kn.kernel_cross(w.desc, w.h, w.x[a:a + 1], w.x)[0]
        krow[a] += p["noise_var"]
        d2 = kn.pair_d2(w.x[a:a + 1], w.x)[0]
        share = (M[a][None, :] & M).any(axis=1)
        pat = (d2 < p["r_core"] ** 2) | share
        pat[a] = True
        assert np.array_equal(gc, np.nonzero(pat)[0]), "row %d pattern" % a
        assert np.all(gu.check_k_entries(gv, krow[gc], 2.0)), "row %d values" % a
    nnz = rp[-1]
    gu.log("  nnz=%d (%.1f per row)" % (nnz, nnz / n))
    assert 60 < nnz / n < 200
