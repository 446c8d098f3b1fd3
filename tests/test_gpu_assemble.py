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


def test_assemble_crowded_cells():
    """Cells holding more rows than one row group of the row kernels (64):
    600 points in a cube of side 0.004 (at most 8 cells, so one holds at
    least 75) over 300 uniform points, both combinations."""
    gu.need_gpu()
    rng = np.random.default_rng(12)
    x = np.concatenate([0.5 + 0.004 * rng.random((600, 3)), rng.random((300, 3))])
    for comb in (0, 1):
        gu.log("assemble crowded cells, combine %d" % comb)
        desc = wl.KernelDesc(3, 2, 2, 0, comb)
        h = wl.pack_hyper(desc, 1.0, 0.08, np.full((2, 2), 0.7), np.ones((2, 2)),
                          np.full((2, 2), 0.2), rng.random((2, 2, 3)), 1e-4)
        c = gu.ctx()
        n = x.shape[0]
        rp, col, val = c.kernel_assemble(desc, gu.dev(x), h)
        rpn, coln, valn, S = gu.csr_to_host(rp, col, val, n)
        K = kn.kernel_matrix(desc, h, x)
        pat = kn.pattern(desc, h, x)
        bnd = kn.boundary_pairs(desc, h, x)
        gpat = np.zeros((n, n), dtype=bool)
        gpat[np.repeat(np.arange(n), np.diff(rpn)), coln] = True
        assert not ((gpat != pat) & ~bnd).any()
        for a in range(n):
            assert np.all(np.diff(coln[rpn[a]:rpn[a + 1]]) > 0)
        both = gpat & pat
        assert np.all(gu.check_k_entries(S.toarray()[both], K[both], np.abs(np.diag(K)).max()))


def test_assemble_cells_beyond_the_wavefront_merge():
    """Bump-covered cells whose runs exceed what one wavefront merges in
    LDS (512 runs): 6000 points in 3-D, 5 bump functions of 300 small balls
    (radii 0.3-0.6 of the core radius), so a cell covered by several
    functions carries 500-900 runs and is merged by the serial fallback,
    the others by the wavefront merge; pattern and values against the
    oracle."""
    gu.need_gpu()
    w = wl.random_small(6000, 3, 5, 300, 77, per_row=14.0)
    p = wl.unpack_hyper(w.desc, w.h)
    r = np.random.default_rng(5).uniform(0.3 * p["r_core"], 0.6 * p["r_core"], size=(5, 300))
    h = wl.pack_hyper(w.desc, p["sigma2"], p["r_core"], p["a"], p["beta"], r, p["c"], p["noise_var"])
    gu.log("assemble beyond the wavefront merge n=%d n1=5 n2=300" % w.x.shape[0])
    c = gu.ctx()
    n = w.x.shape[0]
    rp, col, val = c.kernel_assemble(w.desc, gu.dev(w.x), h, add_noise=True)
    rpn, coln, valn, S = gu.csr_to_host(rp, col, val, n)
    K = kn.kernel_matrix(w.desc, h, w.x)
    pat = kn.pattern(w.desc, h, w.x)
    bnd = kn.boundary_pairs(w.desc, h, w.x)
    gpat = np.zeros((n, n), dtype=bool)
    gpat[np.repeat(np.arange(n), np.diff(rpn)), coln] = True
    assert not ((gpat != pat) & ~bnd).any()
    both = gpat & pat
    assert np.all(gu.check_k_entries(S.toarray()[both], K[both], np.abs(np.diag(K)).max()))


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


def _membership_band(desc, h, x, eps=1e-9, chunk=100_000):
    """(M_in, M_out)[a, i]: x_a inside some ball of bump function i with the
    balls shrunk / grown by a relative eps (pairs between the two are
    decided by rounding, and their bump values are ~0)."""
    p = kn.unpack(desc, h)
    n1 = max(desc.n1, 1)
    m_in = np.zeros((x.shape[0], n1), dtype=bool)
    m_out = np.zeros((x.shape[0], n1), dtype=bool)
    r2 = p["r"] ** 2
    for s in range(0, x.shape[0], chunk):
        xc = x[s:s + chunk]
        d2 = np.zeros((xc.shape[0], desc.n1, desc.n2))
        for k in range(desc.dim):
            d2 += (xc[:, k][:, None, None] - p["c"][None, :, :, k]) ** 2
        q = d2 / r2[None]
        m_in[s:s + chunk, :desc.n1] = (q < 1.0 - eps).any(axis=2)
        m_out[s:s + chunk, :desc.n1] = (q < 1.0 + eps).any(axis=2)
    return m_in, m_out


@pytest.mark.parametrize("make", [wl.uniform3d_100k, wl.spacetime_4d], ids=["uniform3d_n100000", "spacetime4d_n5000000"])
def test_assemble_rows_at_full_size_sampled(make):
    """Full-size assembly of the 100,000-point 3-D workload (8x4 bumps, ~100
    core entries per row) and of the 5,000,000-point 4-D space-time workload
    (32x8 bumps): for sampled rows (random, inside bump balls, first and
    last) the stored columns lie between the support predicate with the
    radii shrunk and grown by 1e-9 (evaluated over every point), and every
    stored value matches the oracle's kernel entry."""
    gu.need_gpu()
    w = make()
    n = w.x.shape[0]
    eps = 1e-9
    gu.log("assemble sampled rows: %s n=%d" % (w.name, n))
    m_in, m_out = _membership_band(w.desc, w.h, w.x, eps)
    c = gu.ctx()
    rp, col, val = c.kernel_assemble(w.desc, gu.dev(w.x), w.h)
    rp = rp.cpu().numpy()
    rng = np.random.default_rng(1)
    in_bump = np.nonzero(m_in.any(axis=1))[0]
    rows = np.concatenate([rng.choice(n, 16, replace=False), rng.choice(in_bump, 8, replace=False), [0, n - 1]])
    p = kn.unpack(w.desc, w.h)
    rc2 = p["r_core"] ** 2
    inb = np.nonzero(m_out.any(axis=1))[0]      # the few points inside any (grown) ball
    for a in rows:
        lo, hi = rp[a], rp[a + 1]
        gc = col[lo:hi].cpu().numpy()
        gv = val[lo:hi].cpu().numpy()
        assert np.all(np.diff(gc) > 0), "row %d columns not ascending" % a
        d2 = kn.pair_d2(w.x[a:a + 1], w.x)[0]
        pat_lo = d2 < rc2 * (1 - eps)
        pat_hi = d2 < rc2 * (1 + eps)
        pat_lo[inb] |= (m_in[a][None, :] & m_in[inb]).any(axis=1)
        pat_hi[inb] |= (m_out[a][None, :] & m_out[inb]).any(axis=1)
        pat_lo[a] = pat_hi[a] = True
        got = np.zeros(n, dtype=bool)
        got[gc] = True
        assert not (pat_lo & ~got).any(), "row %d misses entries" % a
        assert not (got & ~pat_hi).any(), "row %d stores entries outside the support" % a
        krow = kn.kernel_cross(w.desc, w.h, w.x[a:a + 1], w.x[gc])[0]
        krow[np.searchsorted(gc, a)] += p["noise_var"]
        assert np.all(gu.check_k_entries(gv, krow, 2.0)), "row %d values" % a
    gu.log("  nnz=%d (%.1f per row)" % (rp[-1], rp[-1] / n))
