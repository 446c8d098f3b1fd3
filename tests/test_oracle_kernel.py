"""Pins of the oracle's kernel (Section 2.2) against the printed formulas,
textbook values, brute force and invariants."""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import kernel as kn
from paper_2205_09070_amd import workloads as wl
from tests import mp_literal as ml

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_kstat_constant_matches_printed_prefactor():
    g = _gold("textbook_constants.json")["kstat_constant"]["value"]
    assert kn.C_KSTAT == pytest.approx(g, rel=1e-16)
    assert kn.core_psi(np.array([0.0]), kn.CORE_KSTAT, 2)[0] == pytest.approx(g, rel=1e-15)


@pytest.mark.parametrize("u", [1e-9, 1e-3, 0.1, 0.25, 0.5, 0.6, 0.7, 0.71, 0.72, 0.75,
                               0.8, 0.9, 0.95, 0.99, 0.999, 0.9999, 0.999999])
def test_kstat_value_vs_printed_formula(u):
    # eq:kstat evaluated literally at 40 digits vs the oracle's series/log form
    ref = float(ml.kstat(u))
    got = float(kn.core_psi(np.array([u]), kn.CORE_KSTAT, 2)[0])
    assert abs(got - ref) <= 2e-15 * abs(ref) + 1e-300


@pytest.mark.parametrize("u", [0.05, 0.25, 0.5, 0.7, 0.72, 0.9, 0.99, 0.999])
def test_kstat_derivative_vs_numerical_derivative_of_printed_formula(u):
    ref = float(mp.diff(ml.kstat, mp.mpf(u)))
    got = float(kn.core_dpsi(np.array([u]), kn.CORE_KSTAT, 2)[0])
    assert abs(got - ref) <= 1e-14 * abs(ref)


def test_kstat_support_and_limits():
    u = np.array([1.0, 1.0000001, 2.0, 10.0])
    assert np.all(kn.core_psi(u, kn.CORE_KSTAT, 2) == 0.0)
    assert np.all(kn.core_dpsi(u, kn.CORE_KSTAT, 2) == 0.0)
    assert kn.core_dpsi(np.array([0.0]), kn.CORE_KSTAT, 2)[0] == 0.0


@pytest.mark.parametrize("dim", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("u", [0.0, 0.1, 0.3, 0.5, 0.77, 0.95])
def test_wendland_vs_integral_construction(dim, u):
    # Wendland's construction psi(u) = (l+1)(l+2) int_u^1 t (1-t)^l dt
    ell = dim // 2 + 2
    ref = float(ml.wendland_integral(u, ell))
    got = float(kn.core_psi(np.array([u]), kn.CORE_WENDLAND_C2, dim)[0])
    assert got == pytest.approx(ref, rel=1e-14, abs=1e-300)
    dref = float(mp.diff(lambda t: ml.wendland_integral(t, ell), mp.mpf(u))) if u > 0 else 0.0
    dgot = float(kn.core_dpsi(np.array([u]), kn.CORE_WENDLAND_C2, dim)[0])
    assert dgot == pytest.approx(dref, rel=1e-12, abs=1e-14)


def test_wendland_textbook_values():
    g = _gold("textbook_constants.json")["wendland_c2_tables"]
    p = lambda u, d: float(kn.core_psi(np.array([u]), kn.CORE_WENDLAND_C2, d)[0])
    assert p(0.5, 3) == g["l3_r_half"]
    assert p(0.25, 3) == g["l3_r_quarter"]
    assert p(0.5, 4) == g["l4_r_half"]
    assert p(0.0, 3) == 1.0 and p(1.0, 3) == 0.0


def test_bump_value_vs_printed_formula():
    rng = np.random.default_rng(3)
    desc = wl.KernelDesc(dim=3, n1=2, n2=3)
    x = rng.random((40, 3))
    a = rng.uniform(0.3, 1.2, (2, 3)); b = rng.uniform(0.2, 3.0, (2, 3))
    r = rng.uniform(0.2, 0.5, (2, 3)); c = rng.random((2, 3, 3))
    h = wl.pack_hyper(desc, 1.0, 0.1, a, b, r, c, 1e-4)
    F, M = kn.bump_F(desc, h, x)
    for p in range(x.shape[0]):
        ref = ml.F_row(desc, list(h), list(x[p]))
        for i in range(2):
            assert F[p, i] == pytest.approx(float(ref[i]), rel=1e-13, abs=1e-300)
            inside = any(sum((x[p, k] - c[i, j, k]) ** 2 for k in range(3)) < r[i, j] ** 2
                         for j in range(3))
            assert M[p, i] == inside


def test_bump_centre_value_and_shape_limits():
    desc = wl.KernelDesc(dim=2, n1=1, n2=1)
    c = np.array([[[0.4, 0.6]]])
    for beta in (0.5, 1.0, 7.0):
        h = wl.pack_hyper(desc, 1.0, 0.1, [[0.8]], [[beta]], [[0.2]], c, 1e-4)
        F, _ = kn.bump_F(desc, h, np.array([[0.4, 0.6]]))
        assert F[0, 0] == 0.8        # peak height is a (paper form with +beta)
    # beta -> 0: the bump tends to a flat indicator of height a inside the ball
    h = wl.pack_hyper(desc, 1.0, 0.1, [[0.8]], [[1e-12]], [[0.2]], c, 1e-4)
    F, _ = kn.bump_F(desc, h, np.array([[0.5, 0.6], [0.4, 0.79], [0.4, 0.81]]))
    assert F[0, 0] == pytest.approx(0.8, rel=1e-10)
    assert F[1, 0] == pytest.approx(0.8, rel=1e-9)
    assert F[2, 0] == 0.0


@pytest.mark.parametrize("t", range(6))
def test_bump_derivatives_vs_numerical(t):
    desc = wl.KernelDesc(dim=3, n1=1, n2=1)
    base = [0.7, 1.3, 0.3, 0.45, 0.5, 0.55]     # a, beta, r, c0, c1, c2
    x = np.array([[0.5, 0.6, 0.4], [0.3, 0.5, 0.7], [0.55, 0.35, 0.6]])

    def f_of(v, p):
        hh = list(base)
        hh[t] = v
        return ml.bump_f(list(x[p]), hh[3:], hh[2], hh[0], hh[1])

    h = np.array([1.0, 0.1] + base + [1e-4])
    dF = kn.bump_dF(desc, h, x)
    for p in range(x.shape[0]):
        ref = float(mp.diff(lambda v: f_of(v, p), mp.mpf(base[t])))
        assert dF[p, 0, 0, t] == pytest.approx(ref, rel=1e-12, abs=1e-15)


CASES = [
    (2, kn.CORE_KSTAT, kn.COMBINE_PRODUCT), (2, kn.CORE_KSTAT, kn.COMBINE_SUM),
    (2, kn.CORE_WENDLAND_C2, kn.COMBINE_SUM), (3, kn.CORE_WENDLAND_C2, kn.COMBINE_PRODUCT),
    (3, kn.CORE_WENDLAND_C2, kn.COMBINE_SUM), (4, kn.CORE_WENDLAND_C2, kn.COMBINE_SUM),
]


def _case(dim, core, comb, n=28, seed=11):
    w = wl.random_small(n, dim, 2, 2, seed, core=core, combine=comb, per_row=6.0)
    return w


@pytest.mark.parametrize("dim,core,comb", CASES)
def test_dense_K_brute_force_vs_printed_formulas(dim, core, comb):
    w = _case(dim, core, comb)
    K = kn.kernel_matrix(w.desc, w.h, w.x, add_noise=False)
    h = list(w.h)
    scale = np.abs(np.diag(K)).max()
    for a in range(w.x.shape[0]):
        for b in range(a, w.x.shape[0]):
            ref = float(ml.k_entry(w.desc, h, list(w.x[a]), list(w.x[b])))
            assert abs(K[a, b] - ref) <= 1e-14 * abs(ref) + 1e-15 * scale


@pytest.mark.parametrize("dim,core,comb", CASES)
def test_pattern_brute_force_and_structure(dim, core, comb):
    w = _case(dim, core, comb, n=60, seed=5)
    pat = kn.pattern(w.desc, w.h, w.x)
    K = kn.kernel_matrix(w.desc, w.h, w.x, add_noise=True)
    p = kn.unpack(w.desc, w.h)
    n = w.x.shape[0]
    for a in range(n):
        for b in range(n):
            d2 = sum((w.x[a, k] - w.x[b, k]) ** 2 for k in range(dim))
            core_ab = d2 < p["r_core"] ** 2
            bump_ab = False
            for i in range(w.desc.n1):
                ina = any(sum((w.x[a, k] - p["c"][i, j, k]) ** 2 for k in range(dim)) < p["r"][i, j] ** 2
                          for j in range(w.desc.n2))
                inb = any(sum((w.x[b, k] - p["c"][i, j, k]) ** 2 for k in range(dim)) < p["r"][i, j] ** 2
                          for j in range(w.desc.n2))
                bump_ab = bump_ab or (ina and inb)
            want = a == b or ((core_ab and bump_ab) if comb == kn.COMBINE_PRODUCT else (core_ab or bump_ab))
            assert pat[a, b] == want
    # exact zeros off the pattern, bitwise symmetry, diagonal always stored
    assert np.all(K[~pat] == 0.0)
    assert np.array_equal(K, K.T)
    assert np.all(np.diag(pat))


@pytest.mark.parametrize("dim,core,comb", CASES)
def test_diagonal_formula(dim, core, comb):
    w = _case(dim, core, comb, n=50, seed=2)
    K = kn.kernel_matrix(w.desc, w.h, w.x, add_noise=True)
    F, _ = kn.bump_F(w.desc, w.h, w.x)
    p = kn.unpack(w.desc, w.h)
    psi0 = float(kn.core_psi(np.array([0.0]), core, dim)[0])
    Baa = np.sum(F * F, axis=1)
    want = p["sigma2"] * psi0 * Baa if comb == kn.COMBINE_PRODUCT else p["sigma2"] * psi0 + Baa
    assert np.allclose(np.diag(K), want + p["noise_var"], rtol=1e-15, atol=0)


@pytest.mark.parametrize("dim,core,comb", [
    (2, kn.CORE_KSTAT, kn.COMBINE_PRODUCT), (2, kn.CORE_KSTAT, kn.COMBINE_SUM),
    (3, kn.CORE_WENDLAND_C2, kn.COMBINE_SUM), (3, kn.CORE_WENDLAND_C2, kn.COMBINE_PRODUCT),
    (4, kn.CORE_WENDLAND_C2, kn.COMBINE_SUM)])
def test_positive_semidefinite(dim, core, comb):
    # products and sums of positive definite kernels stay positive (semi)definite
    w = wl.random_small(400, dim, 3, 2, 9, core=core, combine=comb, per_row=30.0)
    K = kn.kernel_matrix(w.desc, w.h, w.x, add_noise=False)
    lam = np.linalg.eigvalsh(K)
    assert lam.min() >= -1e-12 * max(1.0, lam.max())


def test_support_zeros_beyond_every_radius():
    w = wl.random_small(200, 3, 2, 2, 4, per_row=8.0)
    K = kn.kernel_matrix(w.desc, w.h, w.x, add_noise=False)
    p = kn.unpack(w.desc, w.h)
    d2 = kn.pair_d2(w.x, w.x)
    _, M = kn.bump_F(w.desc, w.h, w.x)
    share = (M.astype(int) @ M.T.astype(int)) > 0
    far = (d2 >= p["r_core"] ** 2) & ~share
    assert np.all(K[far] == 0.0)


def test_boundary_pairs_flags_near_ties():
    desc = wl.KernelDesc(dim=1, n1=1, n2=1)
    h = wl.pack_hyper(desc, 1.0, 0.25, [[1.0]], [[1.0]], [[0.01]], [[[5.0]]], 1e-4)
    x = np.array([[0.0], [0.25 * (1 + 1e-14)], [0.5 + 0.25]])
    bp = kn.boundary_pairs(desc, h, x)
    assert bp[0, 1] and bp[1, 0]
    assert not bp[0, 2]


def test_csr_roundtrip():
    w = _case(2, kn.CORE_WENDLAND_C2, kn.COMBINE_SUM, n=40)
    K = kn.kernel_matrix(w.desc, w.h, w.x)
    pat = kn.pattern(w.desc, w.h, w.x)
    rp, col, val = kn.to_csr(K, pat)
    D = np.zeros_like(K)
    for a in range(K.shape[0]):
        cs = col[rp[a]:rp[a + 1]]
        assert np.all(np.diff(cs) > 0)
        D[a, cs] = val[rp[a]:rp[a + 1]]
    assert np.array_equal(D, K)
    assert math.isclose(rp[-1], pat.sum())
