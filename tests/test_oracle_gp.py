"""Pins of the oracle's LML (eqn:log_likelihood), gradient and posterior
(eq:pred_distr): multi-precision LU on tiny inputs, closed forms, finite
differences."""
import mpmath as mp
import numpy as np
import pytest

from oracle import gp
from oracle import kernel as kn
from paper_2205_09070_amd import workloads as wl
from tests import mp_literal as ml

X3 = np.array([[0.30, 0.40], [0.33, 0.44], [0.32, 0.40]])
Y3 = np.array([1.0, -0.5, 0.25])


def _three_point(core, comb):
    desc = wl.KernelDesc(2, 1, 1, core, comb)
    h = wl.pack_hyper(desc, 1.0, 0.1, [[0.8]], [[1.0]], [[0.1]], [[[0.31, 0.41]]], 1e-4)
    return desc, h


@pytest.mark.parametrize("core,comb", [(1, 0), (1, 1), (0, 0), (0, 1)])
def test_three_point_lml_vs_multiprecision_lu(core, comb):
    desc, h = _three_point(core, comb)
    ref = float(ml.lml(desc, list(h), [list(r) for r in X3], list(Y3)))
    got, _, _, _ = gp.lml(desc, h, X3, Y3)
    assert got == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("core,comb", [(1, 0), (0, 1)])
def test_three_point_gradient_vs_multiprecision_differences(core, comb):
    # d lnL / d theta by central differences of the 40-digit literal LML
    desc, h = _three_point(core, comb)
    _, g = gp.lml_grad(desc, h, X3, Y3)
    X = [list(r) for r in X3]
    for t in range(len(h)):
        def f(v):
            hh = [mp.mpf(float(q)) for q in h]
            hh[t] = v
            return ml.lml(desc, hh, X, list(Y3))
        step = mp.mpf(10) ** -12 * max(1.0, abs(h[t]))
        ref = (f(mp.mpf(h[t]) + step) - f(mp.mpf(h[t]) - step)) / (2 * step)
        assert g[t] == pytest.approx(float(ref), rel=1e-10, abs=1e-10)


def test_diagonal_only_closed_form():
    # points farther apart than every support and outside every bump:
    # A is diagonal and ln L = -1/2 sum y^2 / A_aa - 1/2 sum ln A_aa
    desc = wl.KernelDesc(2, 1, 2, kn.CORE_WENDLAND_C2, kn.COMBINE_SUM)
    x = np.array([[0.1, 0.1], [0.9, 0.1], [0.1, 0.9], [0.9, 0.9], [0.5, 0.5]])
    y = np.array([0.3, -1.2, 0.7, 0.05, 2.0])
    h = wl.pack_hyper(desc, 1.7, 0.2, [[0.9, 0.6]], [[1.0, 1.0]], [[0.05, 0.05]],
                      [[[0.3, 0.7], [0.7, 0.3]]], 0.25)
    A = kn.kernel_matrix(desc, h, x)
    assert np.count_nonzero(A - np.diag(np.diag(A))) == 0
    Aii = 1.7 + 0.25
    want = -0.5 * np.sum(y * y) / Aii - 0.5 * 5 * np.log(Aii)
    val, g = gp.lml_grad(desc, h, x, y)
    assert val == pytest.approx(want, rel=1e-15)
    dn = 0.5 * np.sum(y * y) / Aii ** 2 - 0.5 * 5 / Aii
    assert g[-1] == pytest.approx(dn, rel=1e-14)
    assert g[0] == pytest.approx(dn, rel=1e-14)     # d A_aa / d sigma2 = psi(0) = 1
    assert g[1] == 0.0


def test_two_by_two_closed_form():
    desc = wl.KernelDesc(1, 1, 1, kn.CORE_WENDLAND_C2, kn.COMBINE_PRODUCT)
    x = np.array([[0.40], [0.46]])
    y = np.array([0.8, -0.3])
    h = wl.pack_hyper(desc, 1.3, 0.2, [[0.9]], [[0.7]], [[0.3]], [[[0.45]]], 1e-2)
    A = kn.kernel_matrix(desc, h, x)
    a, b, d = A[0, 0], A[0, 1], A[1, 1]
    det = a * d - b * b
    quad = (d * y[0] ** 2 - 2 * b * y[0] * y[1] + a * y[1] ** 2) / det
    val, _, logdet, _ = gp.lml(desc, h, x, y)
    assert logdet == pytest.approx(np.log(det), rel=1e-14)
    assert val == pytest.approx(-0.5 * quad - 0.5 * np.log(det), rel=1e-14)


@pytest.mark.parametrize("dim,core,comb", [(2, 1, 0), (2, 1, 1), (3, 0, 1), (3, 0, 0), (4, 0, 1)])
def test_gradient_vs_central_differences(dim, core, comb):
    w = wl.random_small(70, dim, 2, 2, 21, core=core, combine=comb, per_row=10.0)
    _, g = gp.lml_grad(w.desc, w.h, w.x, w.y)
    for t in range(len(w.h)):
        st = 1e-6 * max(abs(w.h[t]), 1e-3)
        hp = w.h.copy(); hp[t] += st
        hm = w.h.copy(); hm[t] -= st
        fd = (gp.lml(w.desc, hp, w.x, w.y)[0] - gp.lml(w.desc, hm, w.x, w.y)[0]) / (2 * st)
        assert g[t] == pytest.approx(fd, rel=2e-5, abs=1e-6 * max(1.0, np.abs(g).max()))


def test_posterior_far_point_is_prior():
    w = wl.random_small(80, 2, 1, 2, 8, per_row=8.0)
    x0 = np.array([[5.0, 5.0]])
    m, v = gp.posterior_mean_var(w.desc, w.h, w.x, w.y, x0)
    assert m[0] == 0.0
    assert v[0] == pytest.approx(w.h[0] * 1.0, rel=1e-15)   # sigma2 psi(0), no bump there


def test_posterior_interpolates_with_tiny_noise():
    w = wl.random_small(60, 2, 1, 2, 8, per_row=8.0, noise_var=1e-12)
    m, v = gp.posterior_mean_var(w.desc, w.h, w.x, w.y, w.x[:5])
    assert np.allclose(m, w.y[:5], atol=1e-6)
    assert np.all(v >= -1e-9) and np.all(v < 1e-6)


def test_posterior_variance_bounds():
    w = wl.random_small(120, 3, 2, 2, 12, per_row=10.0)
    rng = np.random.default_rng(0)
    x0 = rng.random((30, 3))
    m, v = gp.posterior_mean_var(w.desc, w.h, w.x, w.y, x0)
    prior = np.diag(kn.kernel_cross(w.desc, w.h, x0, x0))
    assert np.all(v <= prior + 1e-14) and np.all(v >= -1e-12)
