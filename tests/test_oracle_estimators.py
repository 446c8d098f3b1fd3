"""Pins of the oracle's probe generator, SLQ, Hutchinson and randomised
Taylor-series log-det estimators."""
import json
import os

import numpy as np
import pytest

from oracle import estimators as es
from oracle import gp
from oracle import kernel as kn
from paper_2205_09070_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLD, "splitmix64_seed0.json")) as f:
        g = json.load(f)
    got = [int(es.splitmix64_output(g["seed"], k)) for k in range(1, 5)]
    assert got == [int(v, 16) for v in g["outputs_hex"]]


def test_rademacher_statistics_and_determinism():
    Z = es.rademacher(7, 4000, 16)
    assert set(np.unique(Z)) == {-1.0, 1.0}
    assert abs(Z.mean()) < 4 / np.sqrt(Z.size)
    C = Z.T @ Z / Z.shape[0]
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() < 5 / np.sqrt(Z.shape[0])
    assert np.array_equal(Z, es.rademacher(7, 4000, 16))
    assert not np.array_equal(Z, es.rademacher(8, 4000, 16))
    # a longer set extends a shorter one (counter-based)
    assert np.array_equal(es.rademacher(7, 100, 16), Z[:100])


def _spd_case(n=250, seed=3):
    w = wl.random_small(n, 2, 2, 2, seed, per_row=12.0, noise_var=1e-2)
    A = kn.kernel_matrix(w.desc, w.h, w.x)
    return w, A


def test_slq_identity_probes_full_lanczos_is_exact():
    w, A = _spd_case(120)
    n = A.shape[0]
    est, _ = es.slq_logdet(A, np.eye(n), n, identity=True)
    exact = np.linalg.slogdet(A)[1]
    assert est == pytest.approx(exact, rel=1e-10)


def test_slq_rademacher_unbiased_within_standard_error():
    w, A = _spd_case(300)
    Z = es.rademacher(1, A.shape[0], 200)
    est, se = es.slq_logdet(A, Z, 80)
    exact = np.linalg.slogdet(A)[1]
    assert abs(est - exact) < 4 * se


def test_lanczos_quadrature_exact_for_polynomial():
    # Gauss quadrature with m nodes is exact for degree 2m-1: check x^3 with m=2
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    A = Q @ np.diag(rng.uniform(0.5, 3.0, 30)) @ Q.T
    z = rng.standard_normal(30)
    al, be = es.lanczos(A, z, 2)
    T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    q = z / np.linalg.norm(z)
    assert np.linalg.matrix_power(T, 3)[0, 0] == pytest.approx(q @ A @ A @ A @ q, rel=1e-12)


def test_hutchinson_identity_probes_equal_exact_gradient():
    w = wl.random_small(60, 2, 2, 2, 4, per_row=8.0)
    n = w.x.shape[0]
    val, g, _, _ = es.stochastic_lml_grad(w.desc, w.h, w.x, w.y, np.eye(n), n, identity=True)
    v0, g0 = gp.lml_grad(w.desc, w.h, w.x, w.y)
    assert val == pytest.approx(v0, rel=1e-9)
    assert np.allclose(g, g0, rtol=1e-9, atol=1e-9 * np.abs(g0).max())


def test_hutchinson_rademacher_unbiased():
    w = wl.random_small(80, 2, 1, 2, 6, per_row=8.0, noise_var=1e-2)
    n = w.x.shape[0]
    _, g0 = gp.lml_grad(w.desc, w.h, w.x, w.y)
    runs = []
    for s in range(12):
        Z = es.rademacher(100 + s, n, 40)
        runs.append(es.stochastic_lml_grad(w.desc, w.h, w.x, w.y, Z, 60)[1])
    runs = np.array(runs)
    mean = runs.mean(axis=0)
    se = runs.std(axis=0, ddof=1) / np.sqrt(runs.shape[0])
    ok = np.abs(mean - g0) <= 4.5 * se + 1e-10 * np.abs(g0).max()
    assert ok.mean() >= 0.9


def test_boutsidis_identity_within_truncation_bound():
    w, A = _spd_case(150)
    n = A.shape[0]
    m = 60
    est, alpha = es.boutsidis_logdet(A, np.eye(n), m, identity=True)
    lam = np.linalg.eigvalsh(A)
    rho = 1.0 - lam.min() / alpha
    bound = n * rho ** (m + 1) / ((m + 1) * (1.0 - rho))
    exact = np.linalg.slogdet(A)[1]
    assert est >= exact - 1e-9          # truncation only drops positive terms
    assert est - exact <= bound + 1e-9


def test_boutsidis_converges_on_well_conditioned_matrix():
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((80, 80)))
    A = Q @ np.diag(rng.uniform(1.0, 2.0, 80)) @ Q.T
    Z = es.rademacher(3, 80, 400)
    est, _ = es.boutsidis_logdet(A, Z, 80)
    assert est == pytest.approx(np.linalg.slogdet(A)[1], rel=2e-2)


def _sum_case(n=200, seed=5, noise=1e-2):
    return wl.random_small(n, 2, 3, 2, seed, combine=kn.COMBINE_SUM, per_row=10.0, noise_var=noise)


def test_lowrank_preconditioner_holds_the_bump_part():
    w = _sum_case()
    A = kn.kernel_matrix(w.desc, w.h, w.x)
    c, F = es.lowrank_terms(w.desc, w.h, w.x)
    R = A - F @ F.T                       # core part + noise
    assert np.allclose(np.diag(R), c, rtol=1e-14, atol=0)
    w.h[0] = 0.0                          # no core: A = noise I + F F^T = M exactly
    A0 = kn.kernel_matrix(w.desc, w.h, w.x)
    c0, F0 = es.lowrank_terms(w.desc, w.h, w.x)
    assert np.allclose(A0, c0 * np.eye(len(A0)) + F0 @ F0.T, rtol=0, atol=1e-15)


def test_lowrank_probe_covariance_is_M():
    w = _sum_case(n=60)
    c, F = es.lowrank_terms(w.desc, w.h, w.x)
    B = es.lowrank_probes(3, c, F, 40000)
    C = B @ B.T / B.shape[1]
    M = c * np.eye(60) + F @ F.T
    assert np.abs(C - M).max() < 5 * np.sqrt(np.diag(M).max() ** 2 / 40000) * 3


def test_preconditioned_estimator_exact_when_A_equals_M():
    # sigma2 = 0: A = M, so ln det A = ln det M and the SLQ part vanishes
    w = _sum_case()
    w.h[0] = 0.0
    val, g, logdet, _ = es.preconditioned_lml_grad(w.desc, w.h, w.x, w.y, 7, 4, 30)
    v0, g0 = gp.lml_grad(w.desc, w.h, w.x, w.y)
    exact = np.linalg.slogdet(kn.kernel_matrix(w.desc, w.h, w.x))[1]
    assert logdet == pytest.approx(exact, rel=1e-11)
    assert val == pytest.approx(v0, rel=1e-11)


def test_preconditioned_estimator_unbiased():
    w = _sum_case(n=150)
    A = kn.kernel_matrix(w.desc, w.h, w.x)
    exact = np.linalg.slogdet(A)[1]
    _, g0 = gp.lml_grad(w.desc, w.h, w.x, w.y)
    lds, ses, gs = [], [], []
    for s in range(8):
        _, g, ld, se = es.preconditioned_lml_grad(w.desc, w.h, w.x, w.y, 50 + s, 30, 60)
        lds.append(ld); ses.append(se); gs.append(g)
    se_mean = np.sqrt(np.sum(np.square(ses))) / len(ses)
    assert abs(np.mean(lds) - exact) < 4.5 * se_mean + 1e-9
    gs = np.array(gs)
    m = gs.mean(axis=0)
    sd = gs.std(axis=0, ddof=1) / np.sqrt(len(gs))
    ok = np.abs(m - g0) <= 4.5 * sd + 1e-9 * np.abs(g0).max()
    assert ok.mean() >= 0.9
