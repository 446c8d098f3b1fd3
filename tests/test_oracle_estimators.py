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
