"""Pins of the oracle's block-preconditioned estimator (SUM combine):
singleton tiles reduce it to the low-rank preconditioner with identical
probes; one tile holding every point makes M = A under the factored
operator (the SLQ part vanishes); the probes have covariance M; the
estimates are unbiased; and the test-side schedule is a partition into
spatially compact tiles."""
import numpy as np
import pytest

from oracle import estimators as es
from oracle import gp
from oracle import kernel as kn
from paper_2205_09070_amd import workloads as wl
from tests import sched_ref


def _case(n=180, seed=5, noise=1e-2, n1=3):
    return wl.random_small(n, 2, n1, 2, seed, combine=kn.COMBINE_SUM, per_row=10.0, noise_var=noise)


def test_singleton_tiles_equal_lowrank_estimator():
    w = _case()
    n = w.x.shape[0]
    tiles = [np.array([i]) for i in np.random.default_rng(1).permutation(n)]
    v1, g1, ld1, se1 = es.block_preconditioned_lml_grad(w.desc, w.h, w.x, w.y, 11, 6, 60, tiles)
    v0, g0, ld0, se0 = es.preconditioned_lml_grad(w.desc, w.h, w.x, w.y, 11, 6, 60)
    assert ld1 == pytest.approx(ld0, rel=1e-10)
    assert v1 == pytest.approx(v0, rel=1e-10)
    assert np.allclose(g1, g0, rtol=1e-8, atol=1e-10 * np.abs(g0).max())


def test_one_tile_makes_M_equal_A():
    w = _case(n=120)
    n = w.x.shape[0]
    tiles = [np.arange(n)[::-1]]
    val, g, logdet, _ = es.block_preconditioned_lml_grad(w.desc, w.h, w.x, w.y, 3, 4, 30, tiles)
    A = kn.kernel_matrix(w.desc, w.h, w.x)
    exact = np.linalg.slogdet(A)[1]
    v0, g0 = gp.lml_grad(w.desc, w.h, w.x, w.y)
    assert logdet == pytest.approx(exact, rel=1e-10)
    assert val == pytest.approx(v0, rel=1e-10)


def test_block_probe_covariance_is_M():
    w = _case(n=48)
    tiles = sched_ref.schedule_tiles(w.x, wl.unpack_hyper(w.desc, w.h)["r_core"])
    blocks, F = es.block_terms(w.desc, w.h, w.x, tiles)
    chols = [np.linalg.cholesky(B) for B in blocks]
    Bp = es.block_probes(9, chols, tiles, F, 40000)
    C = Bp @ Bp.T / Bp.shape[1]
    M = F @ F.T
    for t, B in zip(tiles, blocks):
        M[np.ix_(t, t)] += B
    scale = np.sqrt(np.outer(np.diag(M), np.diag(M)))
    assert (np.abs(C - M) <= 6 * scale / np.sqrt(40000) + 1e-12).all()


def test_block_estimator_unbiased():
    w = _case(n=150, noise=1e-3)
    tiles = sched_ref.schedule_tiles(w.x, wl.unpack_hyper(w.desc, w.h)["r_core"])
    exact = np.linalg.slogdet(kn.kernel_matrix(w.desc, w.h, w.x))[1]
    _, g0 = gp.lml_grad(w.desc, w.h, w.x, w.y)
    lds, ses, gs = [], [], []
    for s in range(8):
        _, g, ld, se = es.block_preconditioned_lml_grad(w.desc, w.h, w.x, w.y, 70 + s, 24, 60, tiles)
        lds.append(ld); ses.append(se); gs.append(g)
    se_mean = np.sqrt(np.sum(np.square(ses))) / len(ses)
    assert abs(np.mean(lds) - exact) < 4.5 * se_mean + 1e-9
    gs = np.array(gs)
    m = gs.mean(axis=0)
    sd = gs.std(axis=0, ddof=1) / np.sqrt(len(gs))
    ok = np.abs(m - g0) <= 4.5 * sd + 1e-9 * np.abs(g0).max()
    assert ok.mean() >= 0.9


def test_block_beats_lowrank_spread():
    # the block part also preconditions the core: the per-probe SLQ values
    # scatter less than with c I + F F^T on the same point set
    w = _case(n=200, noise=1e-3)
    tiles = sched_ref.schedule_tiles(w.x, wl.unpack_hyper(w.desc, w.h)["r_core"])
    _, _, _, se_b = es.block_preconditioned_lml_grad(w.desc, w.h, w.x, w.y, 5, 24, 80, tiles)
    _, _, _, se_l = es.preconditioned_lml_grad(w.desc, w.h, w.x, w.y, 5, 24, 80)
    assert se_b < se_l


@pytest.mark.parametrize("dim", [2, 3])
def test_schedule_tiles_partition_and_compact(dim):
    rng = np.random.default_rng(dim)
    x = rng.random((2000, dim))
    tiles = sched_ref.schedule_tiles(x, 0.05)
    assert all(len(t) == 16 for t in tiles[:-1]) and len(tiles[-1]) == 2000 - 16 * (len(tiles) - 1)
    assert np.array_equal(np.sort(np.concatenate(tiles)), np.arange(2000))
    # Morton tiles are compact: mean tile diameter well below that of random groups
    diam = np.mean([np.ptp(x[t], axis=0).max() for t in tiles[:-1]])
    rnd = np.mean([np.ptp(x[rng.choice(2000, 16, replace=False)], axis=0).max() for _ in range(100)])
    assert diam < 0.5 * rnd
