"""Differential-evolution host logic (sdgp_de_trials / sdgp_de_select through
the C ABI; no GPU): bounds, determinism, the binomial crossover and mutation
rules of DE/rand/1/bin (Storn and Price 1997), selection semantics, and
convergence on a quadratic whose maximiser is known."""
import numpy as np
import pytest

import paper_2205_09070_amd as sd


def _pop(B, nh, seed=0):
    rng = np.random.default_rng(seed)
    lo = -1.0 - rng.random(nh)
    hi = 1.0 + rng.random(nh)
    H = lo + (hi - lo) * rng.random((B, nh))
    return H, lo, hi


def test_trials_stay_in_bounds_and_are_deterministic():
    H, lo, hi = _pop(12, 7)
    T1 = sd.de_trials(H, lo, hi, F=1.5, CR=0.9, seed=5, generation=3)
    T2 = sd.de_trials(H, lo, hi, F=1.5, CR=0.9, seed=5, generation=3)
    T3 = sd.de_trials(H, lo, hi, F=1.5, CR=0.9, seed=5, generation=4)
    assert np.array_equal(T1, T2)
    assert not np.array_equal(T1, T3)
    assert (T1 >= lo).all() and (T1 <= hi).all()


def test_fixed_components_never_move():
    H, lo, hi = _pop(8, 5)
    lo[2] = hi[2] = 0.25
    H[:, 2] = 0.25
    for g in range(1, 6):
        T = sd.de_trials(H, lo, hi, F=0.8, CR=1.0, seed=1, generation=g)
        assert (T[:, 2] == 0.25).all()


def test_zero_crossover_changes_one_component():
    H, lo, hi = _pop(10, 6)
    T = sd.de_trials(H, lo, hi, F=0.5, CR=0.0, seed=2, generation=1)
    changed = (T != H).sum(axis=1)
    assert (changed <= 1).all() and changed.sum() >= 8


def test_full_crossover_is_the_mutant_of_other_members():
    # with CR = 1 and a tiny F every trial is H[r1] + F (H[r2] - H[r3]) ~ H[r1], r1 != m
    H, lo, hi = _pop(9, 4)
    T = sd.de_trials(H, lo, hi, F=1e-9, CR=1.0, seed=3, generation=1)
    for m in range(9):
        d = np.abs(H - T[m]).max(axis=1)
        r1 = int(np.argmin(d))
        assert d[r1] < 1e-8 and r1 != m


def test_selection_rules():
    H = np.zeros((4, 2))
    T = np.ones((4, 2))
    fit = np.array([1.0, 1.0, np.nan, 2.0])
    ft = np.array([0.5, 1.0, -5.0, np.nan])
    H2, fit2, rep = sd.de_select(H, fit, T, ft)
    assert rep == 2
    assert (H2[0] == 0).all() and (H2[1] == 1).all() and (H2[2] == 1).all() and (H2[3] == 0).all()
    assert fit2[1] == 1.0 and fit2[2] == -5.0 and fit2[3] == 2.0


def test_de_finds_the_maximiser_of_a_quadratic():
    rng = np.random.default_rng(11)
    nh, B = 4, 20
    target = rng.uniform(-0.5, 0.5, nh)
    lo, hi = -np.ones(nh), np.ones(nh)
    H = lo + (hi - lo) * rng.random((B, nh))
    f = lambda P: -((P - target) ** 2).sum(axis=1)
    fit = f(H)
    for g in range(1, 401):
        T = sd.de_trials(H, lo, hi, F=0.7, CR=0.9, seed=7, generation=g)
        H, fit, _ = sd.de_select(H, fit, T, f(T))
    best = H[np.argmax(fit)]
    assert np.abs(best - target).max() < 1e-5


@pytest.mark.parametrize("bad", ["few", "outside", "F", "CR", "bounds"])
def test_invalid_arguments(bad):
    H, lo, hi = _pop(6, 3)
    F, CR = 0.7, 0.9
    if bad == "few":
        H = H[:3]
    elif bad == "outside":
        H[1, 1] = hi[1] + 1.0
    elif bad == "F":
        F = 0.0
    elif bad == "CR":
        CR = 1.5
    else:
        lo[0] = hi[0] + 1.0
    with pytest.raises(sd.SdgpError):
        sd.de_trials(H, lo, hi, F=F, CR=CR)
