"""Pins of the sparsity estimate (eq:sparsity_estimate) and objectives."""
import json
import math
import os

import numpy as np
import pytest

from oracle import sparsity as sp
from paper_2205_09070_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_ball_volume_textbook_values():
    with open(os.path.join(GOLD, "textbook_constants.json")) as f:
        g = json.load(f)["unit_ball_volume"]
    for d in (1, 2, 3, 4):
        assert sp.ball_volume(d, 1.0) == pytest.approx(g["dim%d" % d], rel=1e-15)
    assert sp.ball_volume(3, 0.5) == pytest.approx(4.0 / 3.0 * math.pi / 8.0, rel=1e-15)


def test_bound_dominates_measured_bump_fraction():
    # disjoint-support bound (eq:sparsity_estimate) >= measured pair fraction
    rng = np.random.default_rng(0)
    desc = wl.KernelDesc(dim=2, n1=3, n2=2)
    x = rng.random((3000, 2))
    c = 0.2 + 0.6 * rng.random((3, 2, 2))
    r = rng.uniform(0.05, 0.12, (3, 2))
    h = wl.pack_hyper(desc, 1.0, 0.01, np.ones((3, 2)), np.ones((3, 2)), r, c, 1e-4)
    s_meas = sp.measured_bump_fraction(desc, h, x)
    s_bound = sp.sparsity_bound(desc, h)
    assert s_meas <= s_bound * 1.05
    assert s_meas > 0.2 * s_bound       # and it is not vacuous here


def test_bound_is_exact_for_one_disjoint_ball():
    rng = np.random.default_rng(1)
    desc = wl.KernelDesc(dim=2, n1=1, n2=1)
    x = rng.random((20000, 2))
    h = wl.pack_hyper(desc, 1.0, 0.01, [[1.0]], [[1.0]], [[0.2]], [[[0.5, 0.5]]], 1e-4)
    s_meas = sp.measured_bump_fraction(desc, h, x)
    s_bound = sp.sparsity_bound(desc, h)
    assert s_meas == pytest.approx(s_bound, rel=0.05)


def test_augmented_objective_range_and_constraint():
    lml = -123.0
    assert sp.augmented_objective(lml, 0.0) == 2 * lml
    assert sp.augmented_objective(lml, 1.0) == lml
    assert sp.constrained_feasible(0.01, 0.02) and not sp.constrained_feasible(0.03, 0.02)
