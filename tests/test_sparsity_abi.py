"""The library's host-only sparsity estimate and objectives (Section 2.2
eq:sparsity_estimate, Section 2.4) against the pinned oracle; no GPU."""
import os

import numpy as np
import pytest

from oracle import sparsity as sp
from paper_2205_09070_amd import _lib
from paper_2205_09070_amd import workloads as wl

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libsdgp.so not built")


@pytest.mark.parametrize("dim,n1,n2", [(1, 2, 3), (2, 2, 2), (3, 16, 4), (4, 5, 8)])
def test_sparsity_bound_matches_oracle(dim, n1, n2):
    w = wl.random_small(50, dim, n1, n2, 3)
    for vol in (1.0, 2.5):
        got = _lib.sparsity_bound(w.desc, w.h, vol)
        assert got == pytest.approx(sp.sparsity_bound(w.desc, w.h, vol), rel=1e-13)


def test_sparsity_bound_rejects_bad_input():
    w = wl.random_small(50, 2, 2, 2, 3)
    h = w.h.copy()
    h[2 + 2] = -1.0      # radius of bump (0, 0)
    with pytest.raises(_lib.SdgpError):
        _lib.sparsity_bound(w.desc, h)
    with pytest.raises(_lib.SdgpError):
        _lib.sparsity_bound(w.desc, w.h, 0.0)


def test_objectives_match_oracle():
    for lml, s, req in [(-120.5, 0.01, 0.02), (-3.0, 0.5, 0.1), (42.0, 0.0, 1.0)]:
        aug, feas = _lib.sparsity_objective(lml, s, req)
        assert aug == sp.augmented_objective(lml, s)
        assert feas == sp.constrained_feasible(s, req)
