"""Sparsity estimate and sparsity-aware objectives (oracle).

* Ball volume (Section 2.2): Vol_s(dim, r) = pi^(dim/2) / Gamma(dim/2 + 1) r^dim.
* Upper bound of the stored fraction s of eq:sparsity_estimate for the bump
  part of the kernel, assuming disjoint supports:
      sup int_{S_k} = sum_i sum_j sum_k Vol_s(dim, r_ij) Vol_s(dim, r_ik),
  divided by the squared volume of the input domain (1 for the unit cube).
* Constrained objective (eq:constrained): ln L subject to s < requirement.
* Augmented objective (eq:augmented): ln L + (1 - s) ln L.
"""
from __future__ import annotations

import math

import numpy as np

from . import kernel as kn


def ball_volume(dim: int, r: float) -> float:
    return math.pi ** (dim / 2.0) / math.gamma(dim / 2.0 + 1.0) * r ** dim


def sparsity_bound(desc, h, domain_volume: float = 1.0) -> float:
    p = kn.unpack(desc, h)
    tot = 0.0
    for i in range(desc.n1):
        for j in range(desc.n2):
            for k in range(desc.n2):
                tot += ball_volume(desc.dim, p["r"][i, j]) * ball_volume(desc.dim, p["r"][i, k])
    return tot / (domain_volume * domain_volume)


def augmented_objective(lml: float, s: float) -> float:
    return lml + (1.0 - s) * lml


def constrained_feasible(s: float, requirement: float) -> bool:
    return s < requirement


def measured_bump_fraction(desc, h, x) -> float:
    """Fraction of ordered pairs (a, b) that share a bump support."""
    _, M = kn.bump_F(desc, h, x)
    Mi = M.astype(np.int64)
    return float(((Mi @ Mi.T) > 0).sum()) / float(x.shape[0]) ** 2
