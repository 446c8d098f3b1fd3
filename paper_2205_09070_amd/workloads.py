"""Seeded synthetic workloads for the sparsity-discovering GP hot path.

This module only draws inputs: point sets, observations and hyperparameter
vectors with the shapes and distributions of the paper's workloads (the
climate example of Section 3 uses space x time points; the synthetic sets
here stand in for that dataset, which is not available).  It contains none of
the method's arithmetic (no kernel, no covariance, no likelihood), so both the
GPU path and the CPU reference may consume it.

Hyperparameter layout (shared by every consumer):

    h = [sigma2, r_core,
         {a_ij, beta_ij, r_ij, c_ij[0..dim-1]}  for i < n1, j < n2 (j fastest),
         noise_var]

so ``len(h) = 2 + n1*n2*(3+dim) + 1``.  The bump amplitude ``a_ij`` is the
peak height of the bump function of Section 2.2 (the form with ``+beta``).

Draw order for every workload: X, then bump centres, radii, amplitudes and
shape parameters, then the observation field, then the observation noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CORE_WENDLAND_C2 = 0
CORE_KSTAT = 1
COMBINE_PRODUCT = 0
COMBINE_SUM = 1


@dataclass
class KernelDesc:
    dim: int
    n1: int
    n2: int
    core: int = CORE_WENDLAND_C2
    combine: int = COMBINE_SUM

    @property
    def n_hyper(self) -> int:
        return 2 + self.n1 * self.n2 * (3 + self.dim) + 1


@dataclass
class Workload:
    name: str
    desc: KernelDesc
    x: np.ndarray          # [N, dim] float64, caller order
    y: np.ndarray          # [N] float64
    h: np.ndarray          # [n_hyper] float64
    meta: dict = field(default_factory=dict)


def hyper_index(desc: KernelDesc, i: int, j: int) -> int:
    """Offset of bump (i, j)'s parameter block inside h."""
    return 2 + (i * desc.n2 + j) * (3 + desc.dim)


def pack_hyper(desc: KernelDesc, sigma2: float, r_core: float, a, beta, r, c,
               noise_var: float) -> np.ndarray:
    """Pack arrays a, beta, r: [n1, n2] and c: [n1, n2, dim] into h."""
    h = np.zeros(desc.n_hyper, dtype=np.float64)
    h[0] = sigma2
    h[1] = r_core
    for i in range(desc.n1):
        for j in range(desc.n2):
            o = hyper_index(desc, i, j)
            h[o + 0] = a[i][j]
            h[o + 1] = beta[i][j]
            h[o + 2] = r[i][j]
            h[o + 3:o + 3 + desc.dim] = c[i][j]
    h[-1] = noise_var
    return h


def unpack_hyper(desc: KernelDesc, h: np.ndarray) -> dict:
    h = np.asarray(h, dtype=np.float64)
    n1, n2, d = desc.n1, desc.n2, desc.dim
    blk = h[2:2 + n1 * n2 * (3 + d)].reshape(n1, n2, 3 + d)
    return dict(sigma2=float(h[0]), r_core=float(h[1]), a=blk[:, :, 0].copy(),
                beta=blk[:, :, 1].copy(), r=blk[:, :, 2].copy(),
                c=blk[:, :, 3:].copy(), noise_var=float(h[-1]))


def radius_for_neighbours(n_points: int, dim: int, per_row: float) -> float:
    """Radius whose ball holds ``per_row`` points of a unit-density sample.

    Input recipe only: the ball volume is the textbook unit-ball formula.
    """
    unit = math.pi ** (dim / 2.0) / math.gamma(dim / 2.0 + 1.0)
    return (per_row / (n_points * unit)) ** (1.0 / dim)


def _bumps(rng, n1, n2, dim, r_lo, r_hi, a_lo, a_hi, beta=1.0):
    c = rng.random((n1, n2, dim))
    r = rng.uniform(r_lo, r_hi, size=(n1, n2))
    a = rng.uniform(a_lo, a_hi, size=(n1, n2))
    b = np.full((n1, n2), beta)
    return a, b, r, c


def _gauss_field(rng, x, n_bumps=5, width=0.1):
    amp = rng.standard_normal(n_bumps)
    mu = rng.random((n_bumps, x.shape[1]))
    out = np.zeros(x.shape[0])
    for k in range(n_bumps):
        d2 = np.sum((x - mu[k]) ** 2, axis=1)
        out += amp[k] * np.exp(-d2 / (2.0 * width * width))
    return out


def small_2d(n: int = 2000, seed: int = 0, core: int = CORE_WENDLAND_C2,
             combine: int = COMBINE_SUM) -> Workload:
    """2-D parity workload: N points uniform in [0,1)^2, core radius 0.05,
    2 bump functions x 2 centres, y = sin(6 x1) cos(4 x2) + N(0, 0.01^2),
    noise variance 1e-4."""
    rng = np.random.default_rng(seed)
    desc = KernelDesc(dim=2, n1=2, n2=2, core=core, combine=combine)
    x = rng.random((n, 2))
    c = rng.random((2, 2, 2))
    r = rng.uniform(0.05, 0.1, size=(2, 2))
    a = rng.uniform(0.5, 1.0, size=(2, 2))
    b = np.ones((2, 2))
    y = np.sin(6 * x[:, 0]) * np.cos(4 * x[:, 1])
    y = y + 0.01 * rng.standard_normal(n)
    h = pack_hyper(desc, 1.0, 0.05, a, b, r, c, 1e-4)
    return Workload("uniform2d_n%d" % n, desc, x, y, h,
                    dict(seed=seed, per_row_target=None))


def uniform_3d(n: int, per_row: float, n1: int, n2: int, seed: int = 0,
               r_lo: float = 0.03, r_hi: float = 0.06,
               combine: int = COMBINE_SUM) -> Workload:
    """3-D workload: N points uniform in [0,1)^3, Wendland core radius tuned
    for ``per_row`` core neighbours, n1 x n2 bumps with radii U(r_lo, r_hi),
    peak heights U(0.5, 1), beta = 1; y = sum of 5 random Gaussian bumps
    (width 0.1, N(0,1) amplitudes) + N(0, 0.01^2); noise variance 1e-4."""
    rng = np.random.default_rng(seed)
    desc = KernelDesc(dim=3, n1=n1, n2=n2, core=CORE_WENDLAND_C2, combine=combine)
    x = rng.random((n, 3))
    c = rng.random((n1, n2, 3))
    r = rng.uniform(r_lo, r_hi, size=(n1, n2))
    a = rng.uniform(0.5, 1.0, size=(n1, n2))
    b = np.ones((n1, n2))
    y = _gauss_field(rng, x) + 0.01 * rng.standard_normal(n)
    rc = radius_for_neighbours(n, 3, per_row)
    h = pack_hyper(desc, 1.0, rc, a, b, r, c, 1e-4)
    return Workload("uniform3d_n%d" % n, desc, x, y, h,
                    dict(seed=seed, per_row_target=per_row))


def uniform3d_100k(seed: int = 0, combine: int = COMBINE_SUM) -> Workload:
    """N=100,000 in [0,1)^3, ~100 core neighbours per row, 8x4 bumps."""
    return uniform_3d(100_000, 100.0, 8, 4, seed=seed, combine=combine)


def uniform3d_1m(seed: int = 0, combine: int = COMBINE_SUM) -> Workload:
    """N=1,000,000 in [0,1)^3, ~60 core neighbours per row, 16x4 bumps."""
    return uniform_3d(1_000_000, 60.0, 16, 4, seed=seed, combine=combine)


def population_3d(n: int = 200_000, members: int = 64, seed: int = 0,
                  combine: int = COMBINE_SUM):
    """Shared 3-D point set and a population of hyperparameter vectors.

    Each member draws rho ~ U(0.005, 0.02) and uses the core radius
    (0.75 rho^2)^(1/3) (the 3-D ball holding as many points as the 2-D disc
    of radius rho), and its own bump peak heights ~ U(0, 1); the bump
    centres, radii and shapes (8 x 4, radii U(0.03, 0.06), beta = 1) are
    shared.  Returns (Workload of member 0, H [members, n_hyper])."""
    rng = np.random.default_rng(seed)
    n1, n2 = 8, 4
    desc = KernelDesc(dim=3, n1=n1, n2=n2, core=CORE_WENDLAND_C2, combine=combine)
    x = rng.random((n, 3))
    c = rng.random((n1, n2, 3))
    r = rng.uniform(0.03, 0.06, size=(n1, n2))
    b = np.ones((n1, n2))
    rho = rng.uniform(0.005, 0.02, size=members)
    amps = rng.uniform(0.0, 1.0, size=(members, n1, n2))
    y = _gauss_field(rng, x) + 0.01 * rng.standard_normal(n)
    H = np.stack([pack_hyper(desc, 1.0, (0.75 * rho[m] ** 2) ** (1.0 / 3.0),
                             amps[m], b, r, c, 1e-4) for m in range(members)])
    wl = Workload("population3d_n%d_b%d" % (n, members), desc, x, y, H[0].copy(),
                  dict(seed=seed))
    return wl, H


def spacetime_4d(n: int = 5_000_000, seed: int = 0, per_row: float = 50.0,
                 n1: int = 32, n2: int = 8, combine: int = COMBINE_SUM) -> Workload:
    """Space-time set: x1..x3 ~ U[0,1), x4 = t/364 with t ~ U{0..364};
    Wendland core (4-D) radius for ``per_row`` neighbours; n1 x n2 bumps with
    radii U(0.03, 0.06); y = 256 random Fourier features (frequencies
    N(0, 10^2 I), phases U(0, 2 pi), weights N(0, 2/256)) + N(0, 0.05^2)."""
    rng = np.random.default_rng(seed)
    desc = KernelDesc(dim=4, n1=n1, n2=n2, core=CORE_WENDLAND_C2, combine=combine)
    x = np.empty((n, 4))
    x[:, :3] = rng.random((n, 3))
    x[:, 3] = rng.integers(0, 365, size=n) / 364.0
    c = rng.random((n1, n2, 4))
    r = rng.uniform(0.03, 0.06, size=(n1, n2))
    a = rng.uniform(0.5, 1.0, size=(n1, n2))
    b = np.ones((n1, n2))
    om = 10.0 * rng.standard_normal((256, 4))
    ph = rng.uniform(0, 2 * np.pi, size=256)
    w = rng.standard_normal(256) * math.sqrt(2.0 / 256.0)
    y = np.zeros(n)
    for s in range(0, n, 1 << 18):
        y[s:s + (1 << 18)] = np.cos(x[s:s + (1 << 18)] @ om.T + ph) @ w
    y += 0.05 * rng.standard_normal(n)
    rc = radius_for_neighbours(n, 4, per_row)
    h = pack_hyper(desc, 1.0, rc, a, b, r, c, 1e-4)
    return Workload("spacetime4d_n%d" % n, desc, x, y, h, dict(seed=seed))


def random_small(n: int, dim: int, n1: int, n2: int, seed: int,
                 core: int = CORE_WENDLAND_C2, combine: int = COMBINE_SUM,
                 per_row: float = 12.0, r_lo: float = None, r_hi: float = None,
                 noise_var: float = 1e-4) -> Workload:
    """Small random case for parity tests: N points in [0,1)^dim, core radius
    for ``per_row`` neighbours, bumps with radii U(r_lo, r_hi) (default: 1.5x
    to 3x the core radius), peak heights U(0.5, 1), beta U(0.5, 2)."""
    rng = np.random.default_rng(seed)
    desc = KernelDesc(dim=dim, n1=n1, n2=n2, core=core, combine=combine)
    x = rng.random((n, dim))
    rc = radius_for_neighbours(n, dim, per_row)
    lo = 1.5 * rc if r_lo is None else r_lo
    hi = 3.0 * rc if r_hi is None else r_hi
    c = rng.random((n1, n2, dim))
    r = rng.uniform(lo, hi, size=(n1, n2))
    a = rng.uniform(0.5, 1.0, size=(n1, n2))
    b = rng.uniform(0.5, 2.0, size=(n1, n2))
    y = np.sin(5 * x[:, 0]) + 0.3 * np.cos(3 * x[:, -1]) + 0.01 * rng.standard_normal(n)
    y = y - y.mean()
    h = pack_hyper(desc, 1.0, rc, a, b, r, c, noise_var)
    return Workload("random%dd_n%d_s%d" % (dim, n, seed), desc, x, y, h, dict(seed=seed))
