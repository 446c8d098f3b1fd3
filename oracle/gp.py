"""Dense FP64 log marginal likelihood, gradient and posterior (oracle).

* LML (eqn:log_likelihood) with zero prior mean and the additive constant
  dropped, on A = K + V with V = noise_var * I (the noise matrix of
  eq:likelihoodGP / eq:pred_distr):
      ln L = -1/2 y^T A^{-1} y - 1/2 ln det A.
  Solved by a Cholesky factorisation A = L L^T (LAPACK): alpha = A^{-1} y by
  two triangular solves and ln det A = 2 sum ln L_ii.
* Gradient with respect to every raw hyperparameter theta (the standard
  Gaussian-process identity, obtained by differentiating ln L):
      d ln L / d theta = 1/2 alpha^T (dA/dtheta) alpha
                         - 1/2 tr(A^{-1} dA/dtheta),
  with dA/dtheta built densely from the kernel's analytic derivatives.
* Posterior (eq:pred_distr) with m0 = 0:
      mean = kappa^T A^{-1} y,  var = k(x0, x0) - kappa^T A^{-1} kappa.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import kernel as kn


def _chol(A):
    return sla.cho_factor(A, lower=True, check_finite=True)


def lml(desc, h, x, y):
    """Returns (lml, alpha, logdet, yKy)."""
    A = kn.kernel_matrix(desc, h, x, add_noise=True)
    cf = _chol(A)
    y = np.asarray(y, dtype=np.float64)
    alpha = sla.cho_solve(cf, y)
    logdet = 2.0 * np.sum(np.log(np.diag(cf[0])))
    yKy = float(y @ alpha)
    return -0.5 * yKy - 0.5 * logdet, alpha, logdet, yKy


def dA_dtheta(desc, h, x):
    """Dense derivative matrices dA/dtheta for every entry of h, in the
    hyperparameter layout order.  A generator of (index, matrix)."""
    p = kn.unpack(desc, h)
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    psi, u, inside, _ = kn.core_matrix(desc, h, x, x)
    F, _ = kn.bump_F(desc, h, x)
    B = F @ F.T
    dpsi = np.where(inside, kn.core_dpsi(np.where(inside, u, 1.0), desc.core, desc.dim), 0.0)
    dpsi_drc = -(u / p["r_core"]) * dpsi
    prod = desc.combine == kn.COMBINE_PRODUCT
    # sigma2
    yield 0, (psi * B if prod else psi)
    # core radius
    yield 1, (p["sigma2"] * dpsi_drc * B if prod else p["sigma2"] * dpsi_drc)
    # bump parameters
    cfac = p["sigma2"] * psi if prod else None
    dF = kn.bump_dF(desc, h, x)      # [N, n1, n2, 3+d]
    for i in range(desc.n1):
        Fi = F[:, i]
        for j in range(desc.n2):
            base = 2 + (i * desc.n2 + j) * (3 + desc.dim)
            for t in range(3 + desc.dim):
                g = dF[:, i, j, t]
                M = np.outer(g, Fi) + np.outer(Fi, g)
                yield base + t, (cfac * M if prod else M)
    # noise variance
    yield 2 + desc.n1 * desc.n2 * (3 + desc.dim), np.eye(n)


def lml_grad(desc, h, x, y):
    """Returns (lml, grad[n_h]) by the dense analytic formula."""
    A = kn.kernel_matrix(desc, h, x, add_noise=True)
    cf = _chol(A)
    y = np.asarray(y, dtype=np.float64)
    alpha = sla.cho_solve(cf, y)
    logdet = 2.0 * np.sum(np.log(np.diag(cf[0])))
    val = -0.5 * float(y @ alpha) - 0.5 * logdet
    Ainv = sla.cho_solve(cf, np.eye(A.shape[0]))
    grad = np.zeros(len(h))
    for idx, dA in dA_dtheta(desc, h, x):
        grad[idx] = 0.5 * float(alpha @ dA @ alpha) - 0.5 * float(np.sum(Ainv * dA))
    return val, grad


def posterior_mean_var(desc, h, x, y, x0):
    """Posterior mean and variance at test points x0 (eq:pred_distr, m0=0)."""
    A = kn.kernel_matrix(desc, h, x, add_noise=True)
    cf = _chol(A)
    kap = kn.kernel_cross(desc, h, x, x0)            # [N, n0]
    alpha = sla.cho_solve(cf, np.asarray(y, dtype=np.float64))
    mean = kap.T @ alpha
    V = sla.cho_solve(cf, kap)
    kxx = np.diag(kn.kernel_cross(desc, h, x0, x0))
    var = kxx - np.sum(kap * V, axis=0)
    return mean, var
