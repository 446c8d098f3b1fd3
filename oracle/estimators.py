"""Stochastic log-det and trace estimators (oracle).

* Probes: Rademacher vectors from the SplitMix64 generator (Steele, Lea and
  Flood, OOPSLA 2014), used counter-style: the k-th output of the stream
  seeded with ``seed`` is mix(seed + k * 0x9E3779B97F4A7C15) (mod 2^64) with
      mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
              z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31.
  Probe p, row r uses k = p * 2^32 + r + 1 and the sign of bit 63
  (+1 when clear).  Identity probes (e_p for p < N) give exact traces.
* Stochastic Lanczos quadrature (the spec log-det): for each probe z,
  Lanczos on A from z/|z| (full re-orthogonalisation here) builds T_m; with
  T_m = V diag(theta) V^T and tau = V[0, :],
      z^T ln(A) z ~= |z|^2 sum_k tau_k^2 ln theta_k,
  and ln det A = tr ln A ~= s * sum_p z_p^T ln(A) z_p with s = 1/P for random
  probes and s = 1 for the identity set.
* Hutchinson gradient: tr(A^{-1} dA) ~= s * sum_p (A^{-1} z_p)^T dA z_p.
* Randomised Taylor-series log-det of Boutsidis et al. (2017), the method the
  paper used (Section 2.5): with alpha >= lambda_max(A) and C = I - A/alpha,
      ln det A = N ln alpha - sum_{k>=1} tr(C^k) / k,
  truncated after m terms, each trace by the probes above.  alpha is the
  Gershgorin bound max_a sum_b |A_ab|.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import gp
from . import kernel as kn

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix64_output(seed: int, k):
    """k-th output (k >= 1) of the SplitMix64 stream started at ``seed``."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * GOLDEN
    return splitmix64_mix(state)


def rademacher(seed: int, n: int, probes: int):
    """Z[n, probes] with entries +-1 (float64)."""
    rows = np.arange(n, dtype=np.uint64)
    Z = np.empty((n, probes))
    for p in range(probes):
        k = (np.uint64(p) << np.uint64(32)) + rows + np.uint64(1)
        bits = splitmix64_output(seed, k) >> np.uint64(63)
        Z[:, p] = np.where(bits == 0, 1.0, -1.0)
    return Z


def lanczos(A, z, m, tol=1e-13):
    """Lanczos with full re-orthogonalisation from z/|z|.  Returns the
    diagonal and off-diagonal of T (stopping early on invariance)."""
    n = A.shape[0]
    Q = np.zeros((n, m + 1))
    q = z / np.linalg.norm(z)
    Q[:, 0] = q
    al = []
    be = []
    scale = np.abs(A).sum(axis=1).max()
    for k in range(m):
        w = A @ Q[:, k]
        a = float(Q[:, k] @ w)
        w = w - a * Q[:, k] - (be[-1] * Q[:, k - 1] if k > 0 else 0.0)
        w = w - Q[:, :k + 1] @ (Q[:, :k + 1].T @ w)
        w = w - Q[:, :k + 1] @ (Q[:, :k + 1].T @ w)
        al.append(a)
        b = float(np.linalg.norm(w))
        if k == m - 1 or b <= tol * scale:
            break
        be.append(b)
        Q[:, k + 1] = w / b
    return np.array(al), np.array(be)


def quad_log(al, be):
    """e1^T ln(T) e1 for the symmetric tridiagonal T(al, be)."""
    if al.size == 1:
        return float(np.log(al[0]))
    th, V = sla.eigh_tridiagonal(al, be)
    tau = V[0, :]
    return float(np.sum(tau * tau * np.log(th)))


def slq_logdet(A, Z, m, identity: bool = False):
    """Stochastic Lanczos quadrature estimate of ln det A from probe columns
    Z[:, p]; returns (estimate, standard error)."""
    P = Z.shape[1]
    vals = np.empty(P)
    for p in range(P):
        z = Z[:, p]
        al, be = lanczos(A, z, m)
        vals[p] = float(z @ z) * quad_log(al, be)
    if identity:
        return float(vals.sum()), 0.0
    est = float(vals.mean())
    se = float(vals.std(ddof=1) / np.sqrt(P)) if P > 1 else float("nan")
    return est, se


def stochastic_lml_grad(desc, h, x, y, Z, m, identity: bool = False):
    """LML and gradient with the log-det by SLQ and the trace by Hutchinson,
    all solves exact (Cholesky).  Returns (lml, grad, logdet, logdet_se)."""
    A = kn.kernel_matrix(desc, h, x, add_noise=True)
    cf = sla.cho_factor(A, lower=True)
    y = np.asarray(y, dtype=np.float64)
    alpha = sla.cho_solve(cf, y)
    logdet, se = slq_logdet(A, Z, m, identity=identity)
    val = -0.5 * float(y @ alpha) - 0.5 * logdet
    W = sla.cho_solve(cf, Z)
    s = 1.0 if identity else 1.0 / Z.shape[1]
    grad = np.zeros(len(h))
    for idx, dA in gp.dA_dtheta(desc, h, x):
        tr = s * float(np.sum(W * (dA @ Z)))
        grad[idx] = 0.5 * float(alpha @ dA @ alpha) - 0.5 * tr
    return val, grad, logdet, se


def boutsidis_logdet(A, Z, m, identity: bool = False):
    """Truncated randomised Taylor-series log-det (Boutsidis et al. 2017).
    Returns (estimate, alpha)."""
    n = A.shape[0]
    alpha = float(np.abs(A).sum(axis=1).max())
    P = Z.shape[1]
    s = 1.0 if identity else 1.0 / P
    V = Z.copy()
    acc = 0.0
    for k in range(1, m + 1):
        V = V - (A @ V) / alpha          # V = C^k Z
        acc += s * float(np.sum(Z * V)) / k
    return n * np.log(alpha) - acc, alpha
