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


# ---------------------------------------------------------------------------
# Low-rank preconditioned estimators (SUM combine).
#
# Under the SUM combine A = K_core + F F^T + noise_var I with F[a, i] =
# F_i(x_a) of rank <= n1, and the core part plus noise has the constant
# diagonal c = sigma2 psi(0) + noise_var.  M = c I + F F^T is therefore an
# SPD preconditioner that holds the whole bump part of A, and
#     ln det A = ln det M + tr ln(M^{-1/2} A M^{-1/2}),
#     ln det M = (N - n1) ln c + ln det(c I_{n1} + F^T F).
# Probes b_p = sqrt(c) w_p + F v_p with Rademacher w_p (N entries, counters
# p*2^32 + row + 1) and v_p (n1 entries, counters p*2^32 + 2^32 - 1 - i) have
# covariance M, so u_p = M^{-1/2} b_p has identity covariance:
#     tr ln(M^{-1/2} A M^{-1/2}) ~= (1/P) sum_p |u_p|^2 e_1^T ln(T_p) e_1
# with T_p the Lanczos tridiagonal of M^{-1/2} A M^{-1/2} from u_p / |u_p|,
# and E[M^{-1} b b^T] = I gives the trace term of the gradient
#     tr(A^{-1} dA) ~= (1/P) sum_p (A^{-1} b_p)^T dA (M^{-1} b_p).
# (The preconditioned-Lanczos estimator of Gardner et al., NeurIPS 2018.)
# ---------------------------------------------------------------------------

def lowrank_terms(desc, h, x):
    """(c, F) of the SUM-combine preconditioner M = c I + F F^T."""
    if desc.combine != kn.COMBINE_SUM:
        raise ValueError("the low-rank preconditioner needs the SUM combine")
    p = kn.unpack(desc, h)
    F, _ = kn.bump_F(desc, h, x)
    psi0 = float(kn.core_psi(np.array([0.0]), desc.core, desc.dim)[0])
    return p["sigma2"] * psi0 + p["noise_var"], F


def lowrank_probe_signs(seed: int, n1: int, probes: int):
    """V[n1, probes] Rademacher signs from counters p*2^32 + 2^32 - 1 - i."""
    V = np.empty((n1, probes))
    idx = np.arange(n1, dtype=np.uint64)
    for p in range(probes):
        k = (np.uint64(p) << np.uint64(32)) + (np.uint64(0xFFFFFFFF) - idx)
        bits = splitmix64_output(seed, k) >> np.uint64(63)
        V[:, p] = np.where(bits == 0, 1.0, -1.0)
    return V


def lowrank_probes(seed: int, c: float, F, probes: int):
    n, n1 = F.shape
    W = rademacher(seed, n, probes)
    V = lowrank_probe_signs(seed, n1, probes)
    return np.sqrt(c) * W + F @ V


def preconditioned_lml_grad(desc, h, x, y, seed: int, probes: int, m: int):
    """LML and gradient with the preconditioned SLQ / Hutchinson estimators
    (exact solves).  Returns (lml, grad, logdet, logdet_se)."""
    A = kn.kernel_matrix(desc, h, x, add_noise=True)
    c, F = lowrank_terms(desc, h, x)
    n, n1 = F.shape
    M = c * np.eye(n) + F @ F.T
    S = c * np.eye(n1) + F.T @ F
    logdetM = (n - n1) * np.log(c) + np.linalg.slogdet(S)[1]
    lam, U = np.linalg.eigh(M)
    Mmh = (U / np.sqrt(lam)) @ U.T
    Ah = Mmh @ A @ Mmh
    B = lowrank_probes(seed, c, F, probes)
    vals = np.empty(probes)
    for p in range(probes):
        u = Mmh @ B[:, p]
        al, be = lanczos(Ah, u, m)
        vals[p] = float(u @ u) * quad_log(al, be)
    est = float(vals.mean())
    se = float(vals.std(ddof=1) / np.sqrt(probes)) if probes > 1 else float("nan")
    logdet = logdetM + est
    cf = sla.cho_factor(A, lower=True)
    y = np.asarray(y, dtype=np.float64)
    alpha = sla.cho_solve(cf, y)
    val = -0.5 * float(y @ alpha) - 0.5 * logdet
    W = sla.cho_solve(cf, B)
    V = np.linalg.solve(M, B)
    grad = np.zeros(len(h))
    for idx, dA in gp.dA_dtheta(desc, h, x):
        tr = float(np.sum(W * (dA @ V))) / probes
        grad[idx] = 0.5 * float(alpha @ dA @ alpha) - 0.5 * tr
    return val, grad, logdet, se


# ---------------------------------------------------------------------------
# Block preconditioner (SUM combine).
#
# M = B + F F^T with B = blockdiag(B_t), where the row groups T_t (tiles)
# partition the points and B_t = S[T_t, T_t] is the principal submatrix of
# the solver's matrix S on the tile: S = K_core + noise_var I when the
# solver applies the factored operator A = S + F F^T, S = A (the whole
# covariance) otherwise.  Principal submatrices of an SPD matrix are SPD, so
# M is SPD, and every statement of the low-rank section above holds with
#     ln det M = sum_t ln det B_t + ln det(I_{n1} + F^T B^{-1} F)
# (determinant lemma) and probes b_p = L w_p + F v_p, L = blockdiag(L_t),
# B_t = L_t L_t^T (Cholesky with the tile's rows in the given order), w_p and
# v_p the Rademacher vectors of the low-rank probes: Cov(b_p) = L L^T +
# F F^T = M.  With singleton tiles B = c I and L = sqrt(c) I, which is the
# low-rank preconditioner with identical probes.
# ---------------------------------------------------------------------------

def block_terms(desc, h, x, tiles, factored: bool = True):
    """(blocks, F): blocks[t] = S[T_t, T_t] (tile rows in the given order)."""
    if desc.combine != kn.COMBINE_SUM:
        raise ValueError("the block preconditioner needs the SUM combine")
    p = kn.unpack(desc, h)
    x = np.asarray(x, dtype=np.float64)
    F, _ = kn.bump_F(desc, h, x)
    if factored:
        psi = kn.core_matrix(desc, h, x, x)[0]
        S = p["sigma2"] * psi + p["noise_var"] * np.eye(x.shape[0])
    else:
        S = kn.kernel_matrix(desc, h, x, add_noise=True)
    blocks = [S[np.ix_(t, t)] for t in tiles]
    return blocks, F


def block_probes(seed: int, chols, tiles, F, probes: int):
    """b_p = L w_p + F v_p for the tile Cholesky factors ``chols``."""
    n, n1 = F.shape
    W = rademacher(seed, n, probes)
    V = lowrank_probe_signs(seed, n1, probes)
    Bp = F @ V
    for t, L in zip(tiles, chols):
        Bp[t] += L @ W[t]
    return Bp


def block_preconditioned_lml_grad(desc, h, x, y, seed: int, probes: int, m: int, tiles,
                                  factored: bool = True):
    """LML and gradient with the block-preconditioned SLQ / Hutchinson
    estimators (exact solves); tiles: list of caller-row index arrays that
    partition the points.  Returns (lml, grad, logdet, logdet_se)."""
    A = kn.kernel_matrix(desc, h, x, add_noise=True)
    n = A.shape[0]
    tiles = [np.asarray(t, dtype=np.int64) for t in tiles]
    cover = np.sort(np.concatenate(tiles))
    if not np.array_equal(cover, np.arange(n)):
        raise ValueError("tiles must partition the rows")
    blocks, F = block_terms(desc, h, x, tiles, factored)
    chols = [np.linalg.cholesky(Bt) for Bt in blocks]
    Bm = np.zeros((n, n))
    for t, Bt in zip(tiles, blocks):
        Bm[np.ix_(t, t)] = Bt
    M = Bm + F @ F.T
    logdetB = sum(2.0 * float(np.sum(np.log(np.diag(L)))) for L in chols)
    n1 = F.shape[1]
    if n1 > 0:
        S = np.eye(n1) + F.T @ np.linalg.solve(Bm, F)
        logdetM = logdetB + np.linalg.slogdet(S)[1]
    else:
        logdetM = logdetB
    lam, U = np.linalg.eigh(M)
    Mmh = (U / np.sqrt(lam)) @ U.T
    Ah = Mmh @ A @ Mmh
    Bp = block_probes(seed, chols, tiles, F, probes)
    vals = np.empty(probes)
    for p in range(probes):
        u = Mmh @ Bp[:, p]
        al, be = lanczos(Ah, u, m)
        vals[p] = float(u @ u) * quad_log(al, be)
    est = float(vals.mean())
    se = float(vals.std(ddof=1) / np.sqrt(probes)) if probes > 1 else float("nan")
    logdet = logdetM + est
    cf = sla.cho_factor(A, lower=True)
    y = np.asarray(y, dtype=np.float64)
    alpha = sla.cho_solve(cf, y)
    val = -0.5 * float(y @ alpha) - 0.5 * logdet
    W = sla.cho_solve(cf, Bp)
    V = np.linalg.solve(M, Bp)
    grad = np.zeros(len(h))
    for idx, dA in gp.dA_dtheta(desc, h, x):
        tr = float(np.sum(W * (dA @ V))) / probes
        grad[idx] = 0.5 * float(alpha @ dA @ alpha) - 0.5 * tr
    return val, grad, logdet, se
