"""Dense FP64 evaluation of the sparsity-discovering kernel (oracle).

Definitions (Section 2.2):

* compact stationary core of eq:kstat, for u = d / r < 1 with
  S = sqrt(1 - u^2):
      psi(u) = c * (3 u^2 ln(u / (1 + S)) + (2 u^2 + 1) S),
      c = sqrt(2) / (3 sqrt(pi)),
  and 0 for u >= 1.  The paper allows any core ("leading to no restrictions
  on the core kernel"); the Wendland C2 function
      psi(u) = (1 - u)^(l+1) ((l+1) u + 1),  l = floor(dim/2) + 2
  is the second core, positive definite in every dimension it is used in.
* bump functions of eq:bump, with the indicator read as "inside the ball"
  (the printed indicator is 1 outside the ball, which would make the bump
  non-compact):  f_ij(x) = a_ij exp(beta_ij - beta_ij / (1 - q)),
  q = |x - c_ij|^2 / r_ij^2, for q < 1 and 0 otherwise;  F_i = sum_j f_ij.
* kernel of eq:bump_kernel:  K_ab = sigma2 psi(u_ab) * B_ab  (PRODUCT), with
  B_ab = sum_i F_i(x_a) F_i(x_b); the SUM combine K_ab = sigma2 psi(u_ab) + B_ab
  is the "core plus bump products" reading.  Noise adds noise_var on the
  diagonal (diagonal V of eq:likelihoodGP).

The stored-entry predicate (which pairs a sparse K keeps) is decided on the
supports, not on values: pair (a, b) is kept iff a == b, or
  core_ab = d_ab^2 < r^2   and/or   bump_ab = exists i with x_a and x_b both
  strictly inside some ball of bump function i,
with AND for PRODUCT and OR for SUM.

Numerics: near u -> 1 the printed form of eq:kstat cancels catastrophically.
With the identity ln(u/(1+S)) = -atanh(S) and atanh's Taylor series,
  psi(u)/c = sum_{n>=2} 6 S^(2n+1) / (4 n^2 - 1),
which is used for S <= 0.85; the printed form is used above that (its
condition number there is below ~9).  psi(0) = c is the limit of the
printed form.  psi'(u) = 6 c u (S - atanh S), with the series
S - atanh S = -sum_{k>=1} S^(2k+1) / (2k+1) for S <= 0.85.
"""
from __future__ import annotations

import math

import numpy as np

C_KSTAT = math.sqrt(2.0) / (3.0 * math.sqrt(math.pi))
CORE_WENDLAND_C2 = 0
CORE_KSTAT = 1
COMBINE_PRODUCT = 0
COMBINE_SUM = 1
SERIES_S_MAX = 0.85
SERIES_TERMS = 150
BOUNDARY_BAND = 1e-12


def wendland_ell(dim: int) -> int:
    """Wendland smoothness-1 exponent l = floor(dim/2) + 2."""
    return dim // 2 + 2


def _s_of_u(u):
    # S = sqrt(1 - u^2) formed as sqrt((1-u)(1+u)) to keep relative accuracy
    return np.sqrt(np.maximum((1.0 - u) * (1.0 + u), 0.0))


def _kstat_psi(u):
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    inside = u < 1.0
    s = _s_of_u(np.where(inside, u, 0.0))
    ser = inside & (s <= SERIES_S_MAX)
    clo = inside & ~ser
    if np.any(ser):
        ss = s[ser]
        s2 = ss * ss
        acc = np.zeros_like(ss)
        for n in range(SERIES_TERMS + 1, 1, -1):
            acc = acc * s2 + 6.0 / (4.0 * n * n - 1.0)
        out[ser] = C_KSTAT * acc * ss ** 5
    if np.any(clo):
        uu = u[clo]
        ss = s[clo]
        u2 = uu * uu
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.log(uu / (1.0 + ss))
            val = C_KSTAT * (3.0 * u2 * lg + (2.0 * u2 + 1.0) * ss)
        val = np.where(uu == 0.0, C_KSTAT, val)
        out[clo] = val
    return out


def _kstat_dpsi(u):
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    inside = u < 1.0
    s = _s_of_u(np.where(inside, u, 0.0))
    ser = inside & (s <= SERIES_S_MAX)
    clo = inside & ~ser
    if np.any(ser):
        ss = s[ser]
        s2 = ss * ss
        acc = np.zeros_like(ss)
        for k in range(SERIES_TERMS, 0, -1):
            acc = acc * s2 + 1.0 / (2.0 * k + 1.0)
        out[ser] = 6.0 * C_KSTAT * u[ser] * (-(acc * ss ** 3))
    if np.any(clo):
        uu = u[clo]
        ss = s[clo]
        with np.errstate(divide="ignore", invalid="ignore"):
            at = np.log((1.0 + ss) / uu)
            val = 6.0 * C_KSTAT * uu * (ss - at)
        out[clo] = np.where(uu == 0.0, 0.0, val)
    return out


def _wendland_psi(u, dim):
    u = np.asarray(u, dtype=np.float64)
    ell = wendland_ell(dim)
    v = np.where(u < 1.0, 1.0 - u, 0.0)
    return v ** (ell + 1) * ((ell + 1) * u + 1.0) * (u < 1.0)


def _wendland_dpsi(u, dim):
    u = np.asarray(u, dtype=np.float64)
    ell = wendland_ell(dim)
    v = np.where(u < 1.0, 1.0 - u, 0.0)
    return -(ell + 1) * (ell + 2) * u * v ** ell * (u < 1.0)


def core_psi(u, core: int, dim: int):
    """Core profile psi(u), u = distance / core radius; 0 for u >= 1."""
    if core == CORE_KSTAT:
        return _kstat_psi(u)
    if core == CORE_WENDLAND_C2:
        return _wendland_psi(u, dim)
    raise ValueError("unknown core %r" % core)


def core_dpsi(u, core: int, dim: int):
    """d psi / d u; 0 for u >= 1."""
    if core == CORE_KSTAT:
        return _kstat_dpsi(u)
    if core == CORE_WENDLAND_C2:
        return _wendland_dpsi(u, dim)
    raise ValueError("unknown core %r" % core)


def unpack(desc, h):
    n1, n2, d = desc.n1, desc.n2, desc.dim
    h = np.asarray(h, dtype=np.float64)
    if h.shape[0] != 2 + n1 * n2 * (3 + d) + 1:
        raise ValueError("hyperparameter vector has the wrong length")
    blk = h[2:2 + n1 * n2 * (3 + d)].reshape(n1, n2, 3 + d)
    return dict(sigma2=h[0], r_core=h[1], a=blk[:, :, 0], beta=blk[:, :, 1],
                r=blk[:, :, 2], c=blk[:, :, 3:], noise_var=h[-1])


def pair_d2(xa, xb):
    """Squared distances sum_k (xa_k - xb_k)^2, coordinate order k = 0..d-1."""
    xa = np.asarray(xa, dtype=np.float64)
    xb = np.asarray(xb, dtype=np.float64)
    d2 = np.zeros((xa.shape[0], xb.shape[0]))
    for k in range(xa.shape[1]):
        diff = xa[:, k][:, None] - xb[:, k][None, :]
        d2 = d2 + diff * diff
    return d2


def bump_terms(desc, h, x):
    """Per point and bump centre: squared distance ratio q, membership and
    value f_ij(x).  Shapes [N, n1, n2]."""
    p = unpack(desc, h)
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    dist2 = np.zeros((n, desc.n1, desc.n2))
    for k in range(desc.dim):
        diff = x[:, k][:, None, None] - p["c"][None, :, :, k]
        dist2 = dist2 + diff * diff
    r2 = p["r"] * p["r"]
    inside = dist2 < r2[None]
    q = dist2 / r2[None]
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        e = np.exp(p["beta"][None] - p["beta"][None] / (1.0 - q))
    e = np.where(inside, e, 0.0)
    f = p["a"][None] * e
    return dict(dist2=dist2, q=q, inside=inside, expo=e, f=f)


def bump_F(desc, h, x):
    """F[a, i] = sum_j f_ij(x_a) and membership M[a, i] (x_a inside any ball
    of bump function i)."""
    t = bump_terms(desc, h, x)
    return t["f"].sum(axis=2), t["inside"].any(axis=2)


def bump_dF(desc, h, x):
    """Derivatives of f_ij(x_a) with respect to (a, beta, r, c_0..c_{d-1}) of
    centre (i, j).  Shape [N, n1, n2, 3 + dim]; zero outside the ball.

      df/da = f / a (formed as the exponential factor), df/dbeta = -f q/(1-q),
      df/dr = f beta/(1-q)^2 * 2 q / r, df/dc_k = f beta/(1-q)^2 * 2 (x_k-c_k)/r^2
    """
    p = unpack(desc, h)
    x = np.asarray(x, dtype=np.float64)
    t = bump_terms(desc, h, x)
    inside = t["inside"]
    q = np.where(inside, t["q"], 0.0)
    f = t["f"]
    beta = p["beta"][None]
    r = p["r"][None]
    omq = 1.0 - q
    out = np.zeros(f.shape + (3 + desc.dim,))
    out[..., 0] = t["expo"]
    out[..., 1] = -f * q / omq
    g = f * beta / (omq * omq)
    out[..., 2] = g * 2.0 * q / r
    for k in range(desc.dim):
        out[..., 3 + k] = g * 2.0 * (x[:, k][:, None, None] - p["c"][None, :, :, k]) / (r * r)
    out = np.where(inside[..., None], out, 0.0)
    return out


def core_matrix(desc, h, xa, xb):
    """psi(u_ab) for all pairs (zero outside the core support) and u_ab."""
    p = unpack(desc, h)
    d2 = pair_d2(xa, xb)
    rc = p["r_core"]
    inside = d2 < rc * rc
    u = np.sqrt(d2) / rc
    psi = np.where(inside, core_psi(np.where(inside, u, 1.0), desc.core, desc.dim), 0.0)
    return psi, u, inside, d2


def pattern(desc, h, x):
    """Dense boolean matrix of stored entries (support predicate)."""
    x = np.asarray(x, dtype=np.float64)
    p = unpack(desc, h)
    d2 = pair_d2(x, x)
    core = d2 < p["r_core"] ** 2
    _, M = bump_F(desc, h, x)
    bump = (M.astype(np.int64) @ M.T.astype(np.int64)) > 0
    if desc.combine == COMBINE_PRODUCT:
        pat = core & bump
    elif desc.combine == COMBINE_SUM:
        pat = core | bump
    else:
        raise ValueError("unknown combine")
    np.fill_diagonal(pat, True)
    return pat


def kernel_cross(desc, h, xa, xb):
    """k(x_a, x_b) for two point sets (no noise)."""
    p = unpack(desc, h)
    psi, _, _, _ = core_matrix(desc, h, xa, xb)
    Fa, _ = bump_F(desc, h, xa)
    Fb, _ = bump_F(desc, h, xb)
    B = Fa @ Fb.T
    if desc.combine == COMBINE_PRODUCT:
        return p["sigma2"] * psi * B
    if desc.combine == COMBINE_SUM:
        return p["sigma2"] * psi + B
    raise ValueError("unknown combine")


def kernel_matrix(desc, h, x, add_noise: bool = True):
    """Dense K (+ noise_var I when add_noise) on one point set."""
    K = kernel_cross(desc, h, x, x)
    if add_noise:
        K = K + unpack(desc, h)["noise_var"] * np.eye(K.shape[0])
    return K


def boundary_pairs(desc, h, x, band: float = BOUNDARY_BAND):
    """Pairs whose membership in the stored pattern is decided within a
    relative band of a support boundary (|d^2/r^2 - 1| < band for the core,
    |q - 1| < band for a bump centre of either point).  These are excluded
    from bit-exact pattern comparisons."""
    p = unpack(desc, h)
    d2 = pair_d2(x, x)
    core_b = np.abs(d2 / p["r_core"] ** 2 - 1.0) < band
    t = bump_terms(desc, h, x)
    frag = (np.abs(t["q"] - 1.0) < band).any(axis=2)      # [N, n1]
    fi = frag.astype(np.int64)
    anyb = (fi @ np.ones((desc.n1, x.shape[0]), dtype=np.int64)) > 0
    bump_b = anyb | anyb.T
    out = core_b | bump_b
    np.fill_diagonal(out, False)
    return out


def to_csr(K, pat):
    """Canonical CSR (ascending columns, diagonal always present) of the
    stored entries of a dense matrix."""
    n = K.shape[0]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols = []
    vals = []
    for a in range(n):
        cidx = np.nonzero(pat[a])[0]
        cols.append(cidx.astype(np.int32))
        vals.append(K[a, cidx])
        row_ptr[a + 1] = row_ptr[a] + cidx.size
    return row_ptr, np.concatenate(cols), np.concatenate(vals)
