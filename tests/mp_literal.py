"""Multi-precision evaluation of the paper's formulas as printed (test pins).

These evaluate the kernel of Section 2.2 literally -- eq:kstat with its
logarithm, eq:bump with the indicator read as "inside the ball",
eq:bump_kernel and its SUM variant -- in mpmath at 40 significant digits, by
pure-Python loops.  They pin the oracle's FP64 forms (series/atanh rewrites,
vectorised assembly, Cholesky) to the printed definitions.
"""
import mpmath as mp

mp.mp.dps = 40

C = mp.sqrt(2) / (3 * mp.sqrt(mp.pi))


def kstat(u):
    u = mp.mpf(u)
    if u >= 1:
        return mp.mpf(0)
    if u == 0:
        return C
    s = mp.sqrt(1 - u * u)
    return C * (3 * u * u * mp.log(u / (1 + s)) + (2 * u * u + 1) * s)


def wendland_integral(u, ell):
    """Wendland's construction: psi(u) = (l+1)(l+2) int_u^1 t (1-t)^l dt."""
    u = mp.mpf(u)
    if u >= 1:
        return mp.mpf(0)
    return (ell + 1) * (ell + 2) * mp.quad(lambda t: t * (1 - t) ** ell, [u, 1])


def core(u, core_id, dim):
    if core_id == 1:
        return kstat(u)
    ell = dim // 2 + 2
    u = mp.mpf(u)
    if u >= 1:
        return mp.mpf(0)
    return (1 - u) ** (ell + 1) * ((ell + 1) * u + 1)


def bump_f(x, c, r, a, beta):
    d2 = sum((mp.mpf(xk) - mp.mpf(ck)) ** 2 for xk, ck in zip(x, c))
    r = mp.mpf(r)
    if not d2 < r * r:
        return mp.mpf(0)
    q = d2 / (r * r)
    beta = mp.mpf(beta)
    return mp.mpf(a) * mp.exp(-beta / (1 - q) + beta)


def unpack(desc, h):
    n1, n2, d = desc.n1, desc.n2, desc.dim
    bumps = []
    for i in range(n1):
        row = []
        for j in range(n2):
            o = 2 + (i * n2 + j) * (3 + d)
            row.append((h[o], h[o + 1], h[o + 2], [h[o + 3 + k] for k in range(d)]))
        bumps.append(row)
    return mp.mpf(h[0]), mp.mpf(h[1]), bumps, mp.mpf(h[-1])


def F_row(desc, h, x):
    _, _, bumps, _ = unpack(desc, h)
    return [sum(bump_f(x, c, r, a, b) for (a, b, r, c) in bumps[i]) for i in range(desc.n1)]


def k_entry(desc, h, xa, xb):
    sigma2, rc, _, _ = unpack(desc, h)
    d = mp.sqrt(sum((mp.mpf(p) - mp.mpf(q)) ** 2 for p, q in zip(xa, xb)))
    psi = core(d / rc, desc.core, desc.dim)
    Fa = F_row(desc, h, xa)
    Fb = F_row(desc, h, xb)
    B = sum(fa * fb for fa, fb in zip(Fa, Fb))
    if desc.combine == 0:
        return sigma2 * psi * B
    return sigma2 * psi + B


def A_matrix(desc, h, X):
    n = len(X)
    _, _, _, nv = unpack(desc, h)
    A = mp.matrix(n, n)
    for a in range(n):
        for b in range(n):
            A[a, b] = k_entry(desc, h, X[a], X[b]) + (nv if a == b else 0)
    return A


def lml(desc, h, X, y):
    """-1/2 y^T A^{-1} y - 1/2 ln det A by mpmath LU."""
    A = A_matrix(desc, h, X)
    yv = mp.matrix([mp.mpf(v) for v in y])
    alpha = mp.lu_solve(A, yv)
    yKy = sum(yv[i] * alpha[i] for i in range(len(y)))
    return -yKy / 2 - mp.log(mp.det(A)) / 2
