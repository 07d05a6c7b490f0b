"""Multi-indices and Taylor coefficients of 1/|r + h| (test infrastructure only).

The paper expands G(x, y) = 1/(4 pi |x - y|) in a Cartesian Taylor series about the two cell
centres, truncated to |alpha| + |beta| <= q (Sec. 3, Translation operators), and defers the
derivatives to another paper. This oracle computes the Taylor coefficients

  a_gamma(r) = (d^gamma (1/|.|))(r) / gamma!  = coefficient of h^gamma in 1/|r + h|

from the binomial series, which needs no recurrence:

  1/|r + h| = |r|^-1 (1 + t)^(-1/2),  t = (2 r.h + h.h) / |r|^2,
  (1 + t)^(-1/2) = sum_n binom(-1/2, n) t^n,

truncated at total degree Q in h (t^n has degree >= n, so n <= Q suffices). Polynomials in
h are dicts exponent -> coefficient array over a batch of offsets r.
"""

from math import comb, factorial

import numpy as np


def multi_indices(q):
    """All (i, j, k) with i + j + k <= q in graded order: degree d = 0..q, then i descending, j descending."""
    out = []
    for d in range(q + 1):
        for i in range(d, -1, -1):
            for j in range(d - i, -1, -1):
                out.append((i, j, d - i - j))
    return out


def n_coeffs(q):
    return (q + 1) * (q + 2) * (q + 3) // 6


def mi_factorial(a):
    return factorial(a[0]) * factorial(a[1]) * factorial(a[2])


def mi_binom(b, a):
    """C(b, a) = prod_i C(b_i, a_i) (zero unless a <= b componentwise)."""
    return comb(b[0], a[0]) * comb(b[1], a[1]) * comb(b[2], a[2])


def _poly_mul(p, q_, max_deg):
    out = {}
    for e1, c1 in p.items():
        d1 = sum(e1)
        for e2, c2 in q_.items():
            if d1 + sum(e2) > max_deg:
                continue
            e = (e1[0] + e2[0], e1[1] + e2[1], e1[2] + e2[2])
            if e in out:
                out[e] = out[e] + c1 * c2
            else:
                out[e] = c1 * c2
    return out


def taylor_coefficients(r, Q):
    """a_gamma(r) for |gamma| <= Q, for a batch of offsets r of shape (n, 3).

    Returns an array (n, n_coeffs(Q)) in multi_indices(Q) order.
    """
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    r2 = np.sum(r * r, axis=1)
    t = {
        (1, 0, 0): 2.0 * r[:, 0] / r2,
        (0, 1, 0): 2.0 * r[:, 1] / r2,
        (0, 0, 1): 2.0 * r[:, 2] / r2,
        (2, 0, 0): 1.0 / r2,
        (0, 2, 0): 1.0 / r2,
        (0, 0, 2): 1.0 / r2,
    }
    ones = np.ones(len(r))
    series = {(0, 0, 0): ones.copy()}
    power = {(0, 0, 0): ones.copy()}
    for n in range(1, Q + 1):
        power = _poly_mul(power, t, Q)
        cn = (-1) ** n * factorial(2 * n) / (4 ** n * factorial(n) ** 2)  # binom(-1/2, n)
        for e, c in power.items():
            series[e] = series.get(e, 0.0) + cn * c
    inv_r = 1.0 / np.sqrt(r2)
    out = np.zeros((len(r), n_coeffs(Q)))
    for col, e in enumerate(multi_indices(Q)):
        if e in series:
            out[:, col] = series[e] * inv_r
    return out


_M2L_STRUCT = {}


def _m2l_structure(q):
    """For |alpha|+|beta| <= q: mask, index of alpha+beta, and (alpha+beta)!/(alpha! beta!) (-1)^|beta| / (4 pi)."""
    if q not in _M2L_STRUCT:
        mis = multi_indices(q)
        pos = {e: n for n, e in enumerate(mis)}
        K = len(mis)
        mask = np.zeros((K, K), dtype=bool)
        gidx = np.zeros((K, K), dtype=np.int64)
        coef = np.zeros((K, K))
        for ia, al in enumerate(mis):
            for ib, be in enumerate(mis):
                if sum(al) + sum(be) > q:
                    continue
                g = (al[0] + be[0], al[1] + be[1], al[2] + be[2])
                mask[ia, ib] = True
                gidx[ia, ib] = pos[g]
                coef[ia, ib] = mi_factorial(g) / (mi_factorial(al) * mi_factorial(be)) * (-1) ** sum(be) / (4.0 * np.pi)
        _M2L_STRUCT[q] = (mask, gidx, coef)
    return _M2L_STRUCT[q]


def m2l_matrix(r, q):
    """T(w, w') for centre offsets r = x_w - x_w' (batch (n, 3)): lambda = T m (Sec. 3).

    T[alpha, beta] = D^{alpha+beta} g(r) / (alpha! beta!) * (-1)^|beta| for |alpha|+|beta| <= q,
    and 0 otherwise, with g = 1/(4 pi |.|), so D^gamma g = gamma! a_gamma / (4 pi).
    """
    mask, gidx, coef = _m2l_structure(q)
    a = taylor_coefficients(r, q)
    return np.ascontiguousarray(np.where(mask[None], coef[None] * a[:, gidx], 0.0))


def m2m_matrix(d, q):
    """M(w, w') for d = x_w' - x_w (child centre minus parent centre): m_w = M m_w' (Sec. 3).

    Moments about the parent from moments about the child:
    (y - x_w)^beta = sum_{gamma <= beta} C(beta, gamma) d^(beta-gamma) (y - x_w')^gamma.
    """
    mis = multi_indices(q)
    K = len(mis)
    M = np.zeros((K, K))
    for ib, be in enumerate(mis):
        for ig, ga in enumerate(mis):
            if all(ga[i] <= be[i] for i in range(3)):
                M[ib, ig] = mi_binom(be, ga) * np.prod([d[i] ** (be[i] - ga[i]) for i in range(3)])
    return M


def l2l_matrix(d, q):
    """L(w', w) for d = x_w' - x_w (child centre minus parent centre): lambda_w' += L lambda_w (Sec. 3).

    sum_beta lambda^beta (x - x_w)^beta re-expanded about x_w':
    lambda'^alpha = sum_{beta >= alpha} C(beta, alpha) d^(beta-alpha) lambda^beta.
    """
    mis = multi_indices(q)
    K = len(mis)
    Lm = np.zeros((K, K))
    for ia, al in enumerate(mis):
        for ib, be in enumerate(mis):
            if all(al[i] <= be[i] for i in range(3)):
                Lm[ia, ib] = mi_binom(be, al) * np.prod([d[i] ** (be[i] - al[i]) for i in range(3)])
    return Lm


def monomials(x, q):
    """x^alpha for points x of shape (..., 3), all |alpha| <= q: returns (..., n_coeffs(q))."""
    x = np.asarray(x, dtype=np.float64)
    pw = [[np.ones(x.shape[:-1])] for _ in range(3)]  # pw[axis][e] = x_axis^e
    for ax in range(3):
        for e in range(1, q + 1):
            pw[ax].append(pw[ax][-1] * x[..., ax])
    mis = multi_indices(q)
    out = np.empty(x.shape[:-1] + (len(mis),))
    for n, (i, j, k) in enumerate(mis):
        out[..., n] = pw[0][i] * pw[1][j] * pw[2][k]
    return out
