"""Pins of the oracle's Taylor coefficients and translation matrices (Sec. 3, translation operators)."""

import numpy as np
import pytest
from mpmath import diff, mp, mpf
from mpmath import sqrt as msqrt

from oracle import taylor


def test_multi_index_count_and_order():
    for q in range(9):
        mis = taylor.multi_indices(q)
        assert len(mis) == taylor.n_coeffs(q) == len(set(mis))
        assert [sum(m) for m in mis] == sorted(sum(m) for m in mis)


def test_low_order_closed_forms():
    r = np.array([[0.7, -1.3, 0.4]])
    x, y, z = r[0]
    R = np.linalg.norm(r)
    a = taylor.taylor_coefficients(r, 2)[0]
    pos = {e: n for n, e in enumerate(taylor.multi_indices(2))}
    assert np.isclose(a[pos[(0, 0, 0)]], 1 / R, rtol=1e-15)
    assert np.isclose(a[pos[(1, 0, 0)]], -x / R ** 3, rtol=1e-14)
    assert np.isclose(a[pos[(2, 0, 0)]], (3 * x * x - R * R) / (2 * R ** 5), rtol=1e-14)
    assert np.isclose(a[pos[(1, 1, 0)]], 3 * x * y / R ** 5, rtol=1e-14)


@pytest.mark.parametrize("gamma", [(3, 0, 0), (1, 2, 1), (2, 2, 2), (0, 1, 5), (4, 1, 1)])
def test_against_high_precision_derivatives(gamma):
    mp.dps = 40
    r = (mpf("0.9"), mpf("-0.35"), mpf("1.6"))
    d = diff(lambda x, y, z: 1 / msqrt(x * x + y * y + z * z), r, gamma)
    fact = 1
    for g in gamma:
        for k in range(2, g + 1):
            fact *= k
    pos = {e: n for n, e in enumerate(taylor.multi_indices(6))}
    a = taylor.taylor_coefficients(np.array([[0.9, -0.35, 1.6]]), 6)[0]
    assert abs(a[pos[gamma]] - float(d / fact)) <= 1e-12 * abs(float(d / fact)) + 1e-15


def test_harmonic():
    """Laplace: sum_i d^{gamma+2e_i} (1/r) = 0, i.e. sum_i (gamma+2e_i)! a_{gamma+2e_i} = 0."""
    q = 8
    mis = taylor.multi_indices(q)
    pos = {e: n for n, e in enumerate(mis)}
    a = taylor.taylor_coefficients(np.array([[1.1, 0.3, -0.8]]), q)[0]
    for g in mis:
        if sum(g) > q - 2:
            continue
        tot, scale = 0.0, 0.0
        for i in range(3):
            h = list(g)
            h[i] += 2
            h = tuple(h)
            v = taylor.mi_factorial(h) * a[pos[h]]
            tot += v
            scale += abs(v)
        assert abs(tot) <= 1e-12 * scale


def test_series_converges_with_legendre_bound():
    r = np.array([[0.8, -0.5, 1.2]])
    R = np.linalg.norm(r)
    h = np.array([0.2, 0.25, -0.15])
    rho = np.linalg.norm(h) / R
    exact = 1.0 / np.linalg.norm(r[0] + h)
    for Q in (2, 4, 6, 8, 10):
        a = taylor.taylor_coefficients(r, Q)[0]
        approx = a @ taylor.monomials(h, Q)
        bound = rho ** (Q + 1) / (R * (1.0 - rho))  # |P_n| <= 1
        assert abs(approx - exact) <= bound


def test_m2m_and_l2l_are_exact_reexpansions():
    rng = np.random.default_rng(1)
    q = 6
    xc, xp = np.array([0.1, 0.2, -0.05]), np.array([0.0, 0.1, 0.05])
    y = xc + 0.05 * rng.standard_normal((20, 3))
    mc = taylor.monomials(y - xc, q).sum(axis=0)
    mp_ = taylor.monomials(y - xp, q).sum(axis=0)
    assert np.allclose(taylor.m2m_matrix(xc - xp, q) @ mc, mp_, rtol=1e-12, atol=1e-15)
    lam = rng.standard_normal(taylor.n_coeffs(q))
    x = xc + 0.05 * rng.standard_normal((20, 3))
    direct = taylor.monomials(x - xp, q) @ lam
    child = taylor.monomials(x - xc, q) @ (taylor.l2l_matrix(xc - xp, q) @ lam)
    assert np.allclose(direct, child, rtol=1e-12, atol=1e-14)


def test_m2l_sign_convention_single_source():
    """lambda = T m from a point source reproduces G(x, y) with the geometric Taylor error."""
    xw, xs = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.4, -0.3])
    y = xs + np.array([0.1, -0.05, 0.08])
    x = xw + np.array([-0.07, 0.06, 0.02])
    exact = 1.0 / (4 * np.pi * np.linalg.norm(x - y))
    errs = []
    for q in (2, 4, 6, 8):
        m = taylor.monomials(y - xs, q)
        T = taylor.m2l_matrix((xw - xs)[None], q)[0]
        approx = taylor.monomials(x - xw, q) @ (T @ m)
        errs.append(abs(approx - exact) / exact)
    assert all(b < a for a, b in zip(errs, errs[1:])) and errs[-1] < 1e-6
