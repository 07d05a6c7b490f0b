"""Pins of the oracle's exact touching-pair integrals (near-field singular entries).

Independent checks: a closed form for the coincident pair, the self-similarity (additivity
plus degree-5 homogeneity) equations that tie the four equal-size classes together, the
decomposition of the three ratio-2 classes into unit-cube pairs, symmetry and scaling. The
regular (non-touching) unit-cube integrals that enter these identities come from a plain
tensor Gauss-Legendre rule in all six variables, which shares nothing with the oracle's
convolution/Duffy scheme.
"""

import itertools

import numpy as np
import pytest
from mpmath import log, mp, pi, sqrt

from oracle import touching

CLASS_BY_CONTACTS = {0: "self", 1: "face", 2: "edge", 3: "vertex"}


def brute_regular(delta, n=12):
    """int_{[0,1]^3} int_{delta+[0,1]^3} 1/|x-y| by an n^6 tensor Gauss rule (non-touching cubes only)."""
    assert max(abs(d) for d in delta) >= 2
    t, w = np.polynomial.legendre.leggauss(n)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    ds = [(t[:, None] - (delta[ax] + t[None, :])).ravel() for ax in range(3)]
    ww = (w[:, None] * w[None, :]).ravel()
    r2 = ds[0][:, None, None] ** 2 + ds[1][None, :, None] ** 2 + ds[2][None, None, :] ** 2
    W = ww[:, None, None] * ww[None, :, None] * ww[None, None, :]
    return float(np.sum(W / np.sqrt(r2)))


@pytest.fixture(scope="module")
def C():
    return dict(zip(touching.TOUCH_CLASSES, touching.constants(40)))


def unit_pair(delta, C, cache={}):
    """int over unit cubes at integer offset delta: a class constant if they touch, else brute force."""
    d = tuple(sorted(abs(x) for x in delta))
    if max(d) <= 1:
        return C[CLASS_BY_CONTACTS[sum(1 for x in d if x == 1)]]
    if d not in cache:
        cache[d] = brute_regular(d)
    return cache[d]


def test_coincident_cube_closed_form(C):
    # Mean inverse distance of two uniform points in the unit cube (classical closed form).
    mp.dps = 30
    exact = mp.mpf(2) / 5 * (1 + sqrt(2) - 2 * sqrt(3)) - 2 * pi / 3 + 2 * log(1 + sqrt(2)) + 2 * log(2 + sqrt(3))
    assert abs(C["self"] - float(exact)) <= 1e-13 * float(exact)


@pytest.mark.parametrize("name,o", [("self", (0, 0, 0)), ("face", (1, 0, 0)), ("edge", (1, 1, 0)), ("vertex", (1, 1, 1))])
def test_self_similarity(C, name, o):
    """Split both unit cubes into 8 half cubes: C_o = (1/32) sum over the 64 half-cube pairs (a^5 scaling)."""
    total = 0.0
    for c in itertools.product((0, 1), repeat=3):
        for d in itertools.product((0, 1), repeat=3):
            total += unit_pair(tuple(2 * o[i] + d[i] - c[i] for i in range(3)), C)
    assert abs(total / 32.0 - C[name]) <= 1e-13 * C[name]


@pytest.mark.parametrize("name", ["face2", "edge2", "vertex2"])
def test_ratio_two_decomposition(C, name):
    """A side-2 cube is 8 unit cubes: its integral against the unit cube is a sum of unit-pair integrals."""
    (blo, _), (slo, _) = touching.class_geometry(name)
    total = 0.0
    for c in itertools.product((0, 1), repeat=3):
        child_lo = blo + np.array(c)
        total += unit_pair(tuple(int(x) for x in (slo - child_lo)), C)
    assert abs(total - C[name]) <= 1e-13 * C[name]


def test_scaling_and_symmetry(C):
    a_lo, a_hi = np.zeros(3), np.ones(3)
    b_lo, b_hi = np.array([1.0, 0.0, 1.0]), np.array([2.0, 1.0, 2.0])
    base = touching.box_pair_integral(a_lo, a_hi, b_lo, b_hi, n=30)
    assert abs(base - C["edge"]) <= 1e-13 * base
    for s in (0.5, 3.0):
        v = touching.box_pair_integral(s * a_lo, s * a_hi, s * b_lo, s * b_hi, n=30)
        assert abs(v - s ** 5 * base) <= 1e-13 * s ** 5 * base
    swapped = touching.box_pair_integral(b_lo, b_hi, a_lo, a_hi, n=30)
    mirrored = touching.box_pair_integral(-a_hi, -a_lo, -b_hi, -b_lo, n=30)
    assert abs(swapped - base) <= 1e-14 * base and abs(mirrored - base) <= 1e-14 * base


@pytest.mark.parametrize("delta", [(2, 0, 0), (2, 1, 0), (3, 1, 1), (2, 2, 2)])
def test_regular_branch_matches_brute_force(delta):
    lo = np.array(delta, dtype=float)
    v = touching.box_pair_integral(np.zeros(3), np.ones(3), lo, lo + 1.0, n=30)
    assert abs(v - brute_regular(delta)) <= 1e-13 * v


def test_rule_converged():
    c30, c40 = touching.constants(30), touching.constants(40)
    assert np.max(np.abs(c30 - c40) / c40) < 2e-14
