"""Pins of O1, the direct Galerkin evaluation u = A f."""

import math

import numpy as np
import pytest

import synth
from closed_forms import ball_potential, box_potential_cell_averages
from oracle import direct, touching
from oracle.mesh import BCMesh


def naive_entry(t, s, C):
    """A_ts from scratch in long double: float box geometry, Python loops over the 64 point pairs."""
    (lt, it, jt, kt), (ls, is_, js, ks) = t, s
    at, as_ = 2.0 ** -lt, 2.0 ** -ls
    lo_t, lo_s = (it * at, jt * at, kt * at), (is_ * as_, js * as_, ks * as_)
    contacts, touch = 0, True
    for ax in range(3):
        lo, hi = max(lo_t[ax], lo_s[ax]), min(lo_t[ax] + at, lo_s[ax] + as_)
        if lo > hi:
            touch = False
        elif lo == hi:
            contacts += 1
    four_pi = np.longdouble(4) * np.longdouble(math.pi)
    if touch:
        if at == as_:
            name = ["self", "face", "edge", "vertex"][contacts]
        else:
            name = ["", "face2", "edge2", "vertex2"][contacts]
        a = np.longdouble(min(at, as_))
        return np.longdouble(C[name]) * a ** 5 / four_pi
    xi = [np.longdouble(0.5) - np.longdouble(0.5) / np.sqrt(np.longdouble(3)),
          np.longdouble(0.5) + np.longdouble(0.5) / np.sqrt(np.longdouble(3))]
    tot = np.longdouble(0)
    for g in range(8):
        x = [lo_t[ax] + at * xi[(g >> ax) & 1] for ax in range(3)]
        for h in range(8):
            y = [lo_s[ax] + as_ * xi[(h >> ax) & 1] for ax in range(3)]
            tot += 1 / np.sqrt(sum((x[ax] - y[ax]) ** 2 for ax in range(3)))
    return tot * (np.longdouble(at) ** 3 / 8) * (np.longdouble(as_) ** 3 / 8) / four_pi


@pytest.fixture(scope="module")
def C():
    return dict(zip(touching.TOUCH_CLASSES, touching.constants(40)))


@pytest.mark.parametrize("L,rows", [(2, None), (3, [0, 7, 100, 228, 455])])
def test_brute_force(L, rows, C):
    m = BCMesh(L)
    lv = m.leaf_array()
    A = direct.matrix(lv, L)
    rows = range(len(lv)) if rows is None else rows
    for t in rows:
        ref = np.array([naive_entry(tuple(lv[t]), tuple(lv[s]), C) for s in range(len(lv))], dtype=np.longdouble)
        assert np.max(np.abs(A[t] - ref) / ref) < 1e-14


def test_symmetric_and_positive():
    m = BCMesh(3)
    A = direct.matrix(m.leaf_array(), 3)
    assert np.all(A > 0)
    assert np.max(np.abs(A - A.T) / A) < 1e-14  # 64-term sums in swapped order round differently


def _rel_l2(lv, u, exact_avg):
    vol = np.ldexp(1.0, -3 * lv[:, 0].astype(np.int32))
    ub = u / vol
    return np.sqrt(np.sum(vol * (ub - exact_avg) ** 2) / np.sum(vol * exact_avg ** 2))


def test_constant_density_against_box_closed_form():
    """f = 1 is represented exactly, so only the 2x2x2 point rule on non-touching pairs errs (stated: 3.2e-5)."""
    L = 4
    lv = BCMesh(L).leaf_array()
    u = direct.apply(lv, L, np.ones(len(lv)))
    e = _rel_l2(lv, u, box_potential_cell_averages(lv))
    assert 1e-6 < e < 5e-5


def test_uniform_ball():
    """Ball density projected on the BC mesh (8^3-point cell averages): stated error ~1e-2 (coarse interior)."""
    L = 4
    lv = BCMesh(L).leaf_array()
    f = synth.cell_average(lv, synth.ball_indicator(), n=8)
    u = direct.apply(lv, L, f)
    t, w = np.polynomial.legendre.leggauss(6)
    t, w = 0.5 * (t + 1), 0.5 * w
    X, Y, Z = np.meshgrid(t, t, t, indexing="ij")
    W = np.einsum("i,j,k->ijk", w, w, w).ravel()
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    a = np.ldexp(1.0, -lv[:, 0].astype(np.int32))
    pts = lv[:, 1:4] * a[:, None]
    exact = ball_potential(pts[:, None, :] + a[:, None, None] * nodes[None]) @ W
    assert _rel_l2(lv, u, exact) < 1.5e-2


def test_numpy_and_c_entries_agree():
    m = BCMesh(3)
    lv = m.leaf_array()
    n = len(lv)
    ti, si = np.repeat(np.arange(n), n), np.tile(np.arange(n), n)
    a, b = direct.entries(lv, 3, ti, si), direct.entries_numpy(lv, 3, ti, si)
    assert np.max(np.abs(a - b) / b) < 1e-14


# -- level-dependent near-field rule (Sec. 4, near-field quadrature) --------------------------------

def test_gauss_rule_c_matches_numpy():
    """The C loop of the tensor rule against an independent NumPy evaluation, mixed orders."""
    from oracle import _clib

    rng = np.random.default_rng(7)
    gx, gw = direct.gauss_tables()
    for _ in range(12):
        lo_t = rng.random(3)
        lo_s = lo_t + rng.choice([-1, 1], 3) * (0.8 + rng.random(3))
        a_t, a_s = rng.choice([0.25, 0.5, 1.0], 2)
        n_t, n_s = (int(v) for v in rng.integers(1, 8, 2))
        c = _clib.lib().o1_gauss_rule(lo_t, a_t, n_t, lo_s, a_s, n_s, gx, gw)
        assert abs(c - direct.gauss_rule(lo_t, a_t, n_t, lo_s, a_s, n_s)) <= 1e-14 * abs(c)


def test_gauss_rule_two_points_is_the_point_rule():
    from oracle import _clib

    lo_t, lo_s = np.array([0.0, 0.0, 0.0]), np.array([0.5, 0.25, 0.0])
    gx, gw = direct.gauss_tables()
    two = _clib.lib().o1_gauss_rule(lo_t, 0.25, 2, lo_s, 0.125, 2, gx, gw)
    ref = direct.point_rule(lo_t[None], np.array([0.25]), lo_s[None], np.array([0.125]))[0]
    assert abs(two - ref) <= 1e-15 * ref


@pytest.mark.parametrize("lo_s,a_s", [((2.0, 1.0, 0.0), 1.0), ((1.5, 0.0, 0.0), 0.5), ((-1.25, 0.5, 1.0), 0.25)])
def test_gauss_rule_converges_to_the_exact_integral(lo_s, a_s):
    """Non-touching cube pairs of a near field (gaps of a quarter to one cell): the tensor rule tends
    to the exact integral (oracle.touching's convolution quadrature) as the order grows."""
    lo_t = np.zeros(3)
    exact = touching.box_pair_integral(lo_t, lo_t + 1.0, np.array(lo_s), np.array(lo_s) + a_s, n=30) / (4 * np.pi)
    errs = [abs(direct.gauss_rule(lo_t, 1.0, n, lo_s, a_s, n) - exact) / exact for n in (2, 3, 4, 6, 8)]
    assert all(e1 > e2 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-7


def test_level_rule_entries_symmetric_and_only_on_coarse_pairs():
    L = 4
    m = BCMesh(L)
    lv = m.leaf_array()
    orders = direct.near_gauss_orders(lv, L, 1)
    assert np.array_equal(orders, 2 + L - lv[:, 0])
    ti, si = m.near_pairs()
    a = direct.entries(lv, L, ti, si, orders)
    b = direct.entries(lv, L, si, ti, orders)
    assert np.max(np.abs(a - b) / a) < 1e-14
    fixed = direct.entries(lv, L, ti, si)
    finest = (lv[ti, 0] == L) & (lv[si, 0] == L)
    lo_int, size, _, _ = direct.leaf_geometry(lv, L)
    touch = direct.touching_class_index(lo_int[ti], size[ti], lo_int[si], size[si]) >= 0
    assert np.array_equal(a[finest | touch], fixed[finest | touch])  # exact, or the finest level's 2x2x2
    assert np.all(a[~finest & ~touch] != fixed[~finest & ~touch])


@pytest.mark.parametrize("L,marking,fixed_err,level_err", [(4, 0, 3.2e-5, 5.1e-6), (5, 1, 3.1e-6, 1.7e-6)])
def test_level_rule_against_box_closed_form(L, marking, fixed_err, level_err):
    """f = 1 (exact density): the level-dependent near-field rule brings the cell potentials closer
    to the homogeneous-box closed form (stated errors: 3.2e-5 -> 5.1e-6 with the face marking at
    h = 1/16, 3.1e-6 -> 1.7e-6 with the neighbour marking at h = 1/32, sampled leaves)."""
    m = BCMesh(L, marking)
    lv = m.leaf_array()
    tg = np.arange(0, len(lv), 1 if len(lv) < 5000 else 7)
    ex = box_potential_cell_averages(lv[tg])
    e0 = _rel_l2(lv[tg], direct.apply(lv, L, np.ones(len(lv)), tg), ex)
    e1 = _rel_l2(lv[tg], direct.apply_near_order(m, np.ones(len(lv)), tg), ex)
    assert e1 < e0
    assert abs(e0 - fixed_err) < 0.05 * fixed_err and abs(e1 - level_err) < 0.05 * level_err
