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
