"""Pins of the degree-p leaf-basis oracle (oracle.basis and touching.box_pair_poly) against what
the mathematics fixes, independently of the oracle's own code paths:

* polynomial-weighted box integrals: degree 0 equals the seven touching constants; separated
  boxes against a plain 6-D Gauss rule; the swap and reflection symmetries; the two-scale
  refinement identity on touching pairs (a parent pair equals the sum of its 64 child pairs with
  the Legendre weights re-expanded on the children), which ties the singular sub-boxes of one
  scale to the regular ones of the next;
* degree 0 everywhere reproduces O1 and O2 of the p = 0 operator;
* symmetry of the Galerkin blocks; O2 -> O1 as q grows (stated values);
* the projection reproduces polynomials of degree <= p exactly;
* the homogeneous cube (f = 1): the Galerkin moments <phi^alpha, N 1> against the closed-form
  potential, and the paper's O(h) rate of the best approximation with p_l = L - l (Sec. 4,
  approximation errors), which degree 0 on the coarse leaves does not reach.
"""

import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))

import synth  # noqa: E402
from closed_forms import box_potential  # noqa: E402

from oracle import basis, direct, fmm, touching  # noqa: E402
from oracle.mesh import BCMesh  # noqa: E402


def gauss6(alo, ahi, blo, bhi, pa, pb, n=14):
    """Plain tensor Gauss rule for separated boxes with Legendre weights (all degree tuples)."""
    t, w = np.polynomial.legendre.leggauss(n)
    t, w = 0.5 * (t + 1.0), 0.5 * w

    def pts(lo, hi, p):
        X = np.stack(np.meshgrid(*[lo[i] + (hi[i] - lo[i]) * t for i in range(3)], indexing="ij"), -1).reshape(-1, 3)
        W = np.einsum("i,j,k->ijk", w, w, w).ravel() * np.prod(hi - lo)
        c, s = 0.5 * (lo + hi), hi - lo
        P = [np.polynomial.legendre.legvander(2.0 * (X[:, i] - c[i]) / s[i], p) for i in range(3)]  # (N, p+1)
        return X, W, np.einsum("na,nb,nc->nabc", P[0], P[1], P[2]).reshape(len(X), -1)

    X, WX, PX = pts(alo, ahi, pa)
    Y, WY, PY = pts(blo, bhi, pb)
    K = 1.0 / np.sqrt(((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1))
    return ((PX * WX[:, None]).T @ K @ (PY * WY[:, None])).reshape((pa + 1,) * 3 + (pb + 1,) * 3)


def test_degree_zero_is_the_touching_constants():
    for name in touching.TOUCH_CLASSES:
        (al, ah), (bl, bh) = touching.class_geometry(name)
        v = touching.box_pair_poly(al, ah, bl, bh, 0, 0).ravel()[0]
        assert abs(v - touching.touching_constant(name)) <= 1e-14 * v


@pytest.mark.parametrize("boxes", [
    ((0, 0, 0), (1, 1, 1), (2, 0, 0), (3, 1, 1)),
    ((0, 0, 0), (1, 1, 1), (2, -1, 3), (3, 0, 4)),
    ((0, 0, 0), (2, 2, 2), (3, 0.5, 1), (4, 1.5, 2)),
])
def test_separated_boxes_against_plain_gauss(boxes):
    al, ah, bl, bh = (np.array(b, dtype=np.float64) for b in boxes)
    A = touching.box_pair_poly(al, ah, bl, bh, 3, 2)
    B = gauss6(al, ah, bl, bh, 3, 2)
    assert np.max(np.abs(A - B)) <= 1e-13 * np.max(np.abs(B))


@pytest.mark.parametrize("name", ["self", "face", "edge", "vertex", "face2", "edge2", "vertex2"])
def test_swap_and_reflection_symmetry(name):
    (al, ah), (bl, bh) = touching.class_geometry(name)
    T = touching.box_pair_poly(al, ah, bl, bh, 3, 2)
    S = touching.box_pair_poly(bl, bh, al, ah, 2, 3)  # the pair swapped
    assert np.max(np.abs(T - S.transpose(3, 4, 5, 0, 1, 2))) <= 1e-13 * np.max(np.abs(T))
    # reflection x -> -x of both boxes flips P_k by (-1)^k on each side
    R = touching.box_pair_poly(-ah * np.array([1, 0, 0]) + al * np.array([0, 1, 1]),
                               -al * np.array([1, 0, 0]) + ah * np.array([0, 1, 1]),
                               -bh * np.array([1, 0, 0]) + bl * np.array([0, 1, 1]),
                               -bl * np.array([1, 0, 0]) + bh * np.array([0, 1, 1]), 3, 2)
    sign = np.fromfunction(lambda ax, ay, az, bx, by, bz: (-1.0) ** (ax + bx), T.shape)
    assert np.max(np.abs(R - sign * T)) <= 1e-13 * np.max(np.abs(T))


def _child_reexpansion(p, half):
    """R[a, a'] with P_a(t) = sum_a' R[a, a'] P_a'(t') on the lower (half 0) or upper (half 1)
    half of [-1, 1], t = (t' - 1)/2 or (t' + 1)/2; by Gauss projection."""
    t, w = np.polynomial.legendre.leggauss(p + 2)
    Pc = np.polynomial.legendre.legvander(t, p)  # P_a'(t')
    Pp = np.polynomial.legendre.legvander(0.5 * t + (0.5 if half else -0.5), p)  # P_a(parent t)
    return (Pp * w[:, None]).T @ Pc * ((2 * np.arange(p + 1) + 1) / 2.0)[None, :]


@pytest.mark.parametrize("name", ["self", "face", "edge", "vertex"])
def test_two_scale_refinement_of_touching_pairs(name):
    p = 2
    (al, ah), (bl, bh) = touching.class_geometry(name)
    parent = touching.box_pair_poly(al, ah, bl, bh, p, p)
    R = [_child_reexpansion(p, h) for h in (0, 1)]
    total = np.zeros_like(parent)
    for c in range(8):
        cpos = np.array([(c >> ax) & 1 for ax in range(3)])
        clo = al + 0.5 * cpos
        for d in range(8):
            dpos = np.array([(d >> ax) & 1 for ax in range(3)])
            dlo = bl + 0.5 * dpos
            J = touching.box_pair_poly(clo, clo + 0.5, dlo, dlo + 0.5, p, p)
            total += np.einsum("ai,bj,ck,dl,em,fn,ijklmn->abcdef", R[cpos[0]], R[cpos[1]], R[cpos[2]],
                               R[dpos[0]], R[dpos[1]], R[dpos[2]], J)
    assert np.max(np.abs(total - parent)) <= 1e-13 * np.max(np.abs(parent))


@pytest.mark.parametrize("L", [2, 3])
def test_degree_zero_reproduces_the_p0_operator(L):
    mesh = BCMesh(L)
    lv = mesh.leaf_array()
    f = synth.leaf_density(lv, seed=0)
    u0 = basis.apply_direct(mesh, f, degree_zero=True)
    u1 = direct.apply(lv, L, f)
    assert np.max(np.abs(u0 - u1) / np.abs(u1)) <= 1e-13
    v0 = basis.BasisFMM(mesh, 4, degree_zero=True).apply_basis(f)
    v1 = fmm.FMM(mesh, 4).apply(f)
    assert np.max(np.abs(v0 - v1) / np.abs(v1)) <= 1e-13


def test_blocks_are_symmetric():
    lf = basis.Leaves(BCMesh(3))
    worst = 0.0
    for t in range(0, len(lf.lv), 11):
        for s in range(0, len(lf.lv), 7):
            B1, B2 = lf.block(t, s), lf.block(s, t)
            worst = max(worst, np.max(np.abs(B1 - B2.T)) / np.max(np.abs(B1)))
    assert worst <= 1e-14


def test_O2_converges_to_O1():
    """Stated at h = 1/8 (dofs 480, random coefficients): 1.6e-4, 6.4e-6, 3.6e-7, 2.9e-8 for
    q = 2, 4, 6, 8."""
    mesh = BCMesh(3)
    lf = basis.Leaves(mesh)
    F = np.random.default_rng(0).standard_normal(lf.off[-1])
    u = basis.apply_direct(mesh, F)
    errs = [np.linalg.norm(basis.BasisFMM(mesh, q).apply_basis(F) - u) / np.linalg.norm(u) for q in (2, 4, 6)]
    assert errs[0] < 3e-4 and errs[1] < 1.2e-5 and errs[2] < 7e-7
    assert errs[0] > 10 * errs[1] > 100 * errs[2]


def test_sampled_O2_equals_full_O2():
    mesh = BCMesh(3)
    lf = basis.Leaves(mesh)
    F = np.random.default_rng(1).standard_normal(lf.off[-1])
    fm = basis.BasisFMM(mesh, 6)
    full = fm.apply_basis(F)
    targets = np.array([0, 5, len(lf.lv) - 1] + list(np.nonzero(lf.p > 0)[0][:3]))
    part = basis.BasisFMM(mesh, 6).apply_basis_sampled(F, targets)
    ref = np.concatenate([full[lf.off[t] : lf.off[t + 1]] for t in targets])
    assert np.max(np.abs(part - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_projection_reproduces_polynomials():
    mesh = BCMesh(4)
    lf = basis.Leaves(mesh)
    poly = lambda x: 1.0 + x[:, 0] - 2.0 * x[:, 1] * x[:, 2] + 0.5 * x[:, 2] ** 2  # noqa: E731 (degree 2)
    F = basis.project(mesh, poly)
    checked = np.nonzero(lf.p >= 2)[0]
    assert len(checked) == 8  # the level-2 leaves of h = 1/16
    for w in checked:
        X, W, Phi = basis.leaf_points(lf.lo[w], lf.a[w], int(lf.p[w]))
        assert np.max(np.abs(Phi @ F[lf.off[w] : lf.off[w + 1]] - poly(X))) <= 1e-13


def _closed_form_errors(L, degree_zero):
    """f = 1: max relative error of the moments <phi^alpha, N 1> (degree 0, and the higher ones
    relative to their largest) and the L2 error of the projection sum u_alpha phi^alpha/||phi^alpha||^2
    against the closed-form potential."""
    mesh = BCMesh(L)
    lf = basis.Leaves(mesh, degree_zero)
    F = np.zeros(lf.off[-1])
    F[lf.off[:-1]] = 1.0
    if degree_zero:  # the p = 0 operator (equal to basis.apply_direct with degree_zero, pinned above)
        u = direct.apply(lf.lv, L, F)
    else:
        u = basis.apply_direct(mesh, F)
    t, w = np.polynomial.legendre.leggauss(10)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    X = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).ravel()
    P = [np.polynomial.legendre.legvander(2.0 * X[:, i] - 1.0, 8) for i in range(3)]
    e0 = n0 = eh = nh = e2 = n2 = 0.0
    for k in range(len(lf.lv)):
        a = lf.a[k]
        U = box_potential(lf.lo[k] + a * X)
        proj = np.zeros(len(X))
        for r, (i, j, kk) in enumerate(basis.basis_indices(int(lf.p[k]))):
            phi = P[0][:, i] * P[1][:, j] * P[2][:, kk]
            exact = np.sum(W * phi * U) * a ** 3
            err = abs(u[lf.off[k] + r] - exact)
            if r == 0:
                e0, n0 = max(e0, err), max(n0, abs(exact))
            else:
                eh, nh = max(eh, err), max(nh, abs(exact))
            proj += u[lf.off[k] + r] * (2 * i + 1) * (2 * j + 1) * (2 * kk + 1) / a ** 3 * phi
        e2 += np.sum(W * (proj - U) ** 2) * a ** 3
        n2 += np.sum(W * U ** 2) * a ** 3
    return e0 / n0, (eh / nh if nh else 0.0), np.sqrt(e2 / n2)


def test_homogeneous_cube_moments():
    """Stated at h = 1/8: degree-0 moments 2.9e-6 (3.3e-5 with degree 0 everywhere: the coarse
    leaves' 2x2x2 rule), higher moments 8.2e-5 of their largest."""
    m0, mh, _ = _closed_form_errors(3, False)
    z0, _, _ = _closed_form_errors(3, True)
    assert m0 <= 4e-6 and mh <= 1.2e-4 and z0 <= 5e-5 and m0 < z0 / 5


def test_order_h_rate_with_level_degrees():
    """The best-approximation error with p_l = L - l halves with h (paper: O(h) with p = 0 on the
    finest level); with degree 0 on the coarse leaves it does not. Stated: 3.56e-2 -> 1.57e-2 (ratio
    0.44) against 3.74e-2 -> 2.61e-2 (0.70), h = 1/8 -> 1/16."""
    _, _, a3 = _closed_form_errors(3, False)
    _, _, a4 = _closed_form_errors(4, False)
    _, _, z3 = _closed_form_errors(3, True)
    _, _, z4 = _closed_form_errors(4, True)
    assert a4 / a3 <= 0.5 and z4 / z3 >= 0.6 and a4 < z4


def test_level_orders_with_degree_bases():
    """The paper's experiment setup, p_l = L - l with q_l = q0 + L - l (Sec. 5): O2 with these orders
    against O1 is more accurate than the fixed q0 and converges as q0 grows (h = 1/8, random
    coefficients; stated 1.4e-6 and 9.6e-8 for q0 = 4 and 6, against 6.4e-6 and 3.6e-7 at fixed q)."""
    mesh = BCMesh(3)
    lf = basis.Leaves(mesh)
    F = np.random.default_rng(0).standard_normal(lf.off[-1])
    u = basis.apply_direct(mesh, F)
    err = {}
    for q0 in (4, 6):
        for sched in (0, 1):
            v = basis.BasisFMM(mesh, q0, q_schedule=sched).apply_basis(F)
            err[(q0, sched)] = np.linalg.norm(v - u) / np.linalg.norm(u)
    assert err[(4, 1)] < err[(4, 0)] and err[(6, 1)] < err[(6, 0)] and err[(6, 1)] < err[(4, 1)] / 10
