"""Pins of O2, Algorithm 1 step by step."""

import numpy as np
import pytest

import synth
from oracle import direct, fmm
from oracle.mesh import BCMesh


def rel_l2(lv, u, ref):
    vol = np.ldexp(1.0, -3 * lv[:, 0].astype(np.int32))
    return np.sqrt(np.sum(vol * ((u - ref) / vol) ** 2) / np.sum(vol * (ref / vol) ** 2))


@pytest.fixture(scope="module")
def mesh3():
    m = BCMesh(3)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=0)
    return m, lv, f, direct.apply(lv, 3, f)


def test_converges_to_direct(mesh3):
    """O2 - O1 (the truncation error) decreases geometrically in q (stated: 5e-5, 1.2e-6, 6.8e-8 for q=2,4,6)."""
    m, lv, f, u1 = mesh3
    errs = [rel_l2(lv, fmm.apply(m, f, q), u1) for q in (2, 4, 6)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] < 1e-4 and errs[2] < 2e-7


def test_fixed_order_operator_is_symmetric(mesh3):
    """With fixed q the truncated two-centre Taylor kernel is symmetric, so v.(A_q f) = f.(A_q v)."""
    m, lv, f, _ = mesh3
    v = synth.leaf_density(lv, seed=5)
    F = fmm.FMM(m, 4)
    lhs, rhs = v @ F.apply(f), f @ F.apply(v)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_sampled_equals_full():
    m = BCMesh(4)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=3)
    F = fmm.FMM(m, 4)
    full = F.apply(f)
    tg = np.array([0, 3, 400, 1111, 2527])
    assert np.max(np.abs(F.apply_sampled(f, tg) - full[tg]) / np.abs(full[tg])) < 1e-14


def test_level_rule_fmm_converges_to_its_direct_operator():
    """Neighbour marking (Sec. 2) and the level-dependent near-field rule: O2 tends to the operator
    with that rule on the near pairs and the 2x2x2 rule elsewhere (oracle.direct.apply_near_order)
    as q grows (stated at h = 1/32: 1.4e-6 and 8.0e-8 for q = 4 and 6)."""
    m = BCMesh(5, 1)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=0)
    tg = np.arange(0, len(lv), 191)
    u1 = direct.apply_near_order(m, f, tg)
    errs = [np.linalg.norm(fmm.FMM(m, q, near_order=1).apply_sampled(f, tg) - u1) / np.linalg.norm(u1)
            for q in (4, 6)]
    assert errs[0] > errs[1]
    assert errs[0] < 3e-6 and errs[1] < 2e-7


def _rel(lv, u, ref):
    vol = np.ldexp(1.0, -3 * lv[:, 0].astype(np.int32))
    return np.sqrt(np.sum(vol * ((u - ref) / vol) ** 2) / np.sum(vol * (ref / vol) ** 2))


def test_constant_level_orders_are_the_fixed_order_method(mesh3):
    """The per-level code path with q_l = q on every level is the fixed-q O2, value for value."""
    m, lv, f, _ = mesh3
    assert np.array_equal(fmm.FMM(m, 4, q_levels=[4] * 4).apply(f), fmm.FMM(m, 4).apply(f))


def test_level_schedule_error_falls_with_L():
    """Orders q_l = q0 + L - l (Sec. 4, the FMM error bound with level-dependent orders): the FMM
    error against O1 falls geometrically as L grows at fixed q0, while the fixed order stalls
    (stated for q0 = 4 at h = 1/8, 1/16, 1/32: schedule 2.7e-7, 1.1e-7, 2.8e-8; fixed q = 4 about
    1.2e-6 at every h)."""
    errs_s, errs_f = [], []
    for L in (3, 4, 5):
        m = BCMesh(L)
        lv = m.leaf_array()
        f = synth.leaf_density(lv, seed=0)
        tg = np.arange(0, len(lv), max(1, len(lv) // 400))
        u1 = direct.apply(lv, L, f, tg)
        errs_s.append(_rel(lv[tg], fmm.FMM(m, 4, q_schedule=1).apply_sampled(f, tg), u1))
        errs_f.append(_rel(lv[tg], fmm.FMM(m, 4).apply_sampled(f, tg), u1))
    assert errs_s[0] > errs_s[1] > errs_s[2] and errs_s[2] < 6e-8
    assert all(e > 5e-7 for e in errs_f) and all(s < 0.3 * e for s, e in zip(errs_s, errs_f))


def test_level_schedule_converges_in_q0():
    """With the schedule, O2 -> O1 as the finest order q0 grows (stated at h = 1/16: 3.7e-6, 1.0e-6,
    1.1e-7 for q0 = 2, 3, 4)."""
    m = BCMesh(4)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=1)
    tg = np.arange(0, len(lv), 5)
    u1 = direct.apply(lv, 4, f, tg)
    errs = [_rel(lv[tg], fmm.FMM(m, q0, q_schedule=1).apply_sampled(f, tg), u1) for q0 in (2, 3, 4)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 3e-7


def _subtree_moments(m, lv, f, lev, c, order):
    """Brute force: sum over the leaves inside cell (lev, c) of f times the 2x2x2 point rule of
    (x - x_c)^b, |b| <= order, about the cell's own centre."""
    from oracle.taylor import monomials

    a = m.side(lev)
    centre = (np.asarray(c, dtype=np.float64) + 0.5) * a
    inside = (lv[:, 1:] >> (lv[:, :1] - lev)) == np.asarray(c)
    sel = np.nonzero((lv[:, 0] >= lev) & inside.all(axis=1))[0]
    side = np.ldexp(1.0, -lv[sel, 0].astype(np.int32))
    pts, w = direct.gauss_points(lv[sel, 1:] * side[:, None], side)
    mono = monomials(pts - centre, order)  # (n, 8, K)
    return np.einsum("n,ngk->k", f[sel] * w, mono)


def test_exact_moments_are_the_subtree_moments():
    """The exact-moment reading (every cell's moments to the largest level order, M2M untruncated):
    each marked cell's moments equal the point-rule moments of all of its leaves about its centre,
    computed directly (the shift of a polynomial is exact). The reading as printed loses the
    parents' top-degree terms: there the same comparison fails at degree q_l."""
    from oracle.taylor import n_coeffs

    L = 4
    m = BCMesh(L)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=2)
    ex = fmm.FMM(m, 3, q_schedule=1, exact_moments=True)
    pr = fmm.FMM(m, 3, q_schedule=1)
    assert ex.qm_of == [3 + L - 0] * (L + 1) and pr.qm_of == pr.q_of
    mom_ex = ex.upward(ex.moments(f))
    mom_pr = pr.upward(pr.moments(f))
    worst_pr = 0.0
    checked = 0
    for lev in (1, 2, 3):
        for p, c in enumerate(m.levels[lev]):
            if not m.is_refined(lev, c) or p % 3:
                continue
            ref = _subtree_moments(m, lv, f, lev, c, ex.qm_of[lev])
            scale = np.max(np.abs(ref))
            assert np.max(np.abs(mom_ex[lev][p] - ref)) <= 1e-13 * scale
            k0, k = n_coeffs(pr.q_of[lev] - 1), n_coeffs(pr.q_of[lev])  # the degree-q_l block
            top = np.max(np.abs(ref[k0:k]))
            worst_pr = max(worst_pr, np.max(np.abs(mom_pr[lev][p][k0:k] - ref[k0:k])) / top)
            checked += 1
    assert checked >= 10 and worst_pr > 1e-3


def test_exact_moments_converge_to_direct():
    """With the schedule, the exact-moment reading also tends to O1 as q0 grows, and at every q0 it
    is at least as close to O1 as the reading as printed (it only adds moment terms)."""
    m = BCMesh(4)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=1)
    tg = np.arange(0, len(lv), 5)
    u1 = direct.apply(lv, 4, f, tg)
    ex = [_rel(lv[tg], fmm.FMM(m, q0, q_schedule=1, exact_moments=True).apply_sampled(f, tg), u1) for q0 in (2, 3, 4)]
    pr = [_rel(lv[tg], fmm.FMM(m, q0, q_schedule=1).apply_sampled(f, tg), u1) for q0 in (2, 3, 4)]
    assert ex[0] > ex[1] > ex[2] and ex[2] < 3e-7
    assert all(e <= 1.05 * p for e, p in zip(ex, pr))
