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
