"""Level-dependent expansion orders q_l = q + L - l (Sec. 4) on cuda:0, through the C ABI, against
the CPU oracle's Algorithm 1 with the same orders.

Bar: FP64 relative L2(Omega) error <= 1e-10 against O2 with the schedule; mixed precision <= 1e-6.
"""

import sys

import numpy as np
import pytest

import paper_2112_00864_amd as bcv
import synth
from gpu_util import gpu_apply, rel_l2
from oracle import fmm
from oracle.mesh import BCMesh

pytestmark = pytest.mark.gpu
TOL = 1e-10


def announce(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_MESH = {}


def mesh(L, marking=0):
    if (L, marking) not in _MESH:
        m = BCMesh(L, marking)
        _MESH[(L, marking)] = (m, m.leaf_array())
    return _MESH[(L, marking)]


@pytest.mark.parametrize("L,q,nearfield", [(3, 4, bcv.NEAR_QUADRATURE), (4, 4, bcv.NEAR_ASSEMBLED),
                                           (4, 6, bcv.NEAR_QUADRATURE), (4, 8, bcv.NEAR_QUADRATURE)])
def test_schedule_matches_O2(L, q, nearfield):
    """Orders q .. q + L - 2 on levels L .. 2 (at L = 4, q = 8: orders 8, 9, 10)."""
    m, lv = mesh(L)
    f = synth.leaf_density(lv, seed=1)
    announce("schedule L=%d q=%d nearfield %d n=%d" % (L, q, nearfield, len(lv)))
    plan = bcv.plan_interactions(bcv.build_bc_tree(L), q=q, q_schedule=1, nearfield=nearfield)
    F = fmm.FMM(m, q, q_schedule=1)
    ref = F.apply(f)
    u_far = gpu_apply(plan, f, bcv.PART_FAR)
    u = gpu_apply(plan, f)
    e_far = rel_l2(lv, u_far, ref - F.near_field(f, np.arange(len(lv))))
    e = rel_l2(lv, u, ref)
    announce("schedule L=%d q=%d rel-L2 far %.3e total %.3e" % (L, q, e_far, e))
    assert e_far <= TOL and e <= TOL


def test_schedule_neighbour_marking_sampled():
    """h = 1/32 with the neighbour marking (levels 4 and 5 hold leaves), q = 4: orders 4 .. 7."""
    L, q = 5, 4
    m, lv = mesh(L, 1)
    f = synth.leaf_density(lv, seed=2)
    announce("schedule neighbour marking L=%d q=%d" % (L, q))
    plan = bcv.plan_interactions(bcv.build_bc_tree(L, 1), q=q, q_schedule=1)
    u = gpu_apply(plan, f)
    tg = np.unique(np.concatenate([np.arange(0, len(lv), 131), [len(lv) - 1]]))
    ref = fmm.FMM(m, q, q_schedule=1).apply_sampled(f, tg)
    e = rel_l2(lv[tg], u[tg], ref)
    announce("schedule neighbour marking rel-L2 %.3e" % e)
    assert e <= TOL


def test_schedule_mixed_precision():
    L, q = 5, 4
    m, lv = mesh(L)
    f = synth.leaf_density(lv, seed=3)
    t = bcv.build_bc_tree(L)
    announce("schedule mixed vs fp64 L=%d q=%d" % (L, q))
    a = gpu_apply(bcv.plan_interactions(t, q=q, q_schedule=1), f)
    b = gpu_apply(bcv.plan_interactions(t, q=q, q_schedule=1, precision=bcv.MIXED_F32), f)
    c = gpu_apply(bcv.plan_interactions(t, q=q, q_schedule=1, precision=bcv.MIXED_F32,
                                        nearfield=bcv.NEAR_ASSEMBLED), f)
    e, e_a = rel_l2(lv, b, a), rel_l2(lv, c, a)
    announce("schedule mixed rel-L2 %.3e, assembled %.3e" % (e, e_a))
    assert e <= 1e-6 and e_a <= 1e-6


def test_schedule_full_size_sampled():
    """h = 1/128 (L = 7, 219,080 leaves), q = 4: orders 4 .. 9, against O2 at 60 sampled leaves."""
    L, q = 7, 4
    m, lv = mesh(L)
    f = synth.leaf_density(lv, seed=0)
    announce("schedule full size L=7 q=4: plan")
    plan = bcv.plan_interactions(bcv.build_bc_tree(L), q=q, q_schedule=1, nearfield=bcv.NEAR_ASSEMBLED)
    u = gpu_apply(plan, f)
    tg = np.random.default_rng(1).choice(len(lv), 60, replace=False)
    announce("schedule full size L=7: oracle at 60 leaves")
    ref = fmm.FMM(m, q, q_schedule=1).apply_sampled(f, tg)
    e = np.max(np.abs(u[tg] - ref) / np.abs(ref))
    announce("schedule full size max rel %.3e" % e)
    assert e <= TOL


def test_schedule_option_errors():
    t = bcv.build_bc_tree(7)
    with pytest.raises(bcv.BCVError) as e:  # q + L - 2 = 11 > 10
        bcv.plan_interactions(t, q=6, q_schedule=1)
    assert e.value.status == bcv.bcv.EINVAL
    with pytest.raises(bcv.BCVError) as e:
        bcv.plan_interactions(bcv.build_bc_forest([3, 4]), q=4, q_schedule=1)
    assert e.value.status == bcv.bcv.ENOTSUP


@pytest.mark.parametrize("L,q,precision", [(3, 4, bcv.FP64), (4, 4, bcv.FP64), (4, 6, bcv.FP64),
                                           (4, 4, bcv.MIXED_F32)])
def test_exact_moments_match_O2(L, q, precision):
    """The exact-moment reading of the upward pass (every cell's moments to the largest order) against
    O2 with the same reading. The two readings give different operators (the printed one drops the
    parents' top-degree terms, which are small: 5e-10 at L = 4, q = 4), and the FP64 GPU result is
    far closer to its own reading's O2 than to the other's."""
    m, lv = mesh(L)
    f = synth.leaf_density(lv, seed=2)
    announce("schedule, exact moments, L=%d q=%d precision %d" % (L, q, precision))
    tree = bcv.build_bc_tree(L)
    u = gpu_apply(bcv.plan_interactions(tree, q=q, q_schedule=1, exact_moments=True, precision=precision,
                                        nearfield=bcv.NEAR_ASSEMBLED), f)
    ref = fmm.FMM(m, q, q_schedule=1, exact_moments=True).apply(f)
    e = rel_l2(lv, u, ref)
    printed = fmm.FMM(m, q, q_schedule=1).apply(f)
    d = rel_l2(lv, printed, ref)
    announce("exact moments L=%d q=%d: vs O2 %.3e (the printed reading differs by %.3e)" % (L, q, e, d))
    assert e <= (TOL if precision == bcv.FP64 else 1e-6)
    # The GPU follows its own reading, not the other one. At L = 3 the readings coincide: the only
    # dropped terms are the leaves' moments of odd degree q_3 + 1 about their centres, which the
    # symmetric 2x2x2 rule makes zero.
    if precision == bcv.FP64 and L >= 4:
        assert d > 100 * e
