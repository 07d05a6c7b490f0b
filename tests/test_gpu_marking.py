"""The neighbour marking rule (Sec. 2) and the level-dependent near-field rule (Sec. 4) on cuda:0,
through the C ABI, against the CPU oracle.

Bar: FP64 relative L2(Omega) error <= 1e-10 against the oracle computing the same operator (O1 in
direct mode, O2 for the FMM); mixed precision <= 1e-6.
"""

import sys

import numpy as np
import pytest

import paper_2112_00864_amd as bcv
import synth
from gpu_util import gpu_apply, rel_l2
from oracle import direct, fmm
from oracle.mesh import BCMesh

pytestmark = pytest.mark.gpu
TOL = 1e-10
MIXED_TOL = 1e-6


def announce(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_MESH = {}


def mesh(L, marking):
    if (L, marking) not in _MESH:
        m = BCMesh(L, marking)
        _MESH[(L, marking)] = (m, m.leaf_array())
    return _MESH[(L, marking)]


@pytest.mark.parametrize("L,marking", [(3, 0), (4, 0), (4, 1)])
def test_level_rule_direct_mode_matches_O1(L, marking):
    """Direct mode (every pair near) with the level-dependent rule: every non-touching pair takes
    the per-leaf Gauss orders 2 + L - l."""
    m, lv = mesh(L, marking)
    f = synth.leaf_density(lv, seed=0)
    announce("direct near_order=1 L=%d marking=%d n=%d" % (L, marking, len(lv)))
    plan = bcv.plan_interactions(bcv.build_bc_tree(L, marking), q=4, direct=True, nearfield=bcv.NEAR_ASSEMBLED,
                                 near_order=1)
    u = gpu_apply(plan, f)
    ref = direct.apply(lv, L, f, orders=direct.near_gauss_orders(lv, L, 1))
    e = rel_l2(lv, u, ref)
    announce("direct near_order=1 L=%d marking=%d rel-L2 %.3e, ordered entries %d" %
             (L, marking, e, plan.info["n_near_ordered"]))
    assert e <= TOL
    assert np.max(np.abs(u - ref) / np.abs(ref)) < 1e-12
    assert (plan.info["n_near_ordered"] > 0) == (marking == 0 or L > 4)


@pytest.mark.parametrize("near_order", [0, 1])
def test_face_marking_level_rule_fmm_matches_O2(near_order):
    L, q = 4, 6
    m, lv = mesh(L, 0)
    f = synth.leaf_density(lv, seed=1)
    announce("fmm face marking L=%d q=%d near_order=%d" % (L, q, near_order))
    plan = bcv.plan_interactions(bcv.build_bc_tree(L), q=q, nearfield=bcv.NEAR_ASSEMBLED, near_order=near_order)
    F = fmm.FMM(m, q, near_order=near_order)
    near_ref = F.near_field(f, np.arange(len(lv)))
    full_ref = F.apply(f)
    e_near = rel_l2(lv, gpu_apply(plan, f, bcv.PART_NEAR), near_ref)
    e = rel_l2(lv, gpu_apply(plan, f), full_ref)
    announce("fmm face marking near_order=%d rel-L2 near %.3e total %.3e" % (near_order, e_near, e))
    assert e_near <= TOL and e <= TOL


@pytest.mark.parametrize("q,near_order,nearfield", [(4, 0, bcv.NEAR_QUADRATURE), (6, 1, bcv.NEAR_ASSEMBLED),
                                                    (8, 1, bcv.NEAR_ASSEMBLED)])
def test_neighbour_marking_fmm_matches_O2(q, near_order, nearfield):
    """h = 1/32 with the neighbour marking (29,184 leaves, levels 4 and 5), sampled targets."""
    L = 5
    m, lv = mesh(L, 1)
    f = synth.leaf_density(lv, seed=2)
    announce("fmm neighbour marking L=%d q=%d near_order=%d n=%d" % (L, q, near_order, len(lv)))
    plan = bcv.plan_interactions(bcv.build_bc_tree(L, 1), q=q, nearfield=nearfield, near_order=near_order)
    info = plan.info
    assert info["n_leaves"] == len(lv)
    tg = np.unique(np.concatenate([np.arange(0, len(lv), 97), [len(lv) - 1]]))
    F = fmm.FMM(m, q, near_order=near_order)
    u_near = gpu_apply(plan, f, bcv.PART_NEAR)[tg]
    u = gpu_apply(plan, f)[tg]
    e_near = rel_l2(lv[tg], u_near, F.near_field(f, tg))
    e = rel_l2(lv[tg], u, F.apply_sampled(f, tg))
    announce("fmm neighbour marking q=%d near_order=%d rel-L2 near %.3e total %.3e" % (q, near_order, e_near, e))
    assert e_near <= TOL and e <= TOL


def test_neighbour_marking_mixed_precision():
    L, q = 5, 6
    m, lv = mesh(L, 1)
    f = synth.leaf_density(lv, seed=3)
    t = bcv.build_bc_tree(L, 1)
    announce("mixed vs fp64, neighbour marking, level rule, L=%d q=%d" % (L, q))
    a = gpu_apply(bcv.plan_interactions(t, q=q, nearfield=bcv.NEAR_ASSEMBLED, near_order=1), f)
    b = gpu_apply(bcv.plan_interactions(t, q=q, nearfield=bcv.NEAR_ASSEMBLED, near_order=1,
                                        precision=bcv.MIXED_F32), f)
    e = rel_l2(lv, b, a)
    announce("mixed vs fp64 rel-L2 %.3e" % e)
    assert e <= MIXED_TOL


def test_neighbour_marking_full_size_sampled():
    """h = 1/128 (L = 7, 767,488 leaves) with the neighbour marking and the level rule, q = 6: the
    configuration bench.py times for this extension, against O2 at 100 sampled leaves."""
    L, q = 7, 6
    announce("full size neighbour marking L=7: oracle mesh")
    m, lv = mesh(L, 1)
    f = synth.leaf_density(lv, seed=0)
    announce("full size neighbour marking L=7: plan")
    plan = bcv.plan_interactions(bcv.build_bc_tree(L, 1), q=q, nearfield=bcv.NEAR_ASSEMBLED, near_order=1)
    u = gpu_apply(plan, f)
    tg = np.random.default_rng(0).choice(len(lv), 100, replace=False)
    announce("full size neighbour marking L=7: oracle at 100 leaves")
    ref = fmm.FMM(m, q, near_order=1).apply_sampled(f, tg)
    e = np.max(np.abs(u[tg] - ref) / np.abs(ref))
    announce("full size neighbour marking max rel %.3e" % e)
    assert e <= TOL


def test_level_rule_batched_forest():
    """A forest of meshes with both markings: each mesh's leaves match its own plan."""
    Ls, marks = [4, 3, 5], [0, 1, 1]
    t = bcv.build_bc_forest(Ls, marks)
    mesh_of = t.leaf_mesh()
    lv = t.leaves().astype(np.int64)
    f = np.empty(len(lv))
    for mi in range(len(Ls)):  # each mesh's density on its own unit cube
        loc = lv[mesh_of == mi].copy()
        loc[:, 1] -= (4 * mi) << loc[:, 0]
        f[mesh_of == mi] = synth.leaf_density(loc, seed=5 + mi)
    announce("forest near_order=1 Ls=%s marks=%s" % (Ls, marks))
    u = gpu_apply(bcv.plan_interactions(t, q=6, nearfield=bcv.NEAR_ASSEMBLED, near_order=1), f)
    for mi, (L, mk) in enumerate(zip(Ls, marks)):
        sel = mesh_of == mi
        one = gpu_apply(bcv.plan_interactions(bcv.build_bc_tree(L, mk), q=6, nearfield=bcv.NEAR_ASSEMBLED,
                                              near_order=1), f[sel])
        assert rel_l2(lv[sel], u[sel], one) <= 1e-13
