"""The interaction phase on the matrix cores (BCV_MIXED_SPLIT16: FP16 hi/lo operands, three products,
FP32 accumulation) against the oracle and against the other paths.

Bars: relative L2 of cell averages <= 1e-6 against O2 (the mixed paths' gate), near part, far part
and total; the far part (the only part the matrix cores touch) against the FP32 lane-shift path.
The FP16 rows are scaled by max |f|: a density scaled by 2^-40 or 2^40 gives the potential scaled
by exactly that power (the scale is a power of two), f = 0 gives 0.
"""

import sys

import numpy as np
import pytest

sys.path.insert(0, __import__("os").path.dirname(__file__))

import synth  # noqa: E402
from gpu_util import gpu_apply, rel_l2  # noqa: E402
from oracle import fmm  # noqa: E402
from oracle.mesh import BCMesh  # noqa: E402

import paper_2112_00864_amd as bcv  # noqa: E402

pytestmark = pytest.mark.gpu
MIXED_TOL = 1e-6


def announce(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("L,nf", [(3, bcv.NEAR_QUADRATURE), (4, bcv.NEAR_QUADRATURE), (4, bcv.NEAR_ASSEMBLED),
                                  (5, bcv.NEAR_ASSEMBLED)])
def test_split16_against_O2(L, nf):
    m = BCMesh(L)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=1)
    announce("split16 plan L=%d nearfield %d" % (L, nf))
    plan = bcv.plan_interactions(bcv.build_bc_tree(L), q=6, precision=bcv.MIXED_SPLIT16, nearfield=nf)
    F = fmm.FMM(m, 6)
    near_ref = F.near_field(f, np.arange(len(lv)))
    ref = F.apply(f)
    e_near = rel_l2(lv, gpu_apply(plan, f, bcv.PART_NEAR), near_ref)
    u_far = gpu_apply(plan, f, bcv.PART_FAR)
    e_far = rel_l2(lv, u_far, ref - near_ref)
    u = gpu_apply(plan, f)
    e = rel_l2(lv, u, ref)
    announce("split16 L=%d rel-L2 vs O2: near %.3e far %.3e (of the far part) total %.3e" % (L, e_near, e_far, e))
    assert e_near <= MIXED_TOL and e_far <= MIXED_TOL and e <= MIXED_TOL


def test_split16_far_part_against_fp32_and_fp64_full_size():
    """h = 1/128: the far part against the FP32 lane-shift path and the FP64 path, all leaves."""
    L = 7
    lv = BCMesh(L).leaf_array()
    f = synth.leaf_density(lv, seed=0)
    t = bcv.build_bc_tree(L)
    announce("split16 full size L=7")
    far16 = gpu_apply(bcv.plan_interactions(t, q=6, precision=bcv.MIXED_SPLIT16), f, bcv.PART_FAR)
    far32 = gpu_apply(bcv.plan_interactions(t, q=6, precision=bcv.MIXED_F32), f, bcv.PART_FAR)
    far64 = gpu_apply(bcv.plan_interactions(t, q=6), f, bcv.PART_FAR)
    e16, e32 = rel_l2(lv, far16, far64), rel_l2(lv, far32, far64)
    announce("far part vs FP64, L=7: split16 %.3e, FP32 %.3e" % (e16, e32))
    assert e16 <= MIXED_TOL and e32 <= MIXED_TOL


def test_split16_density_scale_and_zero():
    L = 4
    lv = BCMesh(L).leaf_array()
    f = synth.leaf_density(lv, seed=5)
    plan = bcv.plan_interactions(bcv.build_bc_tree(L), q=6, precision=bcv.MIXED_SPLIT16)
    announce("split16 density scaling L=4")
    u = gpu_apply(plan, f)
    for k in (-40, 40):
        us = gpu_apply(plan, np.ldexp(f, k))
        assert np.array_equal(np.ldexp(us, -k), u), k
    assert np.all(gpu_apply(plan, np.zeros(len(lv))) == 0.0)


def test_split16_work_decomposition():
    """Interaction pieces of 16 slots (many split tasks, every piece starting with a gathering slot)
    and one piece per task give the same operator to the mixed gate."""
    L = 5
    m = BCMesh(L)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=3)
    ref = fmm.FMM(m, 6).apply(f)
    t = bcv.build_bc_tree(L)
    for slots in (16, 40, 65536):
        announce("split16 m2l_max_slots=%d" % slots)
        u = gpu_apply(bcv.plan_interactions(t, q=6, precision=bcv.MIXED_SPLIT16, m2l_max_slots=slots), f)
        e = rel_l2(lv, u, ref)
        announce("  rel-L2 vs O2 %.3e" % e)
        assert e <= MIXED_TOL


def test_split16_options():
    t = bcv.build_bc_tree(3)
    for kw in (dict(q=4), dict(q=8), dict(q=4, q_schedule=1)):
        with pytest.raises(bcv.BCVError) as e:
            bcv.plan_interactions(t, precision=bcv.MIXED_SPLIT16, **kw)
        assert e.value.status == bcv.ENOTSUP
