"""The C ABI's domain, order and batching options on the GPU.

* A cube of side s at any position: the VtV potential is s^5 times that of the unit cube (the
  operator scales exactly; the library applies the factor at the end, a power of two here, so the
  comparison is exact), checked against O2 times s^5.
* Fixed expansion orders without kernels of their own (0 to 3, 5, 7) run the level-by-level kernels:
  against O2 with the same constant order, bar 1e-10.
* bcv_vtv_apply_batched: three plans of different meshes, one call, equal to three single applies.
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
TOL = 1e-10


def announce(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_scaled_domain():
    L, q, s = 4, 6, 2.0
    m = BCMesh(L)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=3)
    announce("scaled cube side %g, L=%d" % (s, L))
    u1 = gpu_apply(bcv.plan_interactions(bcv.build_bc_tree(L), q=q), f)
    t2 = bcv.build_bc_tree(L, lo=(1.5, -4.0, 0.25), hi=(3.5, -2.0, 2.25))
    u2 = gpu_apply(bcv.plan_interactions(t2, q=q, nearfield=bcv.NEAR_ASSEMBLED), f)
    u3 = gpu_apply(bcv.plan_interactions(t2, q=q, precision=bcv.MIXED_F32), f)
    ref = fmm.FMM(m, q).apply(f) * s ** 5
    e = rel_l2(lv, u2, ref)
    announce("scaled cube: rel-L2 vs O2 * s^5 %.3e, mixed %.3e" % (e, rel_l2(lv, u3, ref)))
    assert np.array_equal(u2, u1 * s ** 5) or np.max(np.abs(u2 - u1 * s ** 5) / np.abs(u2)) < 1e-14
    assert e <= TOL and rel_l2(lv, u3, ref) <= 1e-6
    with pytest.raises(bcv.BCVError) as ex:
        bcv.plan_interactions(t2, q=q, boundary=True)
    assert ex.value.status == bcv.ENOTSUP


@pytest.mark.parametrize("q", [0, 1, 2, 3, 5, 7])
def test_other_fixed_orders(q):
    L = 4
    m = BCMesh(L)
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=4)
    announce("fixed order q=%d through the per-level kernels, L=%d" % (q, L))
    plan = bcv.plan_interactions(bcv.build_bc_tree(L), q=q)
    u = gpu_apply(plan, f)
    ref = fmm.FMM(m, q).apply(f)
    e = rel_l2(lv, u, ref)
    announce("q=%d rel-L2 vs O2 %.3e" % (q, e))
    assert e <= TOL


def test_batched_apply_equals_single_applies():
    import torch

    Ls = [3, 4, 5]
    plans, fs, us, refs = [], [], [], []
    for k, L in enumerate(Ls):
        t = bcv.build_bc_tree(L)
        lv = t.leaves()
        f = synth.leaf_density(lv, seed=10 + k)
        plan = bcv.plan_interactions(t, q=6, precision=bcv.MIXED_F32 if k == 1 else bcv.FP64)
        plans.append(plan)
        fs.append(torch.tensor(f, device="cuda:0"))
        us.append(torch.full_like(fs[-1], float("nan")))
        refs.append(gpu_apply(plan, f))
    announce("batched apply of %d plans" % len(plans))
    bcv.vtv_apply_batched(plans, fs, us)
    torch.cuda.synchronize()
    for u, r in zip(us, refs):
        assert np.array_equal(u.cpu().numpy(), r)
