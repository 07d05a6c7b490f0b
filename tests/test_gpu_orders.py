"""Expansion orders q = 4, 6, 8 on the h = 1/256 unit-cube BC mesh (L = 8, 896,512 leaves).

For each order: the mixed-precision apply (FP32 interaction phase and far near field, FP64
singular pairs and accumulation) against the FP64 apply on the same plan geometry (bar: relative
L2 of cell averages <= 1e-6), and the FP64 apply against the direct Galerkin sum O1 (every leaf
pair, exact touching integrals, 2x2x2 point rule otherwise) at sampled target leaves: that is
the truncation error of the far field, which must fall with q.
"""

import sys

import numpy as np
import pytest

sys.path.insert(0, __import__("os").path.dirname(__file__))

import synth  # noqa: E402
from gpu_util import gpu_apply, rel_l2  # noqa: E402
from oracle import direct  # noqa: E402
from oracle.mesh import BCMesh  # noqa: E402

import paper_2112_00864_amd as bcv  # noqa: E402

pytestmark = pytest.mark.gpu

L = 8
N_SAMPLE = 12
MIXED_TOL = 1e-6


def announce(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    leaves = BCMesh(L).leaf_array()
    tree = bcv.build_bc_tree(L)
    assert np.array_equal(tree.leaves().astype(np.int64), leaves)
    f = synth.leaf_density(leaves, seed=0)
    sample = np.sort(np.random.default_rng(5).choice(len(leaves), N_SAMPLE, replace=False))
    announce("O1 direct sum at %d sampled leaves of %d" % (N_SAMPLE, len(leaves)))
    ref = direct.apply(leaves, L, f, targets=sample)
    return tree, leaves, f, sample, ref


def test_orders_h256(setup):
    tree, leaves, f, sample, ref = setup
    trunc = {}
    for q in (4, 6, 8):
        announce("h=1/256 q=%d FP64 plan" % q)
        u64 = gpu_apply(bcv.plan_interactions(tree, q=q), f)
        announce("h=1/256 q=%d mixed plan" % q)
        u32 = gpu_apply(bcv.plan_interactions(tree, q=q, precision=bcv.MIXED_F32), f)
        e_mixed = rel_l2(leaves, u32, u64)
        trunc[q] = float(np.max(np.abs(u64[sample] - ref) / np.abs(ref)))
        announce("h=1/256 q=%d: mixed vs FP64 rel-L2 %.3e; FP64 vs O1 at %d leaves: max rel %.3e"
                 % (q, e_mixed, N_SAMPLE, trunc[q]))
        assert np.all(np.isfinite(u64)) and np.all(np.isfinite(u32))
        assert e_mixed <= MIXED_TOL
    assert trunc[8] < trunc[6] < trunc[4] < 1e-4
