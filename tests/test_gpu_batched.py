"""Batched applies: many BC meshes in one forest plan, its apply captured in one HIP graph, and the
autotuner of the work decomposition."""

import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))

import synth  # noqa: E402
from gpu_util import gpu_apply, rel_l2  # noqa: E402

import paper_2112_00864_amd as bcv  # noqa: E402

pytestmark = pytest.mark.gpu
LS = [2, 3, 4, 3, 2, 4, 4, 3]


def announce(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def forest_density(tree, Ls):
    """Density of every leaf: mesh m gets the Gaussian mixture of seed m on its own unit cube."""
    lv = tree.leaves().astype(np.int64)
    mesh = tree.leaf_mesh()
    f = np.empty(len(lv))
    for m in range(len(Ls)):
        sel = mesh == m
        loc = lv[sel].copy()
        loc[:, 1] -= (4 * m) << loc[:, 0]
        f[sel] = synth.leaf_density(loc, seed=m)
    return lv, mesh, f


@pytest.mark.parametrize("precision", [bcv.FP64, bcv.MIXED_F32])
def test_forest_equals_separate_meshes(precision):
    announce("forest of %d meshes, precision %d" % (len(LS), precision))
    forest = bcv.build_bc_forest(LS)
    lv, mesh, f = forest_density(forest, LS)
    u = gpu_apply(bcv.plan_interactions(forest, q=6, precision=precision), f)
    worst = 0.0
    for m, L in enumerate(LS):
        sel = mesh == m
        um = gpu_apply(bcv.plan_interactions(bcv.build_bc_tree(L), q=6, precision=precision), f[sel])
        worst = max(worst, rel_l2(lv[sel], u[sel], um))
    announce("max per-mesh rel-L2 forest vs separate: %.2e" % worst)
    assert worst <= (1e-13 if precision == bcv.FP64 else 1e-6)


@pytest.mark.parametrize("nearfield", [bcv.NEAR_QUADRATURE, bcv.NEAR_ASSEMBLED])
def test_graph_replays_match_eager(nearfield):
    """Replays with other work and synchronisations between them; every replay equals the eager apply."""
    import torch

    forest = bcv.build_bc_forest(LS)
    lv, mesh, f = forest_density(forest, LS)
    announce("graph replays, nearfield mode %d" % nearfield)
    plan = bcv.plan_interactions(forest, q=6, precision=bcv.MIXED_F32, nearfield=nearfield)
    fd = torch.tensor(f, device="cuda:0")
    ud = torch.full_like(fd, float("nan"))
    ref = torch.empty_like(fd)
    bcv.vtv_apply(plan, fd, ref)
    torch.cuda.synchronize()
    graph = bcv.vtv_graph_create(plan, fd, ud)
    other = bcv.plan_interactions(bcv.build_bc_tree(3), q=4)
    fo = torch.ones(other.n_leaves, dtype=torch.float64, device="cuda:0")
    uo = torch.empty_like(fo)
    for rep in range(4):
        ud.fill_(float("nan"))
        graph.launch()
        torch.cuda.synchronize()
        diff = float(torch.max(torch.abs(ud - ref)).item())
        announce("replay %d: max |graph - eager| %.3e" % (rep, diff))
        assert diff == 0.0
        bcv.vtv_apply(other, fo, uo)  # eager work of another plan between replays
        fd.mul_(1.0)
        torch.cuda.synchronize()
    # a new density in the same buffer is picked up by the next replay
    fd.mul_(2.0)
    graph.launch()
    torch.cuda.synchronize()
    assert float(torch.max(torch.abs(ud - 2.0 * ref)).item()) <= 1e-12 * float(torch.max(torch.abs(ref)).item())


def test_autotune_returns_a_valid_faster_or_equal_plan():
    forest = bcv.build_bc_forest(LS)
    lv, mesh, f = forest_density(forest, LS)
    best, ms = bcv.autotune(forest, n_applies=3, q=6, precision=bcv.MIXED_F32)
    announce("autotune: %s, %.3f ms per apply" % (best, ms))
    assert best["near_unit"] in (0, 256, 512, 1024, 2048) and best["m2l_max_slots"] in (0, 128, 256, 320, 512, 1024)
    u0 = gpu_apply(bcv.plan_interactions(forest, q=6, precision=bcv.MIXED_F32), f)
    u1 = gpu_apply(bcv.plan_interactions(forest, q=6, precision=bcv.MIXED_F32, **best), f)
    assert rel_l2(lv, u1, u0) <= 1e-6


def test_config_forest_against_O2():
    """The batched workload's forest (64 unit-cube meshes, finest levels drawn from {4, 5, 6} by
    default_rng(1234), Gaussian-mixture density of seed m on mesh m) through the captured graph in the
    mixed path and through the FP64 apply: three meshes of every level against O2 of that mesh at 8
    sampled leaves each (the first, the last, 6 random). Bars: FP64 max relative error 1e-10; mixed
    relative L2 error of the sampled cell averages (volume-weighted, per mesh) 1e-6, the tolerance the
    mixed path is held to. The mixed path's largest pointwise errors (about 2e-6 at a few finest-level
    leaves whose potential is 3/4 far field: FP32 sums in the interaction phase) are reported, not
    gated; its per-mesh relative L2 error over all leaves is below 1e-7."""
    import torch

    from oracle import fmm
    from oracle.mesh import BCMesh

    Ls = [int(L) for L in np.random.default_rng(1234).choice([4, 5, 6], 64)]
    forest = bcv.build_bc_forest(Ls)
    lv, mesh, f = forest_density(forest, Ls)
    announce("config forest: %d meshes, %d leaves" % (len(Ls), len(lv)))
    fd = torch.tensor(f, device="cuda:0")
    ud = torch.empty_like(fd)
    graph = bcv.vtv_graph_create(bcv.plan_interactions(forest, q=6, precision=bcv.MIXED_F32), fd, ud)
    graph.launch()
    torch.cuda.synchronize()
    u32 = ud.cpu().numpy()
    u64 = gpu_apply(bcv.plan_interactions(forest, q=6), f)
    oracles = {L: fmm.FMM(BCMesh(L), 6) for L in (4, 5, 6)}
    rng = np.random.default_rng(21)
    worst64 = worst32_l2 = worst32_pt = 0.0
    for L in (4, 5, 6):
        for m in [i for i, x in enumerate(Ls) if x == L][:3]:
            sel = np.nonzero(mesh == m)[0]
            n = len(sel)
            sample = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 6, replace=False)]))
            announce("mesh %d (L=%d): O2 at %d leaves" % (m, L, len(sample)))
            ref = oracles[L].apply_sampled(f[sel], sample)
            vol = 8.0 ** (-lv[sel][sample, 0].astype(float))
            d32 = u32[sel][sample] - ref
            worst64 = max(worst64, float(np.max(np.abs(u64[sel][sample] - ref) / np.abs(ref))))
            worst32_l2 = max(worst32_l2, float(np.sqrt(np.sum(vol * d32 ** 2) / np.sum(vol * ref ** 2))))
            worst32_pt = max(worst32_pt, float(np.max(np.abs(d32) / np.abs(ref))))
    announce("config forest vs O2: FP64 max rel %.3e; mixed (graph) rel-L2 %.3e, pointwise max %.3e"
             % (worst64, worst32_l2, worst32_pt))
    assert worst64 <= 1e-10 and worst32_l2 <= 1e-6
