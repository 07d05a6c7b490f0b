"""Mapped (cube-to-ball) meshes on the GPU against the mapped-mesh oracle (oracle/mapped.py).

* the singular rule for touching curved cells on explicit pairs against the oracle's;
* direct mode (every pair near) against O1 on the ball, FP64: the mapped point rule and the singular
  rule for touching curved cells, entry by entry through the sums;
* the FMM against O2 on the ball (q = 4, 6, 8), FP64, and the mixed path;
* a larger ball mesh at sampled leaves;
* f = 1: the cell integrals of the uniform ball's Newton potential R^2/2 - r^2/6;
* a forest mixing unit cubes and balls (the batched workload's kind) against O2 of each mesh.
"""

import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))

import synth  # noqa: E402
from gpu_util import gpu_apply, rel_l2  # noqa: E402

import paper_2112_00864_amd as bcv  # noqa: E402

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def ball_tree(L):
    return bcv.build_bc_tree(L, geometry=bcv.GEOM_BALL)


def density(tree, seed=0):
    return synth.leaf_density(tree.leaves().astype(np.int64), seed=seed)


@pytest.fixture(scope="module")
def ball3():
    from oracle import mapped
    from oracle.mesh import BCMesh

    mm = mapped.MappedMesh(BCMesh(3), "ball")
    return mm


def test_rule_on_explicit_pairs_matches_oracle():
    """The planner's singular rule on explicit pairs (bcv_mapped_pair_entries) against the oracle's
    rule (the same published method at the same orders, written separately), 6 pairs of each of the
    7 touching classes of the h = 1/16 ball mesh; and its argument checks."""
    from oracle import mapped
    from oracle.direct import leaf_geometry, touching_class_index
    from oracle.mesh import BCMesh

    mm = mapped.MappedMesh(BCMesh(4), "ball")
    lo_int, size, _, _ = leaf_geometry(mm.leaves, 4)
    n = len(mm.leaves)
    rng = np.random.default_rng(3)
    ti, si = rng.integers(0, n, 400000), rng.integers(0, n, 400000)
    cls = touching_class_index(lo_int[ti], size[ti], lo_int[si], size[si])
    sel = np.concatenate([rng.choice(np.nonzero(cls == c)[0], 6, replace=False) for c in range(7)])
    gt = np.concatenate([mm.lo[ti[sel]], mm.a[ti[sel], None]], axis=1)
    gs = np.concatenate([mm.lo[si[sel]], mm.a[si[sel], None]], axis=1)
    ours = bcv.mapped_pair_entries(gt, gs)
    ref = mapped.touch_entries(mm, ti[sel], si[sel])
    err = float(np.max(np.abs(ours / ref - 1)))
    announce("explicit pairs: library rule vs oracle rule, 42 pairs of 7 classes: max rel %.2e" % err)
    assert err <= 1e-12
    for bad_s in ([0.5, 0.5, 0.5, 0.0625], [0.0, 0.0, 0.0, 0.3], [0.03, 0.0, 0.0, 0.0625]):  # apart, side, corner
        with pytest.raises(bcv.BCVError) as e:
            bcv.mapped_pair_entries([[0.0, 0.0, 0.0, 0.0625]], [bad_s])
        assert e.value.status == bcv.bcv.EINVAL


@pytest.mark.parametrize("L", [2, 3])
def test_direct_mode_matches_O1(L, ball3):
    from oracle import mapped
    from oracle.mesh import BCMesh

    tree = ball_tree(L)
    f = density(tree)
    announce("ball L=%d direct mode, FP64, %d leaves" % (L, len(f)))
    u = gpu_apply(bcv.plan_interactions(tree, q=6, direct=True, nearfield=bcv.NEAR_ASSEMBLED), f)
    ref = mapped.apply_direct(ball3 if L == 3 else mapped.MappedMesh(BCMesh(L), "ball"), f)
    err = float(np.max(np.abs(u - ref) / np.abs(ref)))
    announce("max rel %.3e" % err)
    assert err <= 1e-12


@pytest.mark.parametrize("q", [4, 6, 8])
def test_fmm_matches_O2(q, ball3):
    from oracle import mapped

    tree = ball_tree(3)
    f = density(tree, seed=1)
    announce("ball L=3 FMM q=%d FP64" % q)
    u = gpu_apply(bcv.plan_interactions(tree, q=q, nearfield=bcv.NEAR_ASSEMBLED), f)
    if q < 8:
        ref = mapped.MappedFMM(ball3, q).apply(f)
        err = float(np.max(np.abs(u - ref) / np.abs(ref)))
    else:  # q = 8: O2 at sampled leaves (its full form takes minutes)
        sample = np.array([0, 1, 57, 200, 301, len(f) - 1])
        ref = mapped.MappedFMM(ball3, q).apply_sampled(f, sample)
        err = float(np.max(np.abs(u[sample] - ref) / np.abs(ref)))
    announce("max rel %.3e" % err)
    assert err <= 1e-10
    parts = {}
    for name, p in (("near", bcv.PART_NEAR), ("far", bcv.PART_FAR)):
        parts[name] = gpu_apply(bcv.plan_interactions(tree, q=q, nearfield=bcv.NEAR_ASSEMBLED), f, parts=p)
    assert np.max(np.abs(parts["near"] + parts["far"] - u)) <= 1e-13 * np.max(np.abs(u))


@pytest.mark.parametrize("precision", [bcv.FP64, bcv.MIXED_F32])
def test_one_and_two_streams_agree(precision):
    """With two streams the mapped apply runs its near field beside M2M and the ball cells' pair kernel
    beside the lattice tasks; every kernel computes the same values in the same order either way."""
    Ls = [4, 3]
    tree = bcv.build_bc_forest(Ls, geometry=[bcv.GEOM_BALL, bcv.GEOM_BOX])
    lv = tree.leaves().astype(np.int64)
    mesh = tree.leaf_mesh()
    f = np.empty(len(lv))
    for m in range(len(Ls)):
        loc = lv[mesh == m].copy()
        loc[:, 1] -= (4 * m) << loc[:, 0]
        f[mesh == m] = synth.leaf_density(loc, seed=4 + m)
    announce("ball + cube forest, streams 1 vs 2, precision %d" % precision)
    a = gpu_apply(bcv.plan_interactions(tree, q=6, nearfield=bcv.NEAR_ASSEMBLED, precision=precision, streams=1), f)
    b = gpu_apply(bcv.plan_interactions(tree, q=6, nearfield=bcv.NEAR_ASSEMBLED, precision=precision, streams=2), f)
    announce("max abs diff %.3e" % float(np.max(np.abs(a - b))))
    assert np.array_equal(a, b)


def test_mixed_precision_against_O2(ball3):
    from oracle import mapped

    tree = ball_tree(3)
    f = density(tree, seed=2)
    announce("ball L=3 FMM q=6 mixed")
    u = gpu_apply(bcv.plan_interactions(tree, q=6, nearfield=bcv.NEAR_ASSEMBLED, precision=bcv.MIXED_F32), f)
    ref = mapped.MappedFMM(ball3, 6).apply(f)
    err = rel_l2(tree.leaves(), u, ref)
    announce("rel-L2 %.3e, max rel %.3e" % (err, float(np.max(np.abs(u - ref) / np.abs(ref)))))
    assert err <= 1e-6


def test_larger_ball_sampled():
    from oracle import mapped
    from oracle.mesh import BCMesh

    L = 5
    tree = ball_tree(L)
    f = density(tree, seed=3)
    n = len(f)
    sample = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(7).choice(n, 8, replace=False)]))
    announce("ball L=%d, %d leaves, O2 at %d leaves" % (L, n, len(sample)))
    u64 = gpu_apply(bcv.plan_interactions(tree, q=6, nearfield=bcv.NEAR_ASSEMBLED), f)
    u32 = gpu_apply(bcv.plan_interactions(tree, q=6, nearfield=bcv.NEAR_ASSEMBLED, precision=bcv.MIXED_F32), f)
    ref = mapped.MappedFMM(mapped.MappedMesh(BCMesh(L), "ball"), 6).apply_sampled(f, sample)
    e64 = float(np.max(np.abs(u64[sample] - ref) / np.abs(ref)))
    e32 = float(np.max(np.abs(u32[sample] - ref) / np.abs(ref)))
    announce("FP64 max rel %.3e; mixed max rel %.3e; mixed vs FP64 rel-L2 over all leaves %.3e"
             % (e64, e32, rel_l2(tree.leaves(), u32, u64)))
    assert e64 <= 1e-10 and rel_l2(tree.leaves(), u32, u64) <= 1e-6


def test_uniform_ball_newton_potential():
    """f = 1 on the ball mesh: u_w against the cell integral of R^2/2 - r^2/6 (10^3 Gauss points
    per cell through the map); the difference is the 2x2x2 rule's discretisation error."""
    from oracle import mapped
    from oracle.mesh import BCMesh

    L = 4
    tree = ball_tree(L)
    n = tree.num_leaves()
    u = gpu_apply(bcv.plan_interactions(tree, q=8, nearfield=bcv.NEAR_ASSEMBLED), np.ones(n))
    mm = mapped.MappedMesh(BCMesh(L), "ball")
    t, w = np.polynomial.legendre.leggauss(10)
    t, w = 0.5 * (t + 1), 0.5 * w
    X = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).ravel()
    pts, J = mapped.map_points("ball", mm.lo[:, None, :] + mm.a[:, None, None] * X[None])
    ex = np.sum(W[None] * J * mapped.ball_potential(pts), axis=1) * mm.a ** 3
    err_max = float(np.max(np.abs(u / ex - 1)))
    err_l2 = rel_l2(tree.leaves(), u, ex)
    announce("uniform ball L=%d: max rel %.3e, rel-L2 %.3e" % (L, err_max, err_l2))
    assert err_max <= 1e-3 and err_l2 <= 2e-4


def test_forest_of_cubes_and_balls_against_O2():
    """A forest alternating unit cubes and balls (levels 3..5): every mesh against O2 of its own kind
    at sampled leaves, FP64 and mixed."""
    from oracle import fmm, mapped
    from oracle.mesh import BCMesh

    Ls = [3, 3, 4, 4, 5, 5]
    geoms = [bcv.GEOM_BOX, bcv.GEOM_BALL] * 3
    forest = bcv.build_bc_forest(Ls, geometry=geoms)
    lv = forest.leaves().astype(np.int64)
    mesh = forest.leaf_mesh()
    f = np.empty(len(lv))
    for m in range(len(Ls)):
        sel = mesh == m
        loc = lv[sel].copy()
        loc[:, 1] -= (4 * m) << loc[:, 0]
        f[sel] = synth.leaf_density(loc, seed=m)
    announce("forest of %d meshes (cubes and balls), %d leaves" % (len(Ls), len(lv)))
    u64 = gpu_apply(bcv.plan_interactions(forest, q=6, nearfield=bcv.NEAR_ASSEMBLED), f)
    u32 = gpu_apply(bcv.plan_interactions(forest, q=6, nearfield=bcv.NEAR_ASSEMBLED, precision=bcv.MIXED_F32), f)
    rng = np.random.default_rng(11)
    worst64 = worst32 = 0.0
    for m, L in enumerate(Ls):
        sel = np.nonzero(mesh == m)[0]
        n = len(sel)
        sample = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 5, replace=False)]))
        if geoms[m] == bcv.GEOM_BALL:
            ref = mapped.MappedFMM(mapped.MappedMesh(BCMesh(L), "ball"), 6).apply_sampled(f[sel], sample)
        else:
            ref = fmm.FMM(BCMesh(L), 6).apply_sampled(f[sel], sample)
        worst64 = max(worst64, float(np.max(np.abs(u64[sel][sample] - ref) / np.abs(ref))))
        worst32 = max(worst32, float(np.max(np.abs(u32[sel][sample] - ref) / np.abs(ref))))
    announce("forest vs O2: FP64 max rel %.3e, mixed max rel %.3e" % (worst64, worst32))
    assert worst64 <= 1e-10 and worst32 <= 1e-5


def test_graph_and_batched_calls_on_a_forest_with_balls():
    """A cube/ball forest: every replay of the captured apply equals the eager apply bit for bit (with
    other eager work between replays), and bcv_vtv_apply_batched over separate ball and cube plans
    equals their applies one by one."""
    import torch

    Ls = [3, 4, 3, 4]
    geoms = [bcv.GEOM_BALL, bcv.GEOM_BOX, bcv.GEOM_BOX, bcv.GEOM_BALL]
    forest = bcv.build_bc_forest(Ls, geometry=geoms)
    f = synth.leaf_density(forest.leaves().astype(np.int64), seed=6)
    plan = bcv.plan_interactions(forest, q=6, nearfield=bcv.NEAR_ASSEMBLED, precision=bcv.MIXED_F32)
    fd = torch.tensor(f, device="cuda:0")
    ud = torch.full_like(fd, float("nan"))
    ref = torch.empty_like(fd)
    bcv.vtv_apply(plan, fd, ref)
    torch.cuda.synchronize()
    graph = bcv.vtv_graph_create(plan, fd, ud)
    other = bcv.plan_interactions(ball_tree(2), q=4, nearfield=bcv.NEAR_ASSEMBLED)
    fo = torch.ones(other.n_leaves, dtype=torch.float64, device="cuda:0")
    uo = torch.empty_like(fo)
    for rep in range(3):
        ud.fill_(float("nan"))
        graph.launch()
        torch.cuda.synchronize()
        diff = float(torch.max(torch.abs(ud - ref)).item())
        announce("cube/ball forest, replay %d: max |graph - eager| %.3e" % (rep, diff))
        assert diff == 0.0
        bcv.vtv_apply(other, fo, uo)
        torch.cuda.synchronize()
    trees = [ball_tree(3), bcv.build_bc_tree(3), ball_tree(4)]
    plans = [bcv.plan_interactions(t, q=6, nearfield=bcv.NEAR_ASSEMBLED) for t in trees]
    fs = [torch.tensor(density(t, seed=k), device="cuda:0") for k, t in enumerate(trees)]
    us = [torch.full_like(x, float("nan")) for x in fs]
    bcv.vtv_apply_batched(plans, fs, us)
    torch.cuda.synchronize()
    for p_, f_, u_ in zip(plans, fs, us):
        one = torch.empty_like(f_)
        bcv.vtv_apply(p_, f_, one)
        torch.cuda.synchronize()
        assert float(torch.max(torch.abs(u_ - one)).item()) == 0.0


def test_scaled_ball_and_neighbour_marking():
    """The ball inscribed in the cube lo + s [0,1]^3 gives s^5 times the unit ball's potentials; a ball
    mesh refined by the neighbour marking rule against O2 of the same mesh."""
    from oracle import mapped
    from oracle.mesh import BCMesh

    t1 = ball_tree(3)
    f = density(t1, seed=8)
    u1 = gpu_apply(bcv.plan_interactions(t1, q=6, nearfield=bcv.NEAR_ASSEMBLED), f)
    s, lo = 0.37, (-1.3, 0.25, 2.0)
    ts = bcv.build_bc_tree(3, lo=lo, hi=tuple(x + s for x in lo), geometry=bcv.GEOM_BALL)
    us = gpu_apply(bcv.plan_interactions(ts, q=6, nearfield=bcv.NEAR_ASSEMBLED), f)
    err = float(np.max(np.abs(us - s ** 5 * u1) / np.abs(s ** 5 * u1)))
    announce("ball of side %.2f against s^5 x unit ball: max rel %.2e" % (s, err))
    assert err <= 1e-13
    tm = bcv.build_bc_tree(4, marking=bcv.MARK_NEIGHBOR, geometry=bcv.GEOM_BALL)
    fm = density(tm, seed=9)
    um = gpu_apply(bcv.plan_interactions(tm, q=6, nearfield=bcv.NEAR_ASSEMBLED), fm)
    n = len(fm)
    sample = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(12).choice(n, 6, replace=False)]))
    ref = mapped.MappedFMM(mapped.MappedMesh(BCMesh(4, marking=1), "ball"), 6).apply_sampled(fm, sample)
    em = float(np.max(np.abs(um[sample] - ref) / np.abs(ref)))
    announce("ball h=1/16, neighbour marking (%d leaves) against O2 at %d leaves: max rel %.2e" % (n, len(sample), em))
    assert em <= 1e-10
