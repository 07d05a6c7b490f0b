"""Degree-p leaf bases (opts.basis_degree = 1, p_l = L - l) on the GPU against the oracle
(oracle.basis): direct mode against O1, the FMM against O2 (all coefficients, q = 4, 6, 8), sampled
leaves of every degree at h = 1/32 and at the bench's h = 1/128 (FP64 bar 1e-10), the near and far
parts, linearity in f, the captured graph, and the O(h) rate of the projected potential of f = 1
against its closed form up to h = 1/64."""

import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))

import paper_2112_00864_amd as bcv  # noqa: E402

from oracle import basis  # noqa: E402
from oracle.mesh import BCMesh  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10


def announce(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def layout(lf):
    """Library positions of the oracle's leaf-major coefficients: alpha = 0 of every leaf first (leaf
    order), then the higher coefficients leaf by leaf (bcv_plan_opts.basis_degree)."""
    nl = len(lf.lv)
    nbs = np.diff(lf.off)
    hi = np.concatenate([[0], np.cumsum(nbs - 1)])
    pos = np.empty(lf.off[-1], dtype=np.int64)
    pos[lf.off[:-1]] = np.arange(nl)
    for w in range(nl):
        pos[lf.off[w] + 1 : lf.off[w + 1]] = nl + hi[w] + np.arange(nbs[w] - 1)
    return pos


def gpu_apply(plan, F, pos, parts=None):
    import torch

    f = np.empty_like(F)
    f[pos] = F
    fd = torch.tensor(f, device="cuda:0")
    ud = torch.full_like(fd, float("nan"))
    if parts is None:
        bcv.vtv_apply(plan, fd, ud)
    else:
        bcv.vtv_apply_parts(plan, fd, ud, parts)
    torch.cuda.synchronize()
    return ud.cpu().numpy()[pos]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_layout_and_sizes():
    m = BCMesh(4)
    lf = basis.Leaves(m)
    plan = bcv.plan_interactions(bcv.build_bc_tree(4), q=6, basis_degree=1, streams=1)
    assert plan.n_dofs == lf.off[-1] and plan.n_leaves == len(lf.lv)
    assert plan.info["n_basis_vals"] > plan.info["n_near"]


def test_direct_against_O1():
    m = BCMesh(3)
    lf = basis.Leaves(m)
    F = np.random.default_rng(0).standard_normal(lf.off[-1])
    plan = bcv.plan_interactions(bcv.build_bc_tree(3), q=6, direct=True, basis_degree=1, streams=1)
    u = gpu_apply(plan, F, layout(lf))
    ref = basis.apply_direct(m, F)
    announce("basis direct L=3 vs O1: rel-L2 %.3e" % rel(u, ref))
    assert rel(u, ref) <= TOL


@pytest.mark.parametrize("q", [4, 6, 8])
def test_fmm_against_O2(q):
    m = BCMesh(3)
    lf = basis.Leaves(m)
    F = np.random.default_rng(q).standard_normal(lf.off[-1])
    plan = bcv.plan_interactions(bcv.build_bc_tree(3), q=q, basis_degree=1, streams=1)
    pos = layout(lf)
    fm = basis.BasisFMM(m, q)
    u = gpu_apply(plan, F, pos)
    ref = fm.apply_basis(F)
    un = gpu_apply(plan, F, pos, bcv.PART_NEAR)
    near = np.concatenate(fm.near_field_basis(F, range(len(lf.lv))))
    announce("basis FMM L=3 q=%d vs O2: total %.3e, near %.3e" % (q, rel(u, ref), rel(un, near)))
    assert rel(u, ref) <= TOL and rel(un, near) <= TOL


@pytest.mark.parametrize("L", [5, 7])
def test_sampled_leaves_of_every_degree(L):
    m = BCMesh(L)
    lf = basis.Leaves(m)
    F = np.random.default_rng(L).standard_normal(lf.off[-1])
    plan = bcv.plan_interactions(bcv.build_bc_tree(L), q=6, basis_degree=1, streams=1)
    u = gpu_apply(plan, F, layout(lf))
    rng = np.random.default_rng(100 + L)
    targets = [0, len(lf.lv) - 1]
    for p in range(0, int(lf.p.max()) + 1):
        cand = np.nonzero(lf.p == p)[0]
        targets += list(rng.choice(cand, min(2, len(cand)), replace=False))
    targets = np.array(sorted(set(int(t) for t in targets)))
    announce("basis L=%d: O2 at %d leaves (degrees %s)" % (L, len(targets), sorted(set(lf.p[targets].tolist()))))
    ref = basis.BasisFMM(m, 6).apply_basis_sampled(F, targets)
    got = np.concatenate([u[lf.off[t] : lf.off[t + 1]] for t in targets])
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    announce("basis L=%d sampled vs O2: max rel %.3e" % (L, err))
    assert err <= TOL


def test_parts_linearity_and_graph():
    import torch

    m = BCMesh(4)
    lf = basis.Leaves(m)
    pos = layout(lf)
    rng = np.random.default_rng(7)
    F1, F2 = rng.standard_normal(lf.off[-1]), rng.standard_normal(lf.off[-1])
    plan = bcv.plan_interactions(bcv.build_bc_tree(4), q=6, basis_degree=1, streams=1)
    u = gpu_apply(plan, F1, pos)
    un = gpu_apply(plan, F1, pos, bcv.PART_NEAR)
    uf = gpu_apply(plan, F1, pos, bcv.PART_FAR)
    assert np.max(np.abs(un + uf - u)) <= 1e-14 * np.max(np.abs(u))
    u12 = gpu_apply(plan, 2.0 * F1 - 3.0 * F2, pos)
    assert rel(u12, 2.0 * u - 3.0 * gpu_apply(plan, F2, pos)) <= 1e-14
    assert np.all(gpu_apply(plan, np.zeros_like(F1), pos) == 0.0)
    f = np.empty_like(F1)
    f[pos] = F1
    fd = torch.tensor(f, device="cuda:0")
    ud = torch.full_like(fd, float("nan"))
    graph = bcv.vtv_graph_create(plan, fd, ud)
    for rep in range(3):
        ud.fill_(float("nan"))
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(ud.cpu().numpy()[pos], u)


@pytest.mark.parametrize("L, q", [(3, 4), (3, 6), (6, 4)])
def test_level_orders_against_O2(L, q):
    """The paper's experiment setup: p_l = L - l with q_l = q + L - l (Sec. 5), against O2 with the same
    orders (all coefficients at h = 1/8; sampled leaves of every degree at h = 1/64)."""
    m = BCMesh(L)
    lf = basis.Leaves(m)
    F = np.random.default_rng(40 + L + q).standard_normal(lf.off[-1])
    plan = bcv.plan_interactions(bcv.build_bc_tree(L), q=q, q_schedule=1, basis_degree=1, streams=1)
    u = gpu_apply(plan, F, layout(lf))
    fm = basis.BasisFMM(m, q, q_schedule=1)
    if L <= 3:
        ref = fm.apply_basis(F)
        err = rel(u, ref)
    else:
        rng = np.random.default_rng(7)
        targets = [0, len(lf.lv) - 1]
        for p in range(int(lf.p.max()) + 1):
            cand = np.nonzero(lf.p == p)[0]
            targets += list(rng.choice(cand, min(2, len(cand)), replace=False))
        targets = np.array(sorted(set(int(t) for t in targets)))
        ref = fm.apply_basis_sampled(F, targets)
        got = np.concatenate([u[lf.off[t] : lf.off[t + 1]] for t in targets])
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    announce("basis + level orders L=%d q=%d vs O2: %.3e" % (L, q, err))
    assert err <= TOL


def test_option_errors():
    tree = bcv.build_bc_tree(3)
    for kw, code in ((dict(basis_degree=2), bcv.EINVAL), (dict(basis_degree=1, precision=bcv.MIXED_F32), bcv.ENOTSUP),
                     (dict(basis_degree=1, boundary=True), bcv.ENOTSUP)):
        with pytest.raises(bcv.BCVError) as e:
            bcv.plan_interactions(tree, **kw)
        assert e.value.status == code
    forest = bcv.build_bc_forest([3, 3])
    with pytest.raises(bcv.BCVError) as e:
        bcv.plan_interactions(forest, q=6, basis_degree=1)
    assert e.value.status == bcv.ENOTSUP


def _projection_error(L, degree):
    """f = 1 on the unit cube: the L2 error of the projection sum_alpha u_alpha phi^alpha / ||phi^alpha||^2
    of the GPU result against the closed-form potential, relative to its norm (a (p + 3)-point rule
    per axis on each leaf)."""
    import torch

    from closed_forms import box_potential

    tree = bcv.build_bc_tree(L)
    lv = tree.leaves().astype(np.int64)
    nl = len(lv)
    p_of = (L - lv[:, 0]) if degree else np.zeros(nl, dtype=np.int64)
    plan = bcv.plan_interactions(tree, q=6, basis_degree=1 if degree else 0, streams=1)
    f = torch.zeros(plan.n_dofs, dtype=torch.float64, device="cuda:0")
    f[:nl] = 1.0  # degree-0 coefficients: f = 1
    u = torch.empty_like(f)
    bcv.vtv_apply(plan, f, u)
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    nb = (p_of + 1) * (p_of + 2) * (p_of + 3) // 6
    hi = np.concatenate([[0], np.cumsum(nb - 1)])
    e2 = n2 = 0.0
    for p in np.unique(p_of):
        sel = np.nonzero(p_of == p)[0]
        t, w = np.polynomial.legendre.leggauss(int(p) + 3)
        t, w = 0.5 * (t + 1.0), 0.5 * w
        X = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
        W = np.einsum("i,j,k->ijk", w, w, w).ravel()
        P = np.polynomial.legendre.legvander(2.0 * X - 1.0, int(p))
        idx = basis.basis_indices(int(p))
        phi = np.stack([P[:, 0, i] * P[:, 1, j] * P[:, 2, k] * (2 * i + 1) * (2 * j + 1) * (2 * k + 1)
                        for i, j, k in idx], axis=1)  # phi^alpha / ||phi^alpha||^2 times the volume
        a = np.ldexp(1.0, -lv[sel, 0].astype(np.int32))
        coef = np.empty((len(sel), len(idx)))
        coef[:, 0] = u[sel]
        for r in range(1, len(idx)):
            coef[:, r] = u[nl + hi[sel] + r - 1]
        proj = (coef @ phi.T) / (a ** 3)[:, None]
        U = box_potential(lv[sel, 1:4][:, None, :] * a[:, None, None] + a[:, None, None] * X[None])
        e2 += float(np.sum(W[None, :] * (proj - U) ** 2 * (a ** 3)[:, None]))
        n2 += float(np.sum(W[None, :] * U ** 2 * (a ** 3)[:, None]))
    return np.sqrt(e2 / n2)


def test_order_h_rate_at_larger_meshes():
    """The paper's O(h) best approximation with p_l = L - l (Sec. 4) carried on to h = 1/64 on the GPU:
    the error of the projected potential halves with h, while degree 0 on the coarse leaves stalls."""
    errs = {deg: [_projection_error(L, deg) for L in (4, 5, 6)] for deg in (0, 1)}
    announce("f = 1, L2 error of the projection, h = 1/16, 1/32, 1/64: p_l = L - l %s; degree 0 %s"
             % (["%.3e" % e for e in errs[1]], ["%.3e" % e for e in errs[0]]))
    r1 = [errs[1][k + 1] / errs[1][k] for k in range(2)]
    r0 = [errs[0][k + 1] / errs[0][k] for k in range(2)]
    assert max(r1) <= 0.55 and min(r0) >= 0.7 and errs[1][2] < 0.5 * errs[0][2]
