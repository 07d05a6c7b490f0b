"""C-ABI library: loads, exports every declared entry point, host-side tree and error paths (no GPU)."""

import os
import re

import numpy as np
import pytest

import paper_2112_00864_amd as bcv
from oracle.mesh import BCMesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bcv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bcv_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = bcv.lib()
    names = declared_functions()
    assert "bcv_vtv_apply" in names and "bcv_plan_interactions" in names and "bcv_build_bc_tree" in names
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("L,marking", [(2, 0), (3, 0), (4, 0), (5, 0), (2, 1), (4, 1), (5, 1), (6, 1)])
def test_tree_matches_oracle_mesh(L, marking):
    """The library's tree against the oracle's mesh (which applies the marking rules by their
    definitions: a face on the boundary, or a boundary cell among the neighbours)."""
    t = bcv.build_bc_tree(L, marking)
    assert np.array_equal(t.leaves().astype(np.int64), BCMesh(L, marking).leaf_array())


@pytest.mark.parametrize("L,marking", [(2, 0), (3, 0), (5, 0), (5, 1)])
def test_tree_faces_match_oracle(L, marking):
    from oracle import boundary

    t = bcv.build_bc_tree(L, marking)
    assert np.array_equal(t.faces().astype(np.int64), boundary.boundary_faces(BCMesh(L, marking)))


def test_forest_has_no_faces():
    with pytest.raises(bcv.BCVError) as e:
        bcv.build_bc_forest([3, 4]).faces()
    assert e.value.status == bcv.bcv.ENOTSUP


def test_tree_argument_errors():
    for L in (1, 10):
        with pytest.raises(bcv.BCVError) as e:
            bcv.build_bc_tree(L)
        assert e.value.status == bcv.bcv.EINVAL
    for mk in (-1, 2):
        with pytest.raises(bcv.BCVError) as e:
            bcv.build_bc_tree(4, marking=mk)
        assert e.value.status == bcv.bcv.EINVAL


def test_plan_argument_errors_before_device_use():
    t = bcv.build_bc_tree(3)
    for kw in ({"q": -1}, {"q": 11}, {"eta0": 0.4}, {"near_order": 2}, {"near_order": 1},  # 1 needs the assembled mode
               {"near_order": 1, "nearfield": bcv.NEAR_QUADRATURE}, {"q_schedule": 2}):
        with pytest.raises(bcv.BCVError) as e:
            bcv.plan_interactions(t, **kw)
        assert e.value.status == bcv.bcv.EINVAL


def test_exact_moments_need_the_level_schedule():
    t = bcv.build_bc_tree(3)
    for kw in ({"exact_moments": True}, {"exact_moments": True, "q_schedule": 1, "basis_degree": 1}):
        with pytest.raises(bcv.BCVError) as e:
            bcv.plan_interactions(t, q=4, **kw)
        assert e.value.status == bcv.bcv.ENOTSUP


def test_schedule_is_not_combined_with_the_boundary_structures():
    with pytest.raises(bcv.BCVError) as e:
        bcv.plan_interactions(bcv.build_bc_tree(3), q=4, q_schedule=1, boundary=True)
    assert e.value.status == bcv.bcv.ENOTSUP


def test_null_handles():
    import ctypes

    lib = bcv.lib()
    n = ctypes.c_int64()
    assert lib.bcv_tree_num_leaves(None, ctypes.byref(n)) == bcv.bcv.EINVAL
    assert lib.bcv_vtv_apply(None, None, None, None) == bcv.bcv.EINVAL
    assert b"NULL" in lib.bcv_last_error()
    lib.bcv_plan_destroy(None)  # no-op
    lib.bcv_tree_destroy(None)


def test_forest_leaves_are_the_meshes_leaves():
    """Each mesh of a forest has exactly the leaves of its own BC mesh, in the same order."""
    from oracle.mesh import BCMesh

    Ls = [3, 4, 2, 3]
    t = bcv.build_bc_forest(Ls)
    lv = t.leaves().astype(np.int64)
    mesh = t.leaf_mesh()
    assert np.array_equal(np.bincount(mesh), [len(BCMesh(L).leaf_array()) for L in Ls])
    for m, L in enumerate(Ls):
        loc = lv[mesh == m].copy()
        loc[:, 1] -= (4 * m) << loc[:, 0]
        assert np.array_equal(loc, BCMesh(L).leaf_array())


def test_forest_with_both_markings():
    Ls, marks = [5, 3, 4], [1, 0, 1]
    t = bcv.build_bc_forest(Ls, marks)
    lv = t.leaves().astype(np.int64)
    mesh = t.leaf_mesh()
    for m, (L, mk) in enumerate(zip(Ls, marks)):
        loc = lv[mesh == m].copy()
        loc[:, 1] -= (4 * m) << loc[:, 0]
        assert np.array_equal(loc, BCMesh(L, mk).leaf_array())


def test_forest_argument_errors():
    for Ls in ([], [1], [10], [3, 0]):
        with pytest.raises(bcv.BCVError) as e:
            bcv.build_bc_forest(Ls)
        assert e.value.status == bcv.bcv.EINVAL


def test_mesh_geometry_arguments():
    """Geometry: a cube box is accepted, a non-cube box or a zero side is refused, the ball map is
    not built (BCV_ENOTSUP)."""
    t = bcv.build_bc_tree(3, lo=(1.0, -2.0, 0.5), hi=(3.0, 0.0, 2.5))
    assert t.num_leaves() == len(BCMesh(3).leaf_array())
    for lo, hi in (((0, 0, 0), (1, 2, 1)), ((0, 0, 0), (0, 1, 1)), ((1, 1, 1), (0, 0, 0))):
        with pytest.raises(bcv.BCVError) as e:
            bcv.build_bc_tree(3, lo=lo, hi=hi)
        assert e.value.status == bcv.bcv.EINVAL
    with pytest.raises(bcv.BCVError) as e:
        bcv.build_bc_tree(3, geometry=7)
    assert e.value.status == bcv.bcv.EINVAL


@pytest.mark.parametrize("lo,side", [((0.0, 0.0, 0.0), 1.0), ((1.0, -2.0, 0.5), 2.0)])
def test_gauss_points_match_oracle(lo, side):
    """The library's Gauss points and weights against the oracle's point rule on the unit cube,
    mapped to the cube lo + side [0,1]^3."""
    from oracle import direct

    L = 4
    hi = tuple(x + side for x in lo)
    t = bcv.build_bc_tree(L, lo=lo, hi=hi)
    xyz, w = t.gauss_points()
    lv = BCMesh(L).leaf_array()
    a = np.ldexp(1.0, -lv[:, 0].astype(np.int32))
    pts, wo = direct.gauss_points(lv[:, 1:4] * a[:, None], a)
    assert np.allclose(xyz, np.asarray(lo) + side * pts, rtol=0, atol=1e-15 * side)
    assert np.allclose(w, side ** 3 * np.broadcast_to(wo[:, None], w.shape), rtol=1e-15, atol=0)


@pytest.mark.parametrize("lo,side", [((0.0, 0.0, 0.0), 1.0), ((1.0, -2.0, 0.5), 2.0)])
def test_ball_gauss_points_match_oracle(lo, side):
    """Ball meshes: the library's mapped Gauss points and weights (cube-to-ball map of its own)
    against the mapped-mesh oracle's, placed in the ball inscribed in lo + side [0,1]^3."""
    from oracle import mapped

    L = 4
    hi = tuple(x + side for x in lo)
    t = bcv.build_bc_tree(L, lo=lo, hi=hi, geometry=bcv.GEOM_BALL)
    xyz, w = t.gauss_points()
    mm = mapped.MappedMesh(BCMesh(L), "ball")
    assert np.abs(xyz - (np.asarray(lo) + side * mm.points)).max() <= 4e-16 * side * (1 + np.abs(lo).max())
    assert np.abs(w / (side ** 3 * mm.weights) - 1).max() <= 1e-13
    assert abs(w.sum() / (np.pi / 6 * side ** 3) - 1) < 1e-3  # the ball's volume, to the rule's error


def test_order_range():
    t = bcv.build_bc_tree(3)
    for q in (-1, 11):
        with pytest.raises(bcv.BCVError) as e:
            bcv.plan_interactions(t, q=q)
        assert e.value.status == bcv.bcv.EINVAL


def test_basis_options_checked_before_device_use():
    t = bcv.build_bc_tree(3)
    with pytest.raises(bcv.BCVError) as e:
        bcv.plan_interactions(t, basis_degree=2)
    assert e.value.status == bcv.bcv.EINVAL
    for kw in ({"precision": bcv.MIXED_F32}, {"boundary": True}):
        with pytest.raises(bcv.BCVError) as e:
            bcv.plan_interactions(t, basis_degree=1, **kw)
        assert e.value.status == bcv.bcv.ENOTSUP


@pytest.mark.parametrize("degrees", [(0, 0), (1, 1), (2, 2), (3, 1), (1, 3), (4, 3)])
def test_touching_basis_blocks_against_oracle(degrees):
    """The library's touching blocks (self-similarity of the cube with regular pairs by 6-D Gauss,
    host) against the oracle's (convolution reduction with Duffy pyramids), every kind of contact."""
    from oracle import basis

    p_t, p_s = degrees
    cases = [((0, 0, 0), 1, 1), ((1, 0, 0), 1, 1), ((0, -1, 1), 1, 1), ((1, 1, -1), 1, 1), ((0, 0, 1), 1, 2),
             ((-2, 0, 0), 1, 2), ((1, -2, 0), 1, 2), ((-2, -2, 1), 1, 2), ((0, 0, -1), 2, 1), ((2, 1, 0), 2, 1),
             ((-1, 2, -1), 2, 1)]
    for off, st, ss in cases:
        got = bcv.touching_basis_block(p_t, p_s, st, ss, off)
        ref = basis.touching_block(np.zeros(3, dtype=np.int64), st, np.array(off), ss, 1.0, p_t, p_s) * 4.0 * np.pi
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)), (off, st, ss)


def test_touching_basis_block_errors():
    for args in ((9, 0, 1, 1, (1, 0, 0)), (0, -1, 1, 1, (1, 0, 0)), (1, 1, 2, 2, (1, 0, 0)),
                 (1, 1, 1, 1, (2, 0, 0)), (1, 1, 1, 2, (-1, 0, -1)), (1, 1, 2, 1, (-2, 0, 0))):
        with pytest.raises(bcv.BCVError) as e:
            bcv.touching_basis_block(*args)
        assert e.value.status == bcv.bcv.EINVAL
