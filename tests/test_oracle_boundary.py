"""Pins of the BtV oracle (boundary-to-volume potentials, Algorithm 3)."""

import numpy as np
import pytest

import synth
from oracle import boundary as B
from oracle import touching
from oracle.mesh import BCMesh


def box_faces(lo, hi):
    """The six faces of the box [lo, hi] with outward normals: (flo, fhi, axis, sign)."""
    out = []
    for ax in range(3):
        for side in (0, 1):
            flo, fhi = np.array(lo, float), np.array(hi, float)
            flo[ax] = fhi[ax] = hi[ax] if side else lo[ax]
            out.append((flo, fhi, ax, 2.0 * side - 1.0))
    return out


@pytest.mark.parametrize("wlo,whi,inside", [
    ((0.25, 0.25, 0.25), (0.5, 0.5, 0.5), True),   # interior cell
    ((0.0, 0.0, 0.0), (0.25, 0.25, 0.25), True),   # corner cell: touches three faces
    ((0.5, 0.0, 0.25), (0.75, 0.25, 0.5), True),   # touches one face
    ((1.0, 0.25, 0.25), (1.25, 0.5, 0.5), False),  # outside, touching a face
    ((-0.5, 1.0, 1.0), (0.0, 1.5, 1.5), False),    # outside, touching a corner only
])
def test_double_layer_gauss_law(wlo, whi, inside):
    """Gauss: the double layer of density 1 on a closed surface is -1 inside and 0 outside, so the
    exact double-layer entries of a cell against the six faces of the unit cube sum to -|w| or 0
    (the touching ones go through the Duffy branch)."""
    tot = sum(B.cell_face_integral(wlo, whi, flo, fhi, ax, sg, "double") for flo, fhi, ax, sg in box_faces(
        (0, 0, 0), (1, 1, 1)))
    vol = np.prod(np.subtract(whi, wlo))
    assert abs(tot - (-vol if inside else 0.0)) <= 1e-13 * vol


def _slab_limit(wlo, whi, flo, fhi, ax, side):
    """V by an independent route: the volume integral of oracle.touching over a slab of thickness t
    on the face, divided by t, Richardson-extrapolated over t = 1e-2, 5e-3, 2.5e-3."""
    vals = []
    for t in (1e-2, 5e-3, 2.5e-3):
        blo, bhi = np.array(flo, float), np.array(fhi, float)
        if side == 1:
            blo[ax] -= t
        else:
            bhi[ax] += t
        vals.append(touching.box_pair_integral(wlo, whi, blo, bhi, n=30) / t / (4 * np.pi))
    r1, r2 = 2 * vals[1] - vals[0], 2 * vals[2] - vals[1]
    return (4 * r2 - r1) / 3


@pytest.mark.parametrize("case,tol", [
    (((0, 0, 0), (1, 1, 1), (0, 0, 0), (1, 1, 0), 2, 0), 2e-6),  # the cell's own face
    (((0, 0, 0), (1, 1, 1), (1, 0, 0), (2, 1, 0), 2, 0), 2e-7),  # coplanar, sharing an edge
    (((0, 0, 0), (1, 1, 1), (1, 1, 0), (2, 2, 0), 2, 0), 2e-8),  # coplanar, sharing a vertex
    (((0, 0, 1), (1, 1, 2), (0, 0, 0), (1, 1, 0), 2, 0), 2e-8),  # one cell apart
    (((0, 0, 0), (2, 2, 2), (2, 0, 0), (2, 1, 1), 0, 1), 2e-6),  # a small face on a big cell
])
def test_single_layer_against_slab_limit(case, tol):
    wlo, whi, flo, fhi, ax, side = case
    v = B.cell_face_integral(wlo, whi, flo, fhi, ax, 2.0 * side - 1.0, "single")
    assert abs(v - _slab_limit(wlo, whi, flo, fhi, ax, side)) <= tol * abs(v)


def test_point_rule_tends_to_exact_with_distance():
    """The 2x2x2 x 2x2 point rule approaches the exact entries as the pair separates."""
    errs = []
    for d in (2.0, 4.0, 8.0):
        wlo, whi = np.array([0.0, 0.0, d]), np.array([1.0, 1.0, d + 1.0])
        flo, fhi = B.face_box(np.zeros(3), 1.0, 2, 1)
        V = B.cell_face_integral(wlo, whi, flo, fhi, 2, 1.0, "single")
        K = B.cell_face_integral(wlo, whi, flo, fhi, 2, 1.0, "double")
        Vp, Kp = B.point_rule(wlo, 1.0, np.zeros(3), 1.0, 2, 1)
        errs.append(max(abs(Vp - V) / V, abs(Kp - K) / abs(K)))
    assert errs[0] > errs[1] > errs[2] and errs[0] < 2e-2 and errs[2] < 2e-4


def test_homogeneity():
    """V scales as length^4 and K as length^3 (both kernels are homogeneous)."""
    args = ((0, 0, 0), (1, 1, 1), (1, 0, 0), (2, 1, 0), 2, -1.0)
    big = ((0, 0, 0), (2, 2, 2), (2, 0, 0), (4, 2, 0), 2, -1.0)
    for kind, p in (("single", 4), ("double", 3)):
        a = B.cell_face_integral(*args, kind)
        b = B.cell_face_integral(*big, kind)
        assert abs(b - 2 ** p * a) <= 1e-12 * abs(b)


@pytest.fixture(scope="module")
def mesh2():
    m = BCMesh(2)
    faces = B.boundary_faces(m)
    lv = m.leaf_array()
    fk = np.column_stack([lv[faces[:, 0]], faces[:, 1:]])
    qf, gf = synth.face_data(fk, seed=0)
    return m, faces, qf, gf, B.apply_direct(m, qf, gf)


def test_boundary_faces_cover_gamma():
    for L in (2, 3):
        m = BCMesh(L)
        faces = B.boundary_faces(m)
        assert len(faces) == 6 * 4 ** L
        assert np.all(m.leaf_array()[faces[:, 0], 0] == L)


def test_exact_cover():
    """Every (leaf, face) pair is near (the face's cell has an ancestor at the leaf's level among
    the leaf's neighbours) or far at exactly one level (ancestors in each other's interaction
    lists, the source a boundary cell)."""
    m = BCMesh(3)
    F = B.BtVFMM(m, 2)
    lv = F.leaves
    for t in range(0, len(lv), 23):
        lev, i, j, k = lv[t]
        near = set(F.near_faces(t))
        for f, (leaf, ax, side) in enumerate(F.faces):
            _, fi, fj, fk = lv[leaf]
            hits = 0
            for l in range(1, lev + 1):
                tc = (i >> (lev - l), j >> (lev - l), k >> (lev - l))
                sc = (fi >> (m.L - l), fj >> (m.L - l), fk >> (m.L - l))
                if sc in m.interaction_list(l, tc):
                    assert m.on_boundary(l, sc)
                    hits += 1
            assert hits + (f in near) == 1


def test_o2_converges_to_o1(mesh2):
    """O2 - O1 decreases geometrically in q (stated: about 4e-5, 8e-6, 4e-7 for q = 4, 6, 8 at L = 2)."""
    m, faces, qf, gf, u1 = mesh2
    errs = [np.linalg.norm(B.BtVFMM(m, q).apply(qf, gf) - u1) / np.linalg.norm(u1) for q in (4, 6, 8)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] < 1e-4 and errs[2] < 1e-6


def test_representation_formula(mesh2):
    """Green's representation formula: for harmonic u, V[du/dn] - K[u] = u in the cube. With face
    averages as data and cell averages as output, the BtV result matches the cell averages of u to
    discretisation accuracy (stated: 1.8e-3 relative at L = 2, 6.9e-4 at L = 3)."""
    m, faces, qf, gf, u1 = mesh2
    lv = m.leaf_array()
    charges, poles = synth.harmonic_params(0)
    avg = synth.cell_average(lv, lambda x: synth.harmonic(x, charges, poles), n=4)
    vol = np.ldexp(1.0, -3 * lv[:, 0].astype(np.int32))
    err = np.linalg.norm(u1 / vol - avg) / np.linalg.norm(avg)
    assert err < 5e-3


def test_library_touching_table_matches_oracle():
    """The library's touching (cell, face) table (host computation, self-similarity of the pair)
    against the oracle's convolution integrals, all 108 classes where cell and face meet."""
    import itertools

    import paper_2112_00864_amd as bcv

    V, K = bcv.boundary_touching_integrals()
    n = 0
    for ax in range(3):
        for o in itertools.product((-1, 0, 1), repeat=3):
            for side in (0, 1):
                c = (((ax * 3 + o[0] + 1) * 3 + o[1] + 1) * 3 + o[2] + 1) * 2 + side
                flo, fhi = B.face_box(np.array(o, float), 1.0, ax, side)
                if not np.all(np.maximum(flo, 0) <= np.minimum(fhi, 1)):
                    assert V[c] == 0.0 and K[c] == 0.0
                    continue
                n += 1
                ev = B.cell_face_integral(np.zeros(3), np.ones(3), flo, fhi, ax, 2.0 * side - 1, "single")
                ek = B.cell_face_integral(np.zeros(3), np.ones(3), flo, fhi, ax, 2.0 * side - 1, "double")
                assert abs(V[c] - ev) <= 1e-13 * abs(ev)
                assert abs(K[c] - ek) <= 1e-13 * abs(ek)
    assert n == 108


def test_vtb_is_the_adjoint_of_the_btv_single_layer(mesh2):
    """VtB (Algorithm 2) and the single-layer part of BtV (Algorithm 3) have the same entries
    V_lf, so <VtB f, q>_faces = <f, BtV(q, 0)>_leaves: exactly for O1, and for O2 too, whose
    fixed-q truncated two-centre kernel is symmetric and whose near sets agree."""
    m, faces, qf, gf, _ = mesh2
    lv = m.leaf_array()
    f = synth.leaf_density(lv, seed=0)
    zero = np.zeros(len(faces))
    u1 = B.vtb_direct(m, f)
    b1 = B.apply_direct(m, qf, zero)
    assert abs(u1 @ qf - f @ b1) <= 1e-14 * abs(u1 @ qf)
    u2 = B.VtBFMM(m, 4).apply(f)
    b2 = B.BtVFMM(m, 4).apply(qf, zero)
    assert abs(u2 @ qf - f @ b2) <= 1e-14 * abs(u2 @ qf)
    # and O2 -> O1 (stated: 3.8e-6 at q = 4, 6.2e-8 at q = 6)
    assert np.linalg.norm(u2 - u1) / np.linalg.norm(u1) < 1e-5


def test_vtb_constant_density_box_closed_form():
    """f = 1: the face integrals of the homogeneous-box potential (closed form, tests/closed_forms.py)
    at point-rule accuracy (stated: 7.8e-5 relative at h = 1/4)."""
    import closed_forms

    m = BCMesh(2)
    lv = m.leaf_array()
    faces = B.boundary_faces(m)
    u = B.VtBFMM(m, 6).apply(np.ones(len(lv)))
    a = 0.25
    ref = np.empty(len(faces))
    g, w = np.polynomial.legendre.leggauss(8)
    g, w = 0.5 * (g + 1), 0.5 * w
    for n, (leaf, ax, side) in enumerate(faces):
        _, i, j, k = lv[leaf]
        lo = np.array([i, j, k]) * a
        o1, o2 = (ax + 1) % 3, (ax + 2) % 3
        tot = 0.0
        for s, ws in zip(g, w):
            for t, wt in zip(g, w):
                p = lo.copy()
                p[ax] += side * a
                p[o1] += a * s
                p[o2] += a * t
                tot += ws * wt * closed_forms.box_potential(p)
        ref[n] = tot * a * a
    assert np.max(np.abs(u - ref) / np.abs(ref)) < 3e-4


@pytest.mark.parametrize("L", [2, 3])
def test_sampled_direct_sums_equal_the_loops(L):
    """The vectorised O1 forms at sampled targets (apply_direct_sampled over all faces,
    vtb_direct_sampled over all leaves) against the entry-by-entry loops (apply_direct, vtb_direct),
    which share only the entry definitions with them: the first and last leaf and face, the coarse
    and fine leaves among 20 random ones."""
    m = BCMesh(L)
    faces = B.boundary_faces(m)
    lv = m.leaf_array()
    fk = np.column_stack([lv[faces[:, 0]], faces[:, 1:]])
    qf, gf = synth.face_data(fk, seed=0)
    rng = np.random.default_rng(3)
    first_of_level = [int(np.argmax(lv[:, 0] == lev)) for lev in np.unique(lv[:, 0])]
    t = np.unique(np.concatenate([[0, len(lv) - 1], first_of_level, rng.choice(len(lv), 20, replace=False)]))
    assert len(np.unique(lv[t, 0])) == len(np.unique(lv[:, 0]))
    a = B.apply_direct(m, qf, gf, targets=t)
    b = B.apply_direct_sampled(m, qf, gf, t)
    assert np.max(np.abs(a - b) / np.abs(a)) <= 1e-13
    f = synth.leaf_density(lv, seed=0)
    fsel = np.unique(np.concatenate([[0, len(faces) - 1], rng.choice(len(faces), 20, replace=False)]))
    u = B.vtb_direct(m, f, face_idx=fsel)
    v = B.vtb_direct_sampled(m, f, fsel)
    assert np.max(np.abs(u - v) / np.abs(u)) <= 1e-13
