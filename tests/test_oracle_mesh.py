"""Pins of the oracle's BC mesh and lists (Sec. 2 and Sec. 3 of the paper)."""

import itertools
import math

import numpy as np
import pytest

from oracle.mesh import BCMesh, STENCIL, neighbour_offset


def test_neighbour_stencil_matches_separation_ratio():
    # eq. def:sepRatio with rho = a sqrt(3)/2 (eq. def:diam), evaluated in floating point away from the tie.
    for o in itertools.product(range(-4, 5), repeat=3):
        n2 = sum(x * x for x in o)
        if n2 == 12:
            assert not neighbour_offset(o)  # eta == eta0 exactly: strict inequality excludes it
            continue
        eta = math.inf if n2 == 0 else math.sqrt(3.0) / math.sqrt(n2)
        assert neighbour_offset(o) == (eta > 0.5)
    assert len(STENCIL) == 171
    assert (2, 2, 2) not in STENCIL and (3, 1, 1) in STENCIL


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_levels_and_leaf_tiling(L):
    m = BCMesh(L)
    counts = m.level_counts()
    for lev in range(L):
        assert counts[lev + 1][0] == 8 * counts[lev][1]  # C_{l+1} = children of M_l
    # eq. spaceDecomp:Om: the leaves tile Omega exactly once (rasterised at level L).
    n = 1 << L
    cover = np.zeros((n, n, n), dtype=np.int32)
    for lev, i, j, k in m.leaves:
        s = 1 << (L - lev)
        cover[i * s:(i + 1) * s, j * s:(j + 1) * s, k * s:(k + 1) * s] += 1
    assert np.all(cover == 1)
    # M_l are exactly the cells with a face on the boundary (marking reading), l < L.
    for lev in range(L):
        for c in m.levels[lev]:
            assert m.is_refined(lev, c) == any(x in (0, (1 << lev) - 1) for x in c)


def test_leaf_counts_cross_check():
    # Leaf and cell counts of the cube BC mesh recomputed from the definitions (regression values).
    assert [len(BCMesh(L).leaves) for L in (2, 3, 4, 5)] == [64, 456, 2528, 11992]


@pytest.mark.parametrize("L", [3, 4])
def test_two_to_one_balance(L):
    m = BCMesh(L)
    lv = m.leaf_array()
    size = 1 << (L - lv[:, 0])
    lo = lv[:, 1:4] * size[:, None]
    for t in range(len(lv)):
        lo2 = np.maximum(lo[t], lo)
        hi2 = np.minimum(lo[t] + size[t], lo + size[:, None])
        touch = np.all(lo2 <= hi2, axis=1)
        assert np.all(np.abs(lv[touch, 0] - lv[t, 0]) <= 1)


@pytest.mark.parametrize("L", [3, 4])
def test_exact_cover_of_omega_times_omega(L):
    """eq. spaceDecomp:OmOm: every ordered leaf pair is in exactly one near block or one far block."""
    m = BCMesh(L)
    n = len(m.leaves)
    cov = np.zeros((n, n), dtype=np.int16)
    ti, si = m.near_pairs()
    np.add.at(cov, (ti, si), 1)
    desc = {}

    def leaves_of(lev, c):
        key = (lev, c)
        if key not in desc:
            desc[key] = np.array([m.leaf_index[t] for t in m.leaf_descendants(lev, c)])
        return desc[key]

    for lev, c in m.all_cells():
        il = m.interaction_list(lev, c)
        if il:
            b = np.concatenate([leaves_of(lev, s) for s in il])
            cov[np.ix_(leaves_of(lev, c), b)] += 1
    assert cov.min() == 1 and cov.max() == 1


@pytest.mark.parametrize("L", [3, 4])
def test_interaction_lists(L):
    m = BCMesh(L)
    sizes_n, sizes_i = [], []
    ilists = {(lev, c): set(m.interaction_list(lev, c)) for lev, c in m.all_cells()}
    for (lev, c), il in ilists.items():
        nb = set(m.neighbours(lev, c))
        sizes_n.append(len(nb))
        sizes_i.append(len(il))
        assert not (nb & il)  # I(w) and N(w) are disjoint
        for s in il:
            assert c in ilists[(lev, s)]  # symmetric
            p, ps = (c[0] >> 1, c[1] >> 1, c[2] >> 1), (s[0] >> 1, s[1] >> 1, s[2] >> 1)
            assert neighbour_offset(tuple(x - y for x, y in zip(p, ps)))  # parents are neighbours
    # Theorem 1: list sizes are bounded (same maxima at every L for this mesh).
    assert max(sizes_n) == 101 and max(sizes_i) == 304


def test_list_counts_cross_check():
    m = BCMesh(4)
    ti, _ = m.near_pairs()
    assert len(ti) == 359920
    assert len(m.interaction_pairs()) == 734160


# -- marking rule 1: M_l = {w in C_l : N(w) meets B_l} (Sec. 2) --------------------------------------

def _neighbour_marking_counts(L):
    """(#C_l, #M_l, #L*_l) of marking rule 1 in closed form. A level-l cell d cells away from the
    nearest boundary plane has the boundary cell straight across that plane at offset d, and every
    boundary cell at least d away along some axis, so it is marked iff d^2 < 12 (d <= 3). Every cell
    with d <= 3 exists (its parent has d <= 1), so with n = 2^l: #M_l = n^3 - max(n - 8, 0)^3 for
    l < L, #C_0 = 1 and #C_{l+1} = 8 #M_l."""
    out, c = [], 1
    for lev in range(L + 1):
        n = 1 << lev
        m = n ** 3 - max(n - 8, 0) ** 3 if lev < L else 0
        out.append((c, m, c - m))
        c = 8 * m
    return out


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6])
def test_neighbour_marking_counts(L):
    assert BCMesh(L, 1).level_counts() == _neighbour_marking_counts(L)


def test_neighbour_marking_rule_and_tiling():
    L = 5
    m = BCMesh(L, 1)
    # the rule itself, by the separation ratio in floating point (eq. def:sepRatio, def:diam)
    for lev in range(L):
        a = 2.0 ** -lev
        bnd = [c for c in m.levels[lev] if m.on_boundary(lev, c)]
        for c in m.levels[lev][::7]:
            eta = [math.inf if b == c else math.sqrt(3.0) * a / math.dist(m.centre(lev, b), m.centre(lev, c))
                   for b in bnd]
            assert m.is_refined(lev, c) == (max(eta) > 0.5 + 1e-12)
    n = 1 << L
    cover = np.zeros((n, n, n), dtype=np.int32)
    for lev, i, j, k in m.leaves:
        s = 1 << (L - lev)
        cover[i * s:(i + 1) * s, j * s:(j + 1) * s, k * s:(k + 1) * s] += 1
    assert np.all(cover == 1)


def test_neighbour_marking_balance_and_near_levels():
    """Touching leaves differ by at most one level; near-field pairs by at most two (marking rule 1
    refines in shells four cells thick), against L - 1 with the face rule."""
    L = 6
    m = BCMesh(L, 1)
    lv = m.leaf_array()
    size = 1 << (L - lv[:, 0])
    lo = lv[:, 1:4] * size[:, None]
    gaps = set()
    for t in range(0, len(lv), 211):
        lo2 = np.maximum(lo[t], lo)
        hi2 = np.minimum(lo[t] + size[t], lo + size[:, None])
        touch = np.all(lo2 <= hi2, axis=1)
        assert np.all(np.abs(lv[touch, 0] - lv[t, 0]) <= 1)
        lev, i, j, k = m.leaves[t]
        gaps.update(abs(s[0] - lev) for s in m.near_leaf_sources(lev, (i, j, k)))
    assert max(gaps) == 2


def test_neighbour_marking_exact_cover_sampled():
    """eq. spaceDecomp:OmOm for marking rule 1: for sampled target leaves, every source leaf is in
    exactly one near block or one far block (interaction list of an ancestor pair)."""
    L = 5
    m = BCMesh(L, 1)
    n = len(m.leaves)
    desc = {}

    def leaves_of(lev, c):
        if (lev, c) not in desc:
            desc[(lev, c)] = np.array([m.leaf_index[t] for t in m.leaf_descendants(lev, c)])
        return desc[(lev, c)]

    for t in range(0, n, 1453):
        lev, i, j, k = m.leaves[t]
        cov = np.zeros(n, dtype=np.int16)
        np.add.at(cov, [m.leaf_index[s] for s in m.near_leaf_sources(lev, (i, j, k))], 1)
        for lp in range(lev + 1):
            anc = m.ancestor(lev, (i, j, k), lp)
            for s in m.interaction_list(lp, anc):
                cov[leaves_of(lp, s)] += 1
        assert cov.min() == 1 and cov.max() == 1
