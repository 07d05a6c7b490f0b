"""Boundary-concentrated cube-octree mesh and its cell lists (test infrastructure only).

Follows Section 2 of the paper (Boundary Concentrated Mesh) and Section 3 (Boundary
Concentrated FMM), written for axis-aligned cubes of the unit cube [0,1]^3:

  * levels C_l, boundary cells B_l, marked cells M_l, leaves L_l = C_l minus M_l,
    C_{l+1} = children of M_l, L*_l = L_l for l < L and L*_L = C_L (Sec. 2);
  * centre x_w and diameter rho_w (eq. def:diam), separation ratio (eq. def:sepRatio),
    neighbours N(w) (eq. def:neighbors);
  * interaction list I(w): children of the parent's neighbours that are not neighbours of
    w; at level 0, C_0 minus N(w) (Sec. 2, after eq. spaceDecomp:Om);
  * N_L(w), N_M(w) and the extended neighbour list N*(w) (Sec. 3, before Lemma 1).

Marking rules (l < L):
  marking=0  M_l = B_l: cells with a face on the boundary are refined (the default);
  marking=1  M_l = {w in C_l : N(w) meets B_l}: cells with a boundary cell among their
             neighbours are refined (Sec. 2, the definition of M_l).
A marked source in N_M(w) stands for all of its leaf descendants, since the density lives
on leaves.

A cell is a tuple (i, j, k) at a level l; it is the cube [i, i+1] x [j, j+1] x [k, k+1]
scaled by 2^-l. A leaf is identified by (l, i, j, k).
"""

import itertools

import numpy as np

ETA0 = 0.5


def neighbour_offset(o, eta0=ETA0):
    """True if two level-l cubes at integer offset o are neighbours (eq. def:neighbors).

    A cube of side a has rho = a*sqrt(3)/2 (eq. def:diam), so eq. def:sepRatio gives
    eta = (rho + rho')/|x - x'| = sqrt(3)/|o| and eta > eta0 iff eta0^2 |o|^2 < 3.
    For eta0 = 0.5 the test reads |o|^2 < 12 and is exact in floating point; the tie
    |o|^2 = 12 (offset (2,2,2)) is not a neighbour because the inequality is strict.
    o = 0 is a neighbour (eta(w,w) = infinity).
    """
    n2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2]
    return eta0 * eta0 * n2 < 3.0


STENCIL = [o for o in itertools.product(range(-3, 4), repeat=3) if neighbour_offset(o)]


def morton_key(i, j, k, bits):
    """Interleave bits of (i, j, k): bit b of i goes to 3b, of j to 3b+1, of k to 3b+2."""
    key = 0
    for b in range(bits):
        key |= ((i >> b) & 1) << (3 * b)
        key |= ((j >> b) & 1) << (3 * b + 1)
        key |= ((k >> b) & 1) << (3 * b + 2)
    return key


def children(c):
    i, j, k = c
    return [(2 * i + dx, 2 * j + dy, 2 * k + dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]


def parent(c):
    return (c[0] >> 1, c[1] >> 1, c[2] >> 1)


class BCMesh:
    """The BC refinement of the unit cube down to level L (Sec. 2)."""

    def __init__(self, L, marking=0):
        if not 1 <= L <= 9:
            raise ValueError("L must be in 1..9")
        if marking not in (0, 1):
            raise ValueError("marking must be 0 or 1")
        self.L = L
        self.marking = marking
        self.levels = []  # level -> list of cells (i,j,k), Morton order at that level
        self.index = []  # level -> {cell: position}
        self.refined = []  # level -> set of marked cells M_l (empty at level L)
        cells = [(0, 0, 0)]
        for lev in range(L + 1):
            cells = sorted(cells, key=lambda c, b=lev: morton_key(*c, b))
            self.levels.append(cells)
            self.index.append({c: n for n, c in enumerate(cells)})
            if lev < L and marking == 0:
                marked = [c for c in cells if self.on_boundary(lev, c)]  # M_l = B_l
            elif lev < L:  # M_l: some neighbour in C_l is a boundary cell
                marked = [c for c in cells if any(self.on_boundary(lev, nb) for nb in self.neighbours(lev, c))]
            else:
                marked = []  # every level-L cell is a leaf: L*_L = C_L
            self.refined.append(set(marked))
            cells = [ch for c in marked for ch in children(c)]  # C_{l+1}
        leaves = [(lev, *c) for lev in range(L + 1) for c in self.levels[lev] if c not in self.refined[lev]]
        leaves.sort(key=lambda t: morton_key(t[1] << (L - t[0]), t[2] << (L - t[0]), t[3] << (L - t[0]), L))
        self.leaves = leaves  # sorted by the Morton key of the lower corner at level-L resolution
        self.leaf_index = {t: n for n, t in enumerate(leaves)}

    # -- Sec. 2 sets -------------------------------------------------------------------------
    @staticmethod
    def on_boundary(lev, c):
        """w in B_l: the cube has a face on the boundary of [0,1]^3."""
        top = (1 << lev) - 1
        return any(x == 0 or x == top for x in c)

    def exists(self, lev, c):
        return c in self.index[lev]

    def is_refined(self, lev, c):
        return c in self.refined[lev]

    def side(self, lev):
        return 2.0 ** (-lev)

    def centre(self, lev, c):
        a = self.side(lev)
        return np.array([(c[0] + 0.5) * a, (c[1] + 0.5) * a, (c[2] + 0.5) * a])

    # -- lists ----------------------------------------------------------------------------------
    def neighbours(self, lev, c):
        """N(w): cells of C_l with eta(w, w') > eta0, including w itself (eq. def:neighbors)."""
        idx = self.index[lev]
        out = []
        for o in STENCIL:
            cc = (c[0] + o[0], c[1] + o[1], c[2] + o[2])
            if cc in idx:
                out.append(cc)
        return out

    def interaction_list(self, lev, c):
        """I(w): cells of C_l whose parents are neighbours of w's parent, minus N(w).

        At level 0, I(w) = C_0 minus N(w), which is empty because C_0 is the root alone.
        """
        if lev == 0:
            return [cc for cc in self.levels[0] if not neighbour_offset(tuple(x - y for x, y in zip(cc, c)))]
        out = []
        for pp in self.neighbours(lev - 1, parent(c)):
            if not self.is_refined(lev - 1, pp):
                continue  # a leaf parent-neighbour has no children in C_l
            for cc in children(pp):
                o = (cc[0] - c[0], cc[1] - c[1], cc[2] - c[2])
                if not neighbour_offset(o):
                    out.append(cc)
        return out

    def leaf_descendants(self, lev, c):
        """All leaves contained in cell (lev, c) (the cell itself if it is a leaf)."""
        if not self.is_refined(lev, c):
            return [(lev, *c)]
        out = []
        for ch in children(c):
            out.extend(self.leaf_descendants(lev + 1, ch))
        return out

    def ancestor(self, lev, c, target_level):
        """pi_l(w): the ancestor of (lev, c) at target_level <= lev."""
        s = lev - target_level
        return (c[0] >> s, c[1] >> s, c[2] >> s)

    def extended_neighbours(self, lev, c):
        """N*(w) = N_M(w) union the N_L of every ancestor pi_l'(w), l' = 0..l(w) (Sec. 3).

        Returned as (level, cell, refined) triples of cells at any level.
        """
        out = []
        for nb in self.neighbours(lev, c):
            if self.is_refined(lev, nb):
                out.append((lev, nb, True))  # N_M(w)
        for lp in range(lev + 1):
            anc = self.ancestor(lev, c, lp)
            for nb in self.neighbours(lp, anc):
                if not self.is_refined(lp, nb):
                    out.append((lp, nb, False))  # N_L(pi_l'(w))
        return out

    def near_leaf_sources(self, lev, c):
        """Leaves y such that (w, y) lies in w x N*(w): marked cells expanded to their leaves."""
        out = []
        for lp, nb, refined in self.extended_neighbours(lev, c):
            if refined:
                out.extend(self.leaf_descendants(lp, nb))
            else:
                out.append((lp, *nb))
        return out

    # -- whole-mesh enumerations ---------------------------------------------------------------
    def all_cells(self):
        for lev in range(self.L + 1):
            for c in self.levels[lev]:
                yield lev, c

    def level_counts(self):
        """(#C_l, #M_l, #L*_l) per level."""
        return [(len(self.levels[lev]), len(self.refined[lev]), len(self.levels[lev]) - len(self.refined[lev]))
                for lev in range(self.L + 1)]

    def leaf_array(self):
        """Leaves as an int array (n, 4) of (level, i, j, k) in leaf order."""
        return np.array(self.leaves, dtype=np.int64).reshape(-1, 4)

    def near_pairs(self):
        """All near (target leaf index, source leaf index) pairs, as two int arrays."""
        ti, si = [], []
        for n, (lev, i, j, k) in enumerate(self.leaves):
            for s in self.near_leaf_sources(lev, (i, j, k)):
                ti.append(n)
                si.append(self.leaf_index[s])
        return np.array(ti, dtype=np.int64), np.array(si, dtype=np.int64)

    def interaction_pairs(self):
        """All M2L pairs as a list of (level, target cell, source cell)."""
        out = []
        for lev, c in self.all_cells():
            for s in self.interaction_list(lev, c):
                out.append((lev, c, s))
        return out
