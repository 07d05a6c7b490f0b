"""O2: the BC-FMM of Algorithm 1 evaluated phase by phase in FP64 (test infrastructure only).

The far field is represented by order-q Cartesian Taylor expansions (Sec. 3, translation
operators); every phase works on whole levels with dense translation matrices:

  near field    sum of the Galerkin entries (oracle.direct) over each leaf's extended neighbour
                list, a marked neighbour standing for all of its leaves
  moments       the 2x2x2 point rule applied to the monomials (x - centre)^b, |b| <= q, per leaf
  upward pass   children's moments shifted to their parent's centre, finest level first
  interaction   derivative matrices T applied to the moments of each cell's interaction list,
                grouped by integer offset
  downward pass parents' local coefficients shifted to their children, coarsest level first
  evaluation    the local expansion integrated over each leaf with the 2x2x2 point rule

The far field of a leaf pair is therefore the order-q Taylor polynomial of G about the centres
of the ancestors that meet in an interaction list, integrated with the same point rule as
the near field; as q grows the result tends to O1 (oracle.direct).

Expansion order: fixed q by default. q_schedule=1 takes the paper's level-dependent orders
q_l = q + (L - l) (Sec. 4, the FMM error discussion; q is the finest level's order). Reading of the
passes with level-dependent orders, as Algorithm 1 prints them: a level-l cell carries moments and
local coefficients of degree <= q_l; leaf moments are computed to q_l; M2M maps a child's moments
(degree <= q_{l+1}) to the parent's degree <= q_l moments, so the parent's top-degree moments receive
only the child's terms of lower degree; the interaction phase at level l truncates to
|alpha| + |beta| <= q_l; L2L keeps the child's degrees <= q_{l+1}. q_levels gives the orders per
level explicitly (a constant list is the fixed-q method). exact_moments=True takes the other reading
of the upward pass: every cell carries moments of degree <= max_l q_l (leaf moments to that degree,
M2M without truncation), so a cell's moments are exactly those of the point rule over all of its
leaves; the interaction at level l still uses the degrees <= q_l of its sources' moments.
near_order=1 gives the near field the level-dependent Gauss rule of oracle.direct (n_l = 2 + L - l
points per axis on a level-l leaf); the moments and the evaluation keep the 2x2x2 rule, so the
result then tends to oracle.direct.apply_near_order as q grows.
`apply` runs every phase over every cell. `apply_sampled` runs the moment and upward phases
over every cell and then the interaction, downward and evaluation phases only along the
ancestor chains of the given target leaves, which yields the same numbers for those leaves.
"""

import numpy as np

from . import direct
from .taylor import l2l_matrix, m2l_matrix, m2m_matrix, monomials, n_coeffs

_CHILD_POS = [(dx, dy, dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]


class FMM:
    def __init__(self, mesh, q, near_order=0, q_schedule=0, q_levels=None, exact_moments=False):
        self.mesh = mesh
        self.q = q
        self.near_order = near_order
        if q_levels is None:
            q_levels = [q + (mesh.L - lev) if q_schedule else q for lev in range(mesh.L + 1)]
        self.q_of = [int(v) for v in q_levels]
        self.K_of = [n_coeffs(v) for v in self.q_of]
        # degrees carried by the moments of each level
        self.qm_of = [max(self.q_of)] * len(self.q_of) if exact_moments else list(self.q_of)
        self.Km_of = [n_coeffs(v) for v in self.qm_of]
        self.K = n_coeffs(q)
        self.leaves = mesh.leaf_array()
        self.orders = None if near_order == 0 else direct.near_gauss_orders(self.leaves, mesh.L, near_order)
        self._cache = {}
        self._rows = self._leaf_rows()

    # -- helpers -----------------------------------------------------------------------------
    def _leaf_rows(self):
        """Per level: (positions of the level's leaves within the level, their leaf indices)."""
        mesh = self.mesh
        rows = []
        for lev in range(mesh.L + 1):
            pos, idx = [], []
            for p, c in enumerate(mesh.levels[lev]):
                key = (lev, *c)
                if key in mesh.leaf_index:
                    pos.append(p)
                    idx.append(mesh.leaf_index[key])
            rows.append((np.array(pos, dtype=np.int64), np.array(idx, dtype=np.int64)))
        return rows

    def _point_moments(self, lev, cells, chunk=8192, order=None):
        """sum_g w_g (x_g - x_w)^b over the 2x2x2 points of level-lev cells, |b| <= order (default
        q_lev): (n, n_coeffs(order))."""
        order = self.q_of[lev] if order is None else order
        a = self.mesh.side(lev)
        lo_all = np.asarray(cells, dtype=np.float64).reshape(-1, 3) * a
        out = np.empty((len(lo_all), n_coeffs(order)))
        for s in range(0, len(lo_all), chunk):
            lo = lo_all[s : s + chunk]
            pts, w = direct.gauss_points(lo, np.full(len(lo), a))
            centre = lo + 0.5 * a
            mono = monomials(pts - centre[:, None, :], order)  # (n, 8, n_coeffs(order))
            out[s : s + chunk] = mono.sum(axis=1) * w[:, None]
        return out

    def _child_offset(self, lev, pos):
        """x_child - x_parent for a parent at level lev and child position pos in {0,1}^3."""
        a = self.mesh.side(lev)
        return np.array([(p - 0.5) * a / 2.0 for p in pos])

    def _m2m(self, lev, pos):
        """Parent (level lev, the degrees its moments carry) from child (level lev + 1) moments."""
        key = ("m2m", lev, pos)
        if key not in self._cache:
            qp, qc = self.qm_of[lev], self.qm_of[lev + 1]
            M = m2m_matrix(self._child_offset(lev, pos), max(qp, qc))
            self._cache[key] = M[: self.Km_of[lev], : self.Km_of[lev + 1]]
        return self._cache[key]

    def _l2l(self, lev, pos):
        """Child (level lev + 1, degree <= q_{lev+1}) from parent (degree <= q_lev) locals."""
        key = ("l2l", lev, pos)
        if key not in self._cache:
            qp, qc = self.q_of[lev], self.q_of[lev + 1]
            Lm = l2l_matrix(self._child_offset(lev, pos), max(qp, qc))
            self._cache[key] = Lm[: self.K_of[lev + 1], : self.K_of[lev]]
        return self._cache[key]

    def _m2l(self, lev, offsets):
        """T(w, w') for integer offsets (target minus source) between level-lev cells."""
        need = [o for o in set(offsets) if ("m2l", lev, o) not in self._cache]
        if need:
            a = self.mesh.side(lev)
            Ts = m2l_matrix(np.array(need, dtype=np.float64) * a, self.q_of[lev])
            for o, T in zip(need, Ts):
                self._cache[("m2l", lev, o)] = T
        return [self._cache[("m2l", lev, o)] for o in offsets]

    # -- Algorithm 1 phases --------------------------------------------------------------------
    def near_field(self, f, targets):
        """Near-field sums of the targets: Galerkin entries over the extended neighbour list times f."""
        mesh = self.mesh
        ti, si = [], []
        for n, t in enumerate(targets):
            lev, i, j, k = mesh.leaves[t]
            for s in mesh.near_leaf_sources(lev, (i, j, k)):
                ti.append(n)
                si.append(mesh.leaf_index[s])
        ti = np.array(ti, dtype=np.int64)
        si = np.array(si, dtype=np.int64)
        vals = direct.entries(self.leaves, mesh.L, np.asarray(targets, dtype=np.int64)[ti], si, self.orders)
        return np.bincount(ti, weights=vals * f[si], minlength=len(targets))

    def moments(self, f):
        """Leaf moments by level: f times the point-rule integral of each monomial about the centre."""
        mesh = self.mesh
        m = [np.zeros((len(mesh.levels[lev]), self.Km_of[lev])) for lev in range(mesh.L + 1)]
        for lev, (pos, idx) in enumerate(self._rows):
            if len(pos):
                cells = [mesh.levels[lev][p] for p in pos]
                m[lev][pos] = self._point_moments(lev, cells, order=self.qm_of[lev]) * f[idx][:, None]
        return m

    def _children_rows(self, lev):
        """For marked cells of level lev: their positions and, per child position, the child rows."""
        mesh = self.mesh
        par = [p for p, c in enumerate(mesh.levels[lev]) if mesh.is_refined(lev, c)]
        kids = {pos: [] for pos in _CHILD_POS}
        for p in par:
            c = mesh.levels[lev][p]
            for pos in _CHILD_POS:
                ch = (2 * c[0] + pos[0], 2 * c[1] + pos[1], 2 * c[2] + pos[2])
                kids[pos].append(mesh.index[lev + 1][ch])
        return np.array(par, dtype=np.int64), {k: np.array(v, dtype=np.int64) for k, v in kids.items()}

    def upward(self, m):
        """Moments of every marked cell from its eight children, finest level first."""
        for lev in range(self.mesh.L - 1, -1, -1):
            par, kids = self._children_rows(lev)
            if len(par) == 0:
                continue
            acc = np.zeros((len(par), self.Km_of[lev]))
            for pos in _CHILD_POS:
                acc += m[lev + 1][kids[pos]] @ self._m2m(lev, pos).T
            m[lev][par] = acc
        return m

    def interaction(self, m):
        """Local coefficients of every cell from the moments of its interaction list, level by level."""
        mesh = self.mesh
        lam = [np.zeros((len(mesh.levels[lev]), self.K_of[lev])) for lev in range(mesh.L + 1)]
        for lev in range(mesh.L + 1):
            groups = {}
            idx = mesh.index[lev]
            for p, c in enumerate(mesh.levels[lev]):
                for s in mesh.interaction_list(lev, c):
                    o = (c[0] - s[0], c[1] - s[1], c[2] - s[2])
                    groups.setdefault(o, ([], []))
                    groups[o][0].append(p)
                    groups[o][1].append(idx[s])
            offsets = list(groups)
            for o, T in zip(offsets, self._m2l(lev, offsets)):
                tp = np.array(groups[o][0], dtype=np.int64)
                sp = np.array(groups[o][1], dtype=np.int64)
                lam[lev][tp] += m[lev][sp, : self.K_of[lev]] @ T.T  # at most one source per offset
        return lam

    def downward(self, lam):
        """Children's local coefficients receive their parent's, shifted, coarsest level first."""
        for lev in range(self.mesh.L):
            par, kids = self._children_rows(lev)
            if len(par) == 0:
                continue
            for pos in _CHILD_POS:
                lam[lev + 1][kids[pos]] += lam[lev][par] @ self._l2l(lev, pos).T
        return lam

    def evaluation(self, lam, u):
        """Adds each leaf's local expansion, integrated over the leaf with the point rule, to u."""
        mesh = self.mesh
        for lev, (pos, idx) in enumerate(self._rows):
            if len(pos):
                cells = [mesh.levels[lev][p] for p in pos]
                u[idx] += np.sum(self._point_moments(lev, cells) * lam[lev][pos], axis=1)
        return u

    def apply(self, f):
        """The BC-FMM potential at every leaf: all phases of Algorithm 1 over all cells."""
        f = np.asarray(f, dtype=np.float64)
        u = self.near_field(f, np.arange(len(self.leaves)))
        m = self.upward(self.moments(f))
        lam = self.downward(self.interaction(m))
        return self.evaluation(lam, u)

    # -- sampled targets ---------------------------------------------------------------------
    def _local_chain(self, lev, c, m, memo):
        """lambda of cell (lev, c): its own interaction-list sum plus L2L of its parent's lambda."""
        key = (lev, c)
        if key in memo:
            return memo[key]
        mesh = self.mesh
        srcs = mesh.interaction_list(lev, c)
        lam = np.zeros(self.K_of[lev])
        if srcs:
            offs = [(c[0] - s[0], c[1] - s[1], c[2] - s[2]) for s in srcs]
            idx = mesh.index[lev]
            for T, s in zip(self._m2l(lev, offs), srcs):
                lam += T @ m[lev][idx[s], : self.K_of[lev]]
        if lev > 0:
            par = (c[0] >> 1, c[1] >> 1, c[2] >> 1)
            pos = (c[0] & 1, c[1] & 1, c[2] & 1)
            lam = lam + self._l2l(lev - 1, pos) @ self._local_chain(lev - 1, par, m, memo)
        memo[key] = lam
        return lam

    def apply_sampled(self, f, targets):
        """The BC-FMM potential at the given target leaves only."""
        f = np.asarray(f, dtype=np.float64)
        targets = np.asarray(targets, dtype=np.int64)
        u = self.near_field(f, targets)
        m = self.upward(self.moments(f))
        memo = {}
        for n, t in enumerate(targets):
            lev, i, j, k = self.mesh.leaves[t]
            lam = self._local_chain(lev, (i, j, k), m, memo)
            u[n] += float(self._point_moments(lev, [(i, j, k)])[0] @ lam)
        return u


def apply(mesh, f, q, targets=None, near_order=0, q_schedule=0, exact_moments=False):
    fm = FMM(mesh, q, near_order, q_schedule, exact_moments=exact_moments)
    return fm.apply(f) if targets is None else fm.apply_sampled(f, targets)
