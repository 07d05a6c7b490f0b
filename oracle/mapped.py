"""Mapped (curved) BC meshes: O1 and O2 on the images of the cube octree (test infrastructure only).

A mapped mesh is the BC octree of Sec. 2 built on the reference cube [0,1]^3 and pushed through a map
Phi: the leaf w is the curved cell Phi(c_w) of the reference cube c_w, and the Galerkin entries are
(Sec. 1.2, degree 0, indicator basis)

    A_ts = int_{Phi(c_t)} int_{Phi(c_s)} G(x, y) dy dx
         = int_{c_t} int_{c_s} G(Phi(xi), Phi(eta)) J(xi) J(eta) d eta d xi,   J = |det D Phi|.

Maps (oracle/mapped.c): "identity" (the cube mesh itself) and "ball", the analytic cube-to-sphere
map (the volume form of the mapping reviewed by Zucker and Higashi, JCGT 7(2), 2018), which takes
[0,1]^3 onto the ball of centre (1/2, 1/2, 1/2) and radius 1/2.

Readings (the paper works with tetrahedral meshes of a polyhedron, not with mapped cells):
  * the lists N, I and N* are those of the reference octree: neighbourhood (eq. def:neighbors) is
    decided on the reference cubes, whose images the cells are;
  * a cell's expansion centre is the image of its reference centre; P2M, M2M, M2L, L2L and L2P are
    the Taylor translations of Sec. 3 between these (no longer lattice) centres;
  * non-touching pairs take the 2x2x2 Gauss rule of each reference cube, mapped: points Phi(xi_g),
    weights (a^3/8) J(xi_g); moments and evaluation use the same points;
  * touching pairs (the closed reference cubes meet) take the singular rule of mapped.c (Duffy
    pyramids in the relative coordinate, tensor Gauss elsewhere) with the orders RULE; pairs with
    sides in ratio 2 split the larger cube into its children.
With the identity map everything reduces to oracle.direct and oracle.fmm (the touching entries to
the singular rule's approximation of the exact constants).
"""

import numpy as np

from . import _clib
from .direct import gauss_tables
from .taylor import m2l_matrix, monomials, multi_indices, n_coeffs, mi_binom

MAPS = {"identity": 0, "ball": 1}
# singular-rule orders: lambda (radial Duffy), mu (the two Duffy directions), z (boxes away from the
# singularity), s (the inner box), r (regular sub-pairs of a ratio-2 pair)
RULE = dict(n_lam=5, n_mu=7, n_z=5, n_s=3, n_r=4)

_XI = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
_REF = np.array([[_XI[i], _XI[j], _XI[k]] for k in (0, 1) for j in (0, 1) for i in (0, 1)])  # (8, 3)
_CHILD_POS = [(dx, dy, dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]


def map_points(kind, x):
    """Phi(x) and J(x) for reference points x (..., 3)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    shape = x.shape[:-1]
    flat = x.reshape(-1, 3)
    p = np.empty_like(flat)
    j = np.empty(len(flat))
    _clib.lib().om_map(MAPS[kind], len(flat), np.ascontiguousarray(flat), p, j)
    return p.reshape(shape + (3,)), j.reshape(shape)


class MappedMesh:
    """A BC mesh (oracle.mesh.BCMesh) and a map: leaf geometry and point rules."""

    def __init__(self, mesh, kind="ball"):
        if kind not in MAPS:
            raise ValueError("map must be one of %s" % sorted(MAPS))
        self.mesh = mesh
        self.kind = kind
        lv = mesh.leaf_array()
        self.leaves = lv
        self.a = np.ldexp(1.0, -lv[:, 0].astype(np.int32))
        self.lo = lv[:, 1:4] * self.a[:, None]
        pts, jac = map_points(kind, self.lo[:, None, :] + self.a[:, None, None] * _REF[None])
        self.points = pts  # (n, 8, 3)
        self.weights = (self.a ** 3 / 8.0)[:, None] * jac  # (n, 8)
        self.touch_cache = {}  # (target, source, rule) -> singular-rule entry

    def centre(self, lev, cells):
        """Images of the reference centres of level-lev cells (n, 3)."""
        a = 2.0 ** (-lev)
        ref = (np.asarray(cells, dtype=np.float64).reshape(-1, 3) + 0.5) * a
        return map_points(self.kind, ref)[0]

    def touching(self, ti, si):
        """True where the closed reference cubes of leaves ti and si meet."""
        lo_t, lo_s = self.lo[ti], self.lo[si]
        hi_t, hi_s = lo_t + self.a[ti, None], lo_s + self.a[si, None]
        return np.all(np.maximum(lo_t, lo_s) <= np.minimum(hi_t, hi_s), axis=1)


def point_rule(mm, ti, si):
    """sum_g sum_g' w_g w_g' G(x_g, y_g') with the mapped 2x2x2 rules (non-touching pairs)."""
    out = np.empty(len(ti))
    for b in range(0, len(ti), 65536):
        t, s = ti[b : b + 65536], si[b : b + 65536]
        d = mm.points[t][:, :, None, :] - mm.points[s][:, None, :, :]
        r = np.sqrt(np.sum(d * d, axis=-1))
        out[b : b + 65536] = np.einsum("ng,nh,ngh->n", mm.weights[t], mm.weights[s], 1.0 / r) / (4.0 * np.pi)
    return out


def touch_entries(mm, ti, si, rule=None):
    """Entries of touching pairs by the singular rule of mapped.c (cached per mesh)."""
    rule = RULE if rule is None else rule
    rk = tuple(rule[k] for k in ("n_lam", "n_mu", "n_z", "n_s", "n_r"))
    ti = np.asarray(ti, dtype=np.int64)
    si = np.asarray(si, dtype=np.int64)
    keys = [(int(t), int(s), rk) for t, s in zip(ti, si)]
    missing = sorted({k for k in keys if k not in mm.touch_cache})
    if missing:
        mt = np.array([k[0] for k in missing], dtype=np.int64)
        ms = np.array([k[1] for k in missing], dtype=np.int64)
        gx, gw = gauss_tables()
        val = np.empty(len(missing))
        c = np.ascontiguousarray
        _clib.lib().om_touch_entries(MAPS[mm.kind], len(mt), c(mm.lo[mt]), c(mm.a[mt]), c(mm.lo[ms]), c(mm.a[ms]),
                                     *rk, gx, gw, val)
        mm.touch_cache.update(zip(missing, val))
    return np.array([mm.touch_cache[k] for k in keys])


def regular_entries(mm, ti, si, n):
    """Entries by the n^3 x n^3 tensor Gauss rule of the two mapped cubes (a high-order check)."""
    gx, gw = gauss_tables()
    ti = np.asarray(ti, dtype=np.int64)
    si = np.asarray(si, dtype=np.int64)
    out = np.empty(len(ti))
    c = np.ascontiguousarray
    _clib.lib().om_regular_entries(MAPS[mm.kind], len(ti), c(mm.lo[ti]), c(mm.a[ti]), c(mm.lo[si]), c(mm.a[si]),
                                   n, gx, gw, out)
    return out


def entries(mm, ti, si, rule=None):
    """A_{ti, si}: the singular rule where the reference cubes touch, the mapped point rule elsewhere."""
    ti = np.asarray(ti, dtype=np.int64)
    si = np.asarray(si, dtype=np.int64)
    t = mm.touching(ti, si)
    out = np.empty(len(ti))
    out[~t] = point_rule(mm, ti[~t], si[~t])
    if np.any(t):
        out[t] = touch_entries(mm, ti[t], si[t], rule)
    return out


def apply_direct(mm, f, targets=None, rule=None):
    """O1 on the mapped mesh: u_t = sum over all leaves s of A_ts f_s."""
    n = len(mm.leaves)
    f = np.asarray(f, dtype=np.float64)
    targets = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    u = np.empty(len(targets))
    step = max(1, 262144 // n)
    for b in range(0, len(targets), step):
        tg = targets[b : b + step]
        vals = entries(mm, np.repeat(tg, n), np.tile(np.arange(n), len(tg)), rule).reshape(len(tg), n)
        u[b : b + step] = vals @ f
    return u


def matrix(mm, rule=None):
    """The dense Galerkin matrix (small meshes only)."""
    n = len(mm.leaves)
    ti = np.repeat(np.arange(n), n)
    si = np.tile(np.arange(n), n)
    return entries(mm, ti, si, rule).reshape(n, n)


_SHIFT = {}


def _shift_structure(q):
    """(rows b, columns g, C(b, g), position of b - g) over the pairs g <= b, |b| <= q."""
    if q not in _SHIFT:
        mis = multi_indices(q)
        pos = {e: n for n, e in enumerate(mis)}
        rows, cols, coef, ex = [], [], [], []
        for ib, be in enumerate(mis):
            for ig, ga in enumerate(mis):
                if all(ga[i] <= be[i] for i in range(3)):
                    rows.append(ib)
                    cols.append(ig)
                    coef.append(mi_binom(be, ga))
                    ex.append(pos[(be[0] - ga[0], be[1] - ga[1], be[2] - ga[2])])
        _SHIFT[q] = tuple(np.array(v) for v in (rows, cols, coef, ex))
    return _SHIFT[q]


def shift_matrices(d, q):
    """M(d)[b, g] = C(b, g) d^(b - g) for g <= b (moments about x_parent from moments about
    x_parent + d); L2L is its transpose. d: (n, 3); returns (n, K, K)."""
    rows, cols, coef, ex = _shift_structure(q)
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    mono = monomials(d, q)
    K = n_coeffs(q)
    M = np.zeros((len(d), K, K))
    M[:, rows, cols] = coef[None, :] * mono[:, ex]
    return M


class MappedFMM:
    """Algorithm 1 on a mapped mesh, phase by phase in FP64 (fixed order q)."""

    def __init__(self, mm, q, rule=None):
        self.mm = mm
        self.mesh = mm.mesh
        self.q = q
        self.K = n_coeffs(q)
        self.rule = rule
        mesh = self.mesh
        self.centres = [self.mm.centre(lev, mesh.levels[lev]) for lev in range(mesh.L + 1)]
        self._rows = []
        for lev in range(mesh.L + 1):
            pos, idx = [], []
            for p, c in enumerate(mesh.levels[lev]):
                key = (lev, *c)
                if key in mesh.leaf_index:
                    pos.append(p)
                    idx.append(mesh.leaf_index[key])
            self._rows.append((np.array(pos, dtype=np.int64), np.array(idx, dtype=np.int64)))

    def _leaf_moment_rows(self, lev, pos, idx):
        """sum_g w_g (x_g - x_w)^b for the given leaves (n, K)."""
        c = self.centres[lev][pos]
        mono = monomials(self.mm.points[idx] - c[:, None, :], self.q)  # (n, 8, K)
        return np.einsum("ng,ngk->nk", self.mm.weights[idx], mono)

    def _children(self, lev):
        mesh = self.mesh
        par = [p for p, c in enumerate(mesh.levels[lev]) if mesh.is_refined(lev, c)]
        kids = []
        for p in par:
            c = mesh.levels[lev][p]
            kids.append([mesh.index[lev + 1][(2 * c[0] + d[0], 2 * c[1] + d[1], 2 * c[2] + d[2])] for d in _CHILD_POS])
        return np.array(par, dtype=np.int64), np.array(kids, dtype=np.int64).reshape(-1, 8)

    # -- Algorithm 1 phases --------------------------------------------------------------------
    def near_field(self, f, targets):
        mesh = self.mesh
        ti, si = [], []
        for n, t in enumerate(targets):
            lev, i, j, k = mesh.leaves[t]
            for s in mesh.near_leaf_sources(lev, (i, j, k)):
                ti.append(n)
                si.append(mesh.leaf_index[s])
        ti = np.array(ti, dtype=np.int64)
        si = np.array(si, dtype=np.int64)
        vals = entries(self.mm, np.asarray(targets, dtype=np.int64)[ti], si, self.rule)
        return np.bincount(ti, weights=vals * f[si], minlength=len(targets))

    def moments(self, f):
        mesh = self.mesh
        m = [np.zeros((len(mesh.levels[lev]), self.K)) for lev in range(mesh.L + 1)]
        for lev, (pos, idx) in enumerate(self._rows):
            if len(pos):
                m[lev][pos] = self._leaf_moment_rows(lev, pos, idx) * f[idx][:, None]
        return m

    def upward(self, m):
        for lev in range(self.mesh.L - 1, -1, -1):
            par, kids = self._children(lev)
            if len(par) == 0:
                continue
            for k in range(8):
                d = self.centres[lev + 1][kids[:, k]] - self.centres[lev][par]
                m[lev][par] += np.einsum("nbg,ng->nb", shift_matrices(d, self.q), m[lev + 1][kids[:, k]])
        return m

    def _pairs(self, lev):
        mesh = self.mesh
        idx = mesh.index[lev]
        tp, sp = [], []
        for p, c in enumerate(mesh.levels[lev]):
            for s in mesh.interaction_list(lev, c):
                tp.append(p)
                sp.append(idx[s])
        return np.array(tp, dtype=np.int64), np.array(sp, dtype=np.int64)

    def interaction(self, m, chunk=4096):
        mesh = self.mesh
        lam = [np.zeros((len(mesh.levels[lev]), self.K)) for lev in range(mesh.L + 1)]
        for lev in range(mesh.L + 1):
            tp, sp = self._pairs(lev)
            for b in range(0, len(tp), chunk):
                t, s = tp[b : b + chunk], sp[b : b + chunk]
                T = m2l_matrix(self.centres[lev][t] - self.centres[lev][s], self.q)
                np.add.at(lam[lev], t, np.einsum("nab,nb->na", T, m[lev][s]))
        return lam

    def downward(self, lam):
        for lev in range(self.mesh.L):
            par, kids = self._children(lev)
            if len(par) == 0:
                continue
            for k in range(8):
                d = self.centres[lev + 1][kids[:, k]] - self.centres[lev][par]
                lam[lev + 1][kids[:, k]] += np.einsum("nbg,nb->ng", shift_matrices(d, self.q), lam[lev][par])
        return lam

    def evaluation(self, lam, u):
        for lev, (pos, idx) in enumerate(self._rows):
            if len(pos):
                u[idx] += np.sum(self._leaf_moment_rows(lev, pos, idx) * lam[lev][pos], axis=1)
        return u

    def apply(self, f):
        f = np.asarray(f, dtype=np.float64)
        u = self.near_field(f, np.arange(len(self.mm.leaves)))
        m = self.upward(self.moments(f))
        lam = self.downward(self.interaction(m))
        return self.evaluation(lam, u)

    # -- sampled targets ---------------------------------------------------------------------
    def _local_chain(self, lev, c, m, memo):
        key = (lev, c)
        if key in memo:
            return memo[key]
        mesh = self.mesh
        idx = mesh.index[lev]
        p = idx[c]
        srcs = [idx[s] for s in mesh.interaction_list(lev, c)]
        lam = np.zeros(self.K)
        if srcs:
            T = m2l_matrix(self.centres[lev][p] - self.centres[lev][srcs], self.q)
            lam += np.einsum("nab,nb->a", T, m[lev][srcs])
        if lev > 0:
            par = (c[0] >> 1, c[1] >> 1, c[2] >> 1)
            d = self.centres[lev][p] - self.centres[lev - 1][mesh.index[lev - 1][par]]
            lam = lam + shift_matrices(d, self.q)[0].T @ self._local_chain(lev - 1, par, m, memo)
        memo[key] = lam
        return lam

    def apply_sampled(self, f, targets):
        f = np.asarray(f, dtype=np.float64)
        targets = np.asarray(targets, dtype=np.int64)
        u = self.near_field(f, targets)
        m = self.upward(self.moments(f))
        memo = {}
        for n, t in enumerate(targets):
            lev, i, j, k = self.mesh.leaves[t]
            lam = self._local_chain(lev, (i, j, k), m, memo)
            p = self.mesh.index[lev][(i, j, k)]
            row = self._leaf_moment_rows(lev, np.array([p]), np.array([t]))[0]
            u[n] += float(row @ lam)
        return u


def ball_potential(x, radius=0.5, centre=(0.5, 0.5, 0.5)):
    """Newton potential of the uniform unit-density ball with G = 1/(4 pi |x - y|): inside,
    R^2/2 - r^2/6 (a textbook closed form)."""
    r2 = np.sum((np.asarray(x) - np.asarray(centre)) ** 2, axis=-1)
    return radius ** 2 / 2.0 - r2 / 6.0
