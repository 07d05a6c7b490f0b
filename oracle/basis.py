"""Degree-p leaf bases for the VtV potential: O1 and O2 with polynomial leaf spaces (test
infrastructure only).

The paper's finite element space (Sec. 1.2, eq. def:femspace:volume) carries polynomials of
degree p_w on each leaf, and its approximation analysis (Sec. 4, approximation errors) takes
p_l = L - l on the leaves of level l, degree p on the finest level (p = 0 in its experiments,
Sec. 5). Readings used here, for cube leaves:

  * basis: on a leaf w of level l, side a, centre c, the Legendre tensor polynomials
        phi^alpha_w(x) = prod_i P_{alpha_i}(2 (x_i - c_i) / a),   |alpha| <= p_w,
    which are orthogonal on w, with phi^0 the indicator of w, so degree 0 is the p = 0 operator
    (the paper's orthonormal basis differs by the diagonal factors |w| / prod_i (2 alpha_i + 1));
  * degrees: p_w = L - l on every leaf (level-L leaves get degree 0); order of the alpha within a
    leaf: total degree 0..p, then alpha_x descending, then alpha_y descending;
  * density f_h = sum_w sum_alpha f_{alpha,w} phi^alpha_w, output u_{alpha,w} = <phi^alpha_w, N f_h>;
  * entries A[(w,alpha),(lam,beta)] = int_w int_lam phi^alpha_w(x) G(x - y) phi^beta_lam(y) dy dx:
    exact when the closed cubes intersect (oracle.touching.box_pair_poly), otherwise the tensor
    Gauss-Legendre rule with n_w = p_w + 2 points per axis on w and n_lam on lam (on the finest
    level the 2x2x2 rule; on coarser levels the rule of the level-raised near field);
  * FMM (Algorithm 1): the moments m^gamma = int (y - c)^gamma f_h(y) dy and the evaluation
    int phi^alpha (x - c)^beta dx use the leaf's own rule; every other phase is unchanged, so
    O2 tends to O1 as q grows.

Coefficient vectors are flat, leaf-major: leaf w's n_p(p_w) coefficients at offsets[w] .. offsets[w+1].
"""

import numpy as np

from . import _clib, fmm, touching
from .taylor import monomials

FOUR_PI = 4.0 * np.pi


def basis_indices(p):
    """Multi-indices of total degree <= p in the leaf's coefficient order."""
    out = []
    for d in range(p + 1):
        for i in range(d, -1, -1):
            for j in range(d - i, -1, -1):
                out.append((i, j, d - i - j))
    return out


def n_basis(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def leaf_degrees(leaves, L):
    """p_w = L - level of every leaf."""
    lev = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)[:, 0]
    return (L - lev).astype(np.int64)


def offsets(degrees):
    """Leaf-major coefficient offsets (n_leaves + 1,)."""
    return np.concatenate([[0], np.cumsum([n_basis(int(p)) for p in degrees])]).astype(np.int64)


def _rule01(n):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def leaf_points(lo, a, p):
    """Gauss points (n^3, 3), weights (n^3,) and basis values (n^3, n_basis(p)) of one leaf with
    the (p + 2)-point rule per axis."""
    t, w = _rule01(p + 2)
    X = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).ravel() * a ** 3
    P = touching.legendre_table(2.0 * X - 1.0, p)  # (p+1, n^3, 3)
    Phi = np.stack([P[i, :, 0] * P[j, :, 1] * P[k, :, 2] for i, j, k in basis_indices(p)], axis=1)
    return np.asarray(lo, dtype=np.float64) + a * X, W, Phi


def _select(full, pa, pb):
    """Rows/columns of a [ax, ay, az, bx, by, bz] tensor in the leaf coefficient order."""
    ia = basis_indices(pa)
    ib = basis_indices(pb)
    A = np.array([[full[a + b] for b in ib] for a in ia])
    return A


def _point_potential(X, Y, q):
    """v(x_g) = sum_h q_h / |x_g - y_h| (plain C loop, oracle/o1.c)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.empty(len(X))
    _clib.lib().o1_point_potential(len(X), X, len(Y), Y, q, out)
    return out


_TOUCH = {}


def touching_block(lo_int_t, size_t, lo_int_s, size_s, a_small, p_t, p_s):
    """Exact block (n_basis(p_t), n_basis(p_s)) of a touching pair, including 1/(4 pi).

    Geometry in integer units of the smaller side; the block of the unit-scale pair is cached per
    configuration and scales with a_small^5."""
    small = min(size_t, size_s)
    key = (tuple((np.asarray(lo_int_s) - np.asarray(lo_int_t)) // small), size_t // small, size_s // small, p_t, p_s)
    if key not in _TOUCH:
        off = np.array(key[0], dtype=np.float64)
        st, ss = float(key[1]), float(key[2])
        full = touching.box_pair_poly(np.zeros(3), np.full(3, st), off, off + ss, p_t, p_s)
        _TOUCH[key] = _select(full, p_t, p_s)
    return _TOUCH[key] * a_small ** 5 / FOUR_PI


class Leaves:
    """Geometry, degrees, rules and coefficient offsets of a mesh's leaves (degree_zero: every
    leaf degree 0 with the 2x2x2 rule, the p = 0 operator of oracle.direct)."""

    def __init__(self, mesh, degree_zero=False):
        self.mesh = mesh
        self.lv = mesh.leaf_array()
        self.L = mesh.L
        self.size = np.left_shift(1, self.L - self.lv[:, 0])  # integer side at level-L resolution
        self.lo_int = self.lv[:, 1:4] * self.size[:, None]
        self.a = np.ldexp(1.0, -self.lv[:, 0].astype(np.int32))
        self.lo = self.lv[:, 1:4] * self.a[:, None]
        self.p = np.zeros(len(self.lv), dtype=np.int64) if degree_zero else leaf_degrees(self.lv, self.L)
        self.off = offsets(self.p)
        self._pts = {}

    def points(self, w):
        if w not in self._pts:
            self._pts[w] = leaf_points(self.lo[w], self.a[w], int(self.p[w]))
        return self._pts[w]

    def touches(self, t, s):
        lo = np.maximum(self.lo_int[t], self.lo_int[s])
        hi = np.minimum(self.lo_int[t] + self.size[t], self.lo_int[s] + self.size[s])
        return bool(np.all(lo <= hi))

    def block(self, t, s):
        """Entry block A[(t, .), (s, .)]: exact if touching, else the two leaves' Gauss rules."""
        if self.touches(t, s):
            return touching_block(self.lo_int[t], int(self.size[t]), self.lo_int[s], int(self.size[s]),
                                  min(self.a[t], self.a[s]), int(self.p[t]), int(self.p[s]))
        X, WX, PX = self.points(t)
        Y, WY, PY = self.points(s)
        K = 1.0 / np.sqrt(((X[:, None, :] - Y[None, :, :]) ** 2).sum(axis=2))
        return (PX * WX[:, None]).T @ K @ (PY * WY[:, None]) / FOUR_PI


def apply_direct(mesh, F, targets=None, degree_zero=False):
    """O1: u_t = sum over ALL leaves s of A[t, s] F_s for the target leaves (default all), as a flat
    vector of the targets' coefficients in target order. Non-touching sources enter through their
    densities at their Gauss points (identical to the entry blocks of Leaves.block)."""
    lf = Leaves(mesh, degree_zero)
    n = len(lf.lv)
    F = np.asarray(F, dtype=np.float64)
    targets = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    ys, qs, owner = [], [], []
    for s in range(n):
        Y, WY, PY = lf.points(s)
        ys.append(Y)
        qs.append(WY * (PY @ F[lf.off[s] : lf.off[s + 1]]))
        owner.append(np.full(len(Y), s))
    Y = np.concatenate(ys)
    q = np.concatenate(qs)
    owner = np.concatenate(owner)
    out = []
    for t in targets:
        X, WX, PX = lf.points(t)
        lo = np.maximum(lf.lo_int[t], lf.lo_int)
        hi = np.minimum(lf.lo_int[t] + lf.size[t], lf.lo_int + lf.size[:, None])
        tch = np.all(lo <= hi, axis=1)  # closed cubes intersect
        far_pts = ~tch[owner]
        v = _point_potential(X, Y[far_pts], q[far_pts]) / FOUR_PI
        u = PX.T @ (WX * v)
        for s in np.nonzero(tch)[0]:
            u = u + lf.block(t, s) @ F[lf.off[s] : lf.off[s + 1]]
        out.append(u)
    return np.concatenate(out) if out else np.zeros(0)


class BasisFMM(fmm.FMM):
    """O2 with degree-p leaf bases: Algorithm 1 with the leaf spaces above; the passes and the
    interaction phase are those of oracle.fmm (fixed order q, or with q_schedule = 1 the
    level-dependent orders q_l = q + L - l: the paper's experiment takes both p_l = L - l and
    q_l = 4 + L - l, Sec. 5)."""

    def __init__(self, mesh, q, degree_zero=False, q_schedule=0):
        super().__init__(mesh, q, q_schedule=q_schedule)
        self.lf = Leaves(mesh, degree_zero)

    def near_field_basis(self, F, targets):
        """Near-field coefficients of the targets: sum over the extended neighbour list (marked
        neighbours expanded to their leaves) of the entry blocks times F. The non-touching sources
        enter through their densities at their Gauss points, q_h = W_h f_h(y_h), so that the sum of
        their blocks is Phi_t^T (W_t * sum_s K(x, y_s) q_s) (the same products, associated
        differently); touching sources use their exact blocks."""
        lf = self.lf
        mesh = self.mesh
        out = []
        for t in targets:
            lev, i, j, k = mesh.leaves[t]
            src = np.array([mesh.leaf_index[s] for s in mesh.near_leaf_sources(lev, (i, j, k))], dtype=np.int64)
            lo = np.maximum(lf.lo_int[t], lf.lo_int[src])
            hi = np.minimum(lf.lo_int[t] + lf.size[t], lf.lo_int[src] + lf.size[src][:, None])
            tch = np.all(lo <= hi, axis=1)
            X, WX, PX = lf.points(t)
            far = src[~tch]
            ys, qs = [], []
            for p in np.unique(lf.p[far]):
                grp = far[lf.p[far] == p]
                Yr, Wr, Pr = leaf_points(np.zeros(3), 1.0, int(p))  # reference points of the unit cube
                a = lf.a[grp]
                ys.append((lf.lo[grp][:, None, :] + a[:, None, None] * Yr[None]).reshape(-1, 3))
                Fs = np.stack([F[lf.off[s] : lf.off[s + 1]] for s in grp])  # (n, nb)
                qs.append(((Fs @ Pr.T) * Wr[None, :] * (a ** 3)[:, None]).ravel())
            v = _point_potential(X, np.concatenate(ys), np.concatenate(qs)) if ys else np.zeros(len(X))
            u = PX.T @ (WX * v) / FOUR_PI
            for s in src[tch]:
                u = u + lf.block(t, s) @ F[lf.off[s] : lf.off[s + 1]]
            out.append(u)
        return out

    def moments_basis(self, F):
        """m^gamma of every leaf with the leaf's rule: sum_g w_g (y_g - c)^gamma f_h(y_g), level by
        level (the leaves of a level share their degree and rule)."""
        mesh = self.mesh
        lf = self.lf
        m = [np.zeros((len(mesh.levels[lev]), self.K_of[lev])) for lev in range(mesh.L + 1)]
        for lev, (pos, idx) in enumerate(self._rows):
            if len(pos) == 0:
                continue
            p = int(lf.p[idx[0]])
            a = float(lf.a[idx[0]])
            Yr, Wr, Pr = leaf_points(np.zeros(3), 1.0, p)
            Fs = np.stack([F[lf.off[w] : lf.off[w + 1]] for w in idx])  # (n, nb)
            vals = (Fs @ Pr.T) * Wr[None, :] * a ** 3  # (n, P): w_g f_h(y_g)
            m[lev][pos] = vals @ monomials(a * (Yr - 0.5), self.q_of[lev])
        return m

    def _evaluate(self, w, lam_w):
        """int phi^alpha(x) sum_beta lam^beta (x - c)^beta dx with the leaf's rule."""
        lf = self.lf
        lev = int(lf.lv[w, 0])
        X, WX, PX = lf.points(w)
        centre = lf.lo[w] + 0.5 * lf.a[w]
        return PX.T @ (WX * (monomials(X - centre, self.q_of[lev]) @ lam_w))

    def apply_basis(self, F):
        F = np.asarray(F, dtype=np.float64)
        lf = self.lf
        u = np.concatenate(self.near_field_basis(F, range(len(lf.lv))))
        m = self.upward(self.moments_basis(F))
        lam = self.downward(self.interaction(m))
        for w in range(len(lf.lv)):
            lev = int(lf.lv[w, 0])
            row = self.mesh.index[lev][tuple(lf.lv[w, 1:])]
            u[lf.off[w] : lf.off[w + 1]] += self._evaluate(w, lam[lev][row])
        return u

    def apply_basis_sampled(self, F, targets):
        """The targets' coefficients only (flat, in target order)."""
        F = np.asarray(F, dtype=np.float64)
        lf = self.lf
        near = self.near_field_basis(F, targets)
        m = self.upward(self.moments_basis(F))
        memo = {}
        out = []
        for n, t in enumerate(targets):
            lev, i, j, k = self.mesh.leaves[t]
            lam = self._local_chain(lev, (i, j, k), m, memo)
            out.append(near[n] + self._evaluate(int(t), lam))
        return np.concatenate(out)


def project(mesh, func, n=None):
    """Coefficients of the L2 projection of func onto the leaf spaces: f_alpha = <phi^alpha, func> /
    ||phi^alpha||^2, ||phi^alpha||^2 = |w| / prod_i (2 alpha_i + 1), by a Gauss rule of n points per
    axis (default p_w + 4)."""
    lf = Leaves(mesh)
    out = np.empty(lf.off[-1])
    for w in range(len(lf.lv)):
        p = int(lf.p[w])
        m = n if n is not None else p + 4
        t, wt = _rule01(m)
        X = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
        W = np.einsum("i,j,k->ijk", wt, wt, wt).ravel()
        P = touching.legendre_table(2.0 * X - 1.0, p)
        vals = func(lf.lo[w] + lf.a[w] * X)
        for r, (i, j, k) in enumerate(basis_indices(p)):
            phi = P[i, :, 0] * P[j, :, 1] * P[k, :, 2]
            out[lf.off[w] + r] = np.sum(W * phi * vals) * (2 * i + 1) * (2 * j + 1) * (2 * k + 1)
    return out
