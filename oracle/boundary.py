"""BtV: boundary-to-volume potentials on the BC cube mesh (test infrastructure only).

What is computed (Sec. 1 for the layer potentials, Algorithm 3 for the FMM; degree p = 0 and
the indicator basis on the volume leaves, as for the VtV oracle):

  u_w = <1_w, V[q] - K[g]>_{L2(w)},
  V[q](x) = int_Gamma G(x - y) q(y) dS_y,   K[g](x) = int_Gamma dG(x - y)/dn_y g(y) dS_y,

with G = 1/(4 pi |x - y|), Gamma the boundary of the unit cube with its outward normal n, and
q (the Neumann trace gamma_1 u) and g (the Dirichlet trace gamma_0 u) constant on each
boundary face. For harmonic u, Green's representation formula gives u = V[du/dn] - K[u] in the
domain, which is what the BtV calculation evaluates.

Boundary faces: every cell that meets Gamma has a face on it (a closed cube inside the unit
cube that meets a face plane has its own face in that plane), so every such cell is marked
and refined down to level L: the boundary faces are the faces of level-L leaves that lie on
Gamma. A face is (leaf, axis, side): the leaf's face normal to `axis` on its low (side 0) or
high (side 1) end, outward normal (2 side - 1) e_axis.

Entries, for a volume leaf w and a boundary face f:

  V_wf = int_w int_f G(x - y) dS_y dx,   K_wf = int_w int_f n_f . (x - y) / (4 pi |x - y|^3) dS_y dx
  (dG(x - y)/dn_y = n . grad_y G(x - y) = n . (x - y) / (4 pi |x - y|^3)).

If the closed cell and the closed face meet, the entries are computed exactly (to quadrature
accuracy) by the same convolution reduction as the cube pairs of oracle.touching, with the
face a box of zero thickness: int_w int_f k(x - y) dS_y dx = int_{R^3} prod_i c_i(u_i) k(u) du,
where along the face's normal axis c(u) is the indicator of [w_lo - f, w_hi - f] and along the
other axes the overlap length of the two intervals. Otherwise the 2x2x2 Gauss points of the
cell and the 2x2 Gauss points of the face give the point rule.

O1 (`apply_direct`) sums the entries over all faces; O2 (`BtVFMM`) follows Algorithm 3:
near field over the faces whose level-l ancestor cell is a neighbour of the target leaf (l the
target's level), moments of the boundary cells from their faces (2x2 point rule, so that O2
tends to O1 as q grows), upward pass over the marked cells, interaction phase with sources
restricted to the boundary cells B_l, downward pass and evaluation as in Algorithm 1.
"""

import numpy as np

from .fmm import FMM
from .taylor import multi_indices, n_coeffs

_XI = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))  # 2-point Gauss nodes on [0, 1]


def boundary_faces(mesh):
    """(leaf index, axis, side) of every boundary face, ordered by leaf index, then axis, side."""
    n = 1 << mesh.L
    out = []
    for t, (lev, i, j, k) in enumerate(mesh.leaf_array()):
        if lev != mesh.L:
            continue
        c = (i, j, k)
        for ax in range(3):
            for side in (0, 1):
                if (side == 0 and c[ax] == 0) or (side == 1 and c[ax] == n - 1):
                    out.append((t, ax, side))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def face_box(lo, a, ax, side):
    """Lower and upper corner of a face of the cube [lo, lo + a]; zero extent along ax."""
    flo = np.array(lo, dtype=np.float64)
    fhi = flo + a
    flo[ax] = fhi[ax] = lo[ax] + side * a
    return flo, fhi


# -- exact entries: convolution reduction ----------------------------------------------------------

def _gauss01(n):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def _factor(u, ax, wlo, whi, flo, fhi, normal_axis):
    """c_ax(u): overlap length of [wlo, whi] and [flo + u, fhi + u], or along the face normal
    the indicator of wlo <= f + u <= whi."""
    if ax == normal_axis:
        return ((u >= wlo[ax] - flo[ax]) & (u <= whi[ax] - flo[ax])).astype(np.float64)
    return np.maximum(0.0, np.minimum(whi[ax], fhi[ax] + u) - np.maximum(wlo[ax], flo[ax] + u))


def _breaks(ax, wlo, whi, flo, fhi, normal_axis):
    if ax == normal_axis:
        lo, hi = wlo[ax] - flo[ax], whi[ax] - flo[ax]
        pts = {lo, hi}
    else:
        lo, hi = wlo[ax] - fhi[ax], whi[ax] - flo[ax]
        pts = {lo, hi, wlo[ax] - flo[ax], whi[ax] - fhi[ax]}
    if lo < 0.0 < hi:
        pts.add(0.0)
    return sorted(pts)


def _kernel(u, kind, normal_axis, sign):
    """k(u) times 4 pi: 1/|u| (single layer) or n . u / |u|^3 (double layer), u = x - y."""
    r = np.linalg.norm(u, axis=-1)
    if kind == "single":
        return 1.0 / r
    return sign * u[..., normal_axis] / r ** 3


def cell_face_integral(wlo, whi, flo, fhi, normal_axis, sign, kind, n=24):
    """int_w int_f k(x - y) dS_y dx for the box w = [wlo, whi] and the face f = [flo, fhi]
    (zero extent along normal_axis, outward normal sign * e_normal_axis); k = G (kind
    "single") or dG/dn_y (kind "double")."""
    wlo, whi, flo, fhi = (np.asarray(v, dtype=np.float64) for v in (wlo, whi, flo, fhi))
    br = [_breaks(ax, wlo, whi, flo, fhi, normal_axis) for ax in range(3)]
    g, gw = _gauss01(n)
    total = 0.0
    for ix in range(len(br[0]) - 1):
        for iy in range(len(br[1]) - 1):
            for iz in range(len(br[2]) - 1):
                lo = np.array([br[0][ix], br[1][iy], br[2][iz]])
                hi = np.array([br[0][ix + 1], br[1][iy + 1], br[2][iz + 1]])
                total += _sub_box(lo, hi, wlo, whi, flo, fhi, normal_axis, sign, kind, g, gw)
    return total / (4.0 * np.pi)


def _numerator(u, wlo, whi, flo, fhi, normal_axis):
    out = np.ones(u.shape[:-1])
    for ax in range(3):
        out = out * _factor(u[..., ax], ax, wlo, whi, flo, fhi, normal_axis)
    return out


def _sub_box(lo, hi, wlo, whi, flo, fhi, normal_axis, sign, kind, g, gw):
    h = hi - lo
    if np.any(h <= 0.0):
        return 0.0
    corner_at_origin = all(lo[i] == 0.0 or hi[i] == 0.0 for i in range(3))
    W3 = np.einsum("i,j,k->ijk", gw, gw, gw)
    if not corner_at_origin:
        X, Y, Z = np.meshgrid(lo[0] + h[0] * g, lo[1] + h[1] * g, lo[2] + h[2] * g, indexing="ij")
        u = np.stack([X, Y, Z], axis=-1)
        f = _numerator(u, wlo, whi, flo, fhi, normal_axis) * _kernel(u, kind, normal_axis, sign)
        return float(np.sum(W3 * f)) * h[0] * h[1] * h[2]
    # The origin is a corner: u = sigma * v, v in [0, h]^3, three Duffy pyramids (Duffy 1982):
    # v_k = h_k t, v_j = h_j t s_j; the Jacobian h1 h2 h3 t^2 cancels the kernel's singularity
    # (1/|u| ~ 1/t, n.u/|u|^3 ~ 1/t^2), so the kernel times t^2 is evaluated at uhat = u / t.
    sigma = np.array([1.0 if lo[i] == 0.0 else -1.0 for i in range(3)])
    T, S1, S2 = np.meshgrid(g, g, g, indexing="ij")
    total = 0.0
    for kax in range(3):
        others = [j for j in range(3) if j != kax]
        uhat = np.empty(T.shape + (3,))
        uhat[..., kax] = h[kax]
        uhat[..., others[0]] = h[others[0]] * S1
        uhat[..., others[1]] = h[others[1]] * S2
        uhat = uhat * sigma
        u = uhat * T[..., None]
        if kind == "single":
            scaled = T / np.linalg.norm(uhat, axis=-1)
        else:
            scaled = sign * uhat[..., normal_axis] / np.linalg.norm(uhat, axis=-1) ** 3
        f = _numerator(u, wlo, whi, flo, fhi, normal_axis) * scaled
        total += float(np.sum(W3 * f)) * h[0] * h[1] * h[2]
    return total


# -- point rule ------------------------------------------------------------------------------------

def cell_points(lo, a):
    """2x2x2 Gauss points (8, 3) of the cube [lo, lo + a] and their common weight a^3 / 8."""
    lo = np.asarray(lo, dtype=np.float64)
    pts = np.array([[lo[0] + a * _XI[i], lo[1] + a * _XI[j], lo[2] + a * _XI[k]]
                    for k in (0, 1) for j in (0, 1) for i in (0, 1)])
    return pts, a ** 3 / 8.0


def face_points(lo, a, ax, side):
    """2x2 Gauss points (4, 3) of a face of the cube [lo, lo + a] and their weight a^2 / 4."""
    lo = np.asarray(lo, dtype=np.float64)
    others = [d for d in range(3) if d != ax]
    pts = []
    for j in (0, 1):
        for i in (0, 1):
            p = lo.copy()
            p[ax] = lo[ax] + side * a
            p[others[0]] = lo[others[0]] + a * _XI[i]
            p[others[1]] = lo[others[1]] + a * _XI[j]
            pts.append(p)
    return np.array(pts), a * a / 4.0


def point_rule(wlo, wa, flo, fa, ax, side):
    """(V, K) of a cell and a face by the 2x2x2 x 2x2 point rule."""
    xp, wx = cell_points(wlo, wa)
    yp, wy = face_points(flo, fa, ax, side)
    d = xp[:, None, :] - yp[None, :, :]
    r = np.linalg.norm(d, axis=-1)
    sign = 2.0 * side - 1.0
    V = wx * wy * np.sum(1.0 / r) / (4.0 * np.pi)
    K = wx * wy * np.sum(sign * d[..., ax] / r ** 3) / (4.0 * np.pi)
    return V, K


# -- entries ----------------------------------------------------------------------------------------

class Entries:
    """V_wf and K_wf for (volume leaf, boundary face) pairs of one mesh, exact where the closed
    cell and face meet (cached by their relative position), point rule elsewhere."""

    def __init__(self, mesh, n=24):
        self.mesh = mesh
        self.L = mesh.L
        self.leaves = mesh.leaf_array()
        self.faces = boundary_faces(mesh)
        self.n = n
        self._exact = {}

    def _leaf_int(self, t):
        lev, i, j, k = self.leaves[t]
        s = 1 << (self.L - lev)
        return np.array([i * s, j * s, k * s], dtype=np.int64), s

    def touches(self, t, f):
        lo, s = self._leaf_int(t)
        leaf, ax, side = self.faces[f]
        flo, fs = self._leaf_int(leaf)
        fl = flo.copy()
        fh = flo + fs
        fl[ax] = fh[ax] = flo[ax] + side * fs
        return bool(np.all(np.maximum(lo, fl) <= np.minimum(lo + s, fh)))

    def exact(self, t, f):
        """Exact (V, K) of leaf t and face f, from the cache keyed by relative integer geometry."""
        lo, s = self._leaf_int(t)
        leaf, ax, side = self.faces[f]
        flo, fs = self._leaf_int(leaf)
        key = (tuple(flo - lo), int(s), int(fs), int(ax), int(side))
        if key not in self._exact:
            unit = 1.0  # integer units; scaled below (V ~ length^4, K ~ length^3)
            wlo, whi = np.zeros(3), np.full(3, float(s)) * unit
            fl, fh = face_box((flo - lo).astype(np.float64), float(fs), ax, side)
            sign = 2.0 * side - 1.0
            V = cell_face_integral(wlo, whi, fl, fh, ax, sign, "single", self.n)
            K = cell_face_integral(wlo, whi, fl, fh, ax, sign, "double", self.n)
            self._exact[key] = (V, K)
        h = np.ldexp(1.0, -self.L)
        V, K = self._exact[key]
        return V * h ** 4, K * h ** 3

    def entry(self, t, f):
        if self.touches(t, f):
            return self.exact(t, f)
        lev, i, j, k = self.leaves[t]
        a = np.ldexp(1.0, -int(lev))
        leaf, ax, side = self.faces[f]
        fl, fi, fj, fk = self.leaves[leaf]
        fa = np.ldexp(1.0, -int(fl))
        return point_rule(np.array([i, j, k]) * a, a, np.array([fi, fj, fk]) * fa, fa, ax, side)


def apply_direct(mesh, qf, gf, targets=None, n=24):
    """O1: u_w = sum over all boundary faces f of V_wf q_f - K_wf g_f."""
    E = Entries(mesh, n)
    qf = np.asarray(qf, dtype=np.float64)
    gf = np.asarray(gf, dtype=np.float64)
    targets = np.arange(len(E.leaves)) if targets is None else np.asarray(targets)
    u = np.zeros(len(targets))
    for m, t in enumerate(targets):
        for f in range(len(E.faces)):
            V, K = E.entry(t, f)
            u[m] += V * qf[f] - K * gf[f]
    return u


def apply_direct_sampled(mesh, qf, gf, targets, n=24):
    """O1 at the given target leaves only, with the point rule vectorised over all faces (same
    entries as apply_direct)."""
    E = Entries(mesh, n)
    L = mesh.L
    qf = np.asarray(qf, dtype=np.float64)
    gf = np.asarray(gf, dtype=np.float64)
    lv = E.leaves
    fa = np.ldexp(1.0, -L)
    fleaf = lv[E.faces[:, 0]]
    flo = fleaf[:, 1:4] * fa
    ax, side = E.faces[:, 1], E.faces[:, 2]
    others = np.stack([(ax + 1) % 3, (ax + 2) % 3], axis=1)
    # 2x2 face points (nf, 4, 3)
    fp = np.repeat(flo[:, None, :], 4, axis=1)
    rows = np.arange(len(flo))
    fp[rows, :, ax] += (side * fa)[:, None]
    for m, (i, j) in enumerate([(0, 0), (1, 0), (0, 1), (1, 1)]):
        fp[rows, m, others[:, 0]] += fa * _XI[i]
        fp[rows, m, others[:, 1]] += fa * _XI[j]
    sign = 2.0 * side - 1.0
    out = np.zeros(len(targets))
    for m, t in enumerate(targets):
        lev, i, j, k = lv[t]
        a = np.ldexp(1.0, -int(lev))
        xp, wx = cell_points(np.array([i, j, k]) * a, a)
        d = xp[None, :, None, :] - fp[:, None, :, :]  # (nf, 8, 4, 3)
        r = np.linalg.norm(d, axis=-1)
        V = wx * fa * fa / 4.0 * np.sum(1.0 / r, axis=(1, 2)) / (4.0 * np.pi)
        dn = np.take_along_axis(d, ax[:, None, None, None], axis=-1)[..., 0]
        K = wx * fa * fa / 4.0 * sign * np.sum(dn / r ** 3, axis=(1, 2)) / (4.0 * np.pi)
        if lev == L:  # touching pairs (closed cell and face meet): exact
            lo_t = np.array([i, j, k], dtype=np.int64)
            fl_int = fleaf[:, 1:4].astype(np.int64)
            f_lo, f_hi = fl_int.copy(), fl_int + 1
            f_lo[rows, ax] = f_hi[rows, ax] = fl_int[rows, ax] + side
            meet = np.all(np.maximum(f_lo, lo_t) <= np.minimum(f_hi, lo_t + 1), axis=1)
            for f in np.nonzero(meet)[0]:
                V[f], K[f] = E.exact(t, f)
        out[m] = V @ qf - K @ gf
    return out


# -- O2: Algorithm 3 --------------------------------------------------------------------------------

class BtVFMM(FMM):
    """Algorithm 3 (BC-FMM for the BtV calculation) step by step in FP64."""

    def __init__(self, mesh, q, n=24):
        super().__init__(mesh, q)
        self.E = Entries(mesh, n)
        self.faces = self.E.faces
        # faces in the subtree of every boundary cell, per level
        self._subtree = [dict() for _ in range(mesh.L + 1)]
        for f, (leaf, ax, side) in enumerate(self.faces):
            lev, i, j, k = self.leaves[leaf]
            for l in range(mesh.L + 1):
                c = (i >> (mesh.L - l), j >> (mesh.L - l), k >> (mesh.L - l))
                self._subtree[l].setdefault(c, []).append(f)

    def near_faces(self, t):
        """Faces f whose boundary cell's ancestor at the level of leaf t is a neighbour of t."""
        lev, i, j, k = self.leaves[t]
        out = []
        for nb in self.mesh.neighbours(lev, (i, j, k)):
            out.extend(self._subtree[lev].get(nb, []))
        return out

    def near_field(self, qf, gf, targets):
        u = np.zeros(len(targets))
        for m, t in enumerate(targets):
            for f in self.near_faces(t):
                V, K = self.E.entry(t, f)
                u[m] += V * qf[f] - K * gf[f]
        return u

    def boundary_moments(self, qf, gf):
        """m_w^a = int_{faces of w} (y - x_w)^a q - d/dn (y - x_w)^a g  (2x2 point rule), for w in B_L."""
        mesh = self.mesh
        L = mesh.L
        mis = multi_indices(self.q)
        m = [np.zeros((len(mesh.levels[lev]), self.K)) for lev in range(L + 1)]
        a = mesh.side(L)
        for f, (leaf, ax, side) in enumerate(self.faces):
            _, i, j, k = self.leaves[leaf]
            lo = np.array([i, j, k]) * a
            centre = lo + 0.5 * a
            pts, w = face_points(lo, a, ax, side)
            d = pts - centre  # (4, 3)
            sign = 2.0 * side - 1.0
            row = mesh.index[L][(int(i), int(j), int(k))]
            for n_, al in enumerate(mis):
                mono = np.prod(d ** np.array(al), axis=1)
                if al[ax] > 0:
                    e = list(al)
                    e[ax] -= 1
                    dmono = al[ax] * np.prod(d ** np.array(e), axis=1)
                else:
                    dmono = np.zeros(len(d))
                m[L][row, n_] += w * np.sum(mono * qf[f] - sign * dmono * gf[f])
        return m

    def interaction(self, m):
        """lambda_w = sum over w' in I(w) with w' in B_l of T(w, w') m_w', every cell."""
        mesh = self.mesh
        lam = [np.zeros((len(mesh.levels[lev]), self.K)) for lev in range(mesh.L + 1)]
        for lev in range(mesh.L + 1):
            groups = {}
            idx = mesh.index[lev]
            for p, c in enumerate(mesh.levels[lev]):
                for s in mesh.interaction_list(lev, c):
                    if not mesh.on_boundary(lev, s):
                        continue
                    o = (c[0] - s[0], c[1] - s[1], c[2] - s[2])
                    groups.setdefault(o, ([], []))
                    groups[o][0].append(p)
                    groups[o][1].append(idx[s])
            offsets = list(groups)
            for o, T in zip(offsets, self._m2l(lev, offsets)):
                tp = np.array(groups[o][0], dtype=np.int64)
                sp = np.array(groups[o][1], dtype=np.int64)
                lam[lev][tp] += m[lev][sp] @ T.T
        return lam

    def apply(self, qf, gf):
        qf = np.asarray(qf, dtype=np.float64)
        gf = np.asarray(gf, dtype=np.float64)
        u = self.near_field(qf, gf, np.arange(len(self.leaves)))
        m = self.upward(self.boundary_moments(qf, gf))
        lam = self.downward(self.interaction(m))
        return self.evaluation(lam, u)


# -- VtB: Algorithm 2 --------------------------------------------------------------------------------
#
# u_f = <1_f, N f_h>_{L2(f)} = sum over leaves l of V_lf f_l for every boundary face f: the
# potential's face integrals (degree p = 0 on the faces). The entries are the single-layer entries of
# the BtV calculation (G is symmetric). Algorithm 2: near field of the face's cell w (level L) over
# N*(w) as in Algorithm 1, moments of every leaf, upward pass, interaction phase for the boundary
# cells B_l, downward pass into the boundary children, evaluation of the face's cell's local
# expansion at the face (2x2 point rule).

def vtb_direct(mesh, f, n=24, face_idx=None):
    """O1: u_f = sum over all leaves l of V_lf f_l, for every face or the faces face_idx."""
    E = Entries(mesh, n)
    f = np.asarray(f, dtype=np.float64)
    face_idx = np.arange(len(E.faces)) if face_idx is None else np.asarray(face_idx)
    u = np.zeros(len(face_idx))
    for m, fi in enumerate(face_idx):
        for t in range(len(E.leaves)):
            u[m] += E.entry(t, fi)[0] * f[t]
    return u


class VtBFMM(FMM):
    """Algorithm 2 (BC-FMM for the VtB calculation) step by step in FP64."""

    def __init__(self, mesh, q, n=24):
        super().__init__(mesh, q)
        self.E = Entries(mesh, n)
        self.faces = self.E.faces

    def near_field(self, f):
        mesh = self.mesh
        u = np.zeros(len(self.faces))
        for fi, (leaf, ax, side) in enumerate(self.faces):
            lev, i, j, k = self.leaves[leaf]
            for s in mesh.near_leaf_sources(lev, (i, j, k)):
                t = mesh.leaf_index[s]
                u[fi] += self.E.entry(t, fi)[0] * f[t]
        return u

    def interaction(self, m):
        """lambda_w = sum over I(w) of T(w, w') m_w' for the boundary cells w in B_l."""
        mesh = self.mesh
        lam = [np.zeros((len(mesh.levels[lev]), self.K)) for lev in range(mesh.L + 1)]
        for lev in range(mesh.L + 1):
            idx = mesh.index[lev]
            for p, c in enumerate(mesh.levels[lev]):
                if not mesh.on_boundary(lev, c):
                    continue
                srcs = mesh.interaction_list(lev, c)
                if not srcs:
                    continue
                offs = [(c[0] - s[0], c[1] - s[1], c[2] - s[2]) for s in srcs]
                for T, s in zip(self._m2l(lev, offs), srcs):
                    lam[lev][p] += T @ m[lev][idx[s]]
        return lam

    def downward(self, lam):
        """lambda_w' += L(w', w) lambda_w for w in B_l and its children in B_{l+1}."""
        mesh = self.mesh
        for lev in range(mesh.L):
            for p, c in enumerate(mesh.levels[lev]):
                if not mesh.on_boundary(lev, c) or not mesh.is_refined(lev, c):
                    continue
                for pos in ((dx, dy, dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)):
                    ch = (2 * c[0] + pos[0], 2 * c[1] + pos[1], 2 * c[2] + pos[2])
                    if mesh.on_boundary(lev + 1, ch):
                        lam[lev + 1][mesh.index[lev + 1][ch]] += self._l2l(lev, pos) @ lam[lev][p]
        return lam

    def evaluation_faces(self, lam, u):
        """u_f += int_f sum_a lambda_w^a (y - x_w)^a dS (2x2 point rule), w the face's cell."""
        mesh = self.mesh
        L = mesh.L
        a = mesh.side(L)
        mis = multi_indices(self.q)
        for fi, (leaf, ax, side) in enumerate(self.faces):
            _, i, j, k = self.leaves[leaf]
            lo = np.array([i, j, k]) * a
            pts, w = face_points(lo, a, ax, side)
            d = pts - (lo + 0.5 * a)
            row = mesh.index[L][(int(i), int(j), int(k))]
            mono = np.array([np.prod(d ** np.array(al), axis=1) for al in mis])  # (K, 4)
            u[fi] += w * float(np.sum(mono.sum(axis=1) * lam[L][row]))
        return u

    def apply(self, f):
        f = np.asarray(f, dtype=np.float64)
        u = self.near_field(f)
        m = self.upward(self.moments(f))
        lam = self.downward(self.interaction(m))
        return self.evaluation_faces(lam, u)


def vtb_direct_sampled(mesh, f, face_idx, n=24):
    """O1 of VtB at the given faces only, with the point rule vectorised over all leaves."""
    E = Entries(mesh, n)
    f = np.asarray(f, dtype=np.float64)
    lv = E.leaves
    a = np.ldexp(1.0, -lv[:, 0].astype(np.int32))
    lo = lv[:, 1:4] * a[:, None]
    # 2x2x2 cell points (n, 8, 3)
    ref = np.array([[_XI[i], _XI[j], _XI[k]] for k in (0, 1) for j in (0, 1) for i in (0, 1)])
    cp = lo[:, None, :] + a[:, None, None] * ref[None, :, :]
    wc = a ** 3 / 8.0
    out = np.zeros(len(face_idx))
    for m_, fi in enumerate(face_idx):
        leaf, ax, side = E.faces[fi]
        fl, fi_, fj, fk = lv[leaf]
        fa = np.ldexp(1.0, -int(fl))
        fp, wf = face_points(np.array([fi_, fj, fk]) * fa, fa, ax, side)
        r = np.linalg.norm(cp[:, :, None, :] - fp[None, None, :, :], axis=-1)  # (n, 8, 4)
        V = wc * wf * np.sum(1.0 / r, axis=(1, 2)) / (4.0 * np.pi)
        # touching leaves: exact (they are level-L leaves within one cell of the face's cell)
        near = np.nonzero(np.all(np.abs(lv[:, 1:4] - lv[leaf, 1:4]) <= 1, axis=1) & (lv[:, 0] == fl))[0]
        for t in near:
            if E.touches(t, fi):
                V[t] = E.exact(t, fi)[0]
        out[m_] = V @ f
    return out
