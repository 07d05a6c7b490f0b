"""O1: the Galerkin volume potential u = A f by direct O(N^2) evaluation (test infrastructure only).

Definition (Sec. 1.2, eq. galerkin:vol with degree p = 0 and the indicator basis; Sec. 1.1 for
the Newton potential and G = 1/(4 pi |x - y|)):

  u_w = <1_w, N f_h>_{L2(Omega)} = sum_lambda A_{w lambda} f_lambda,
  A_{w lambda} = int_w int_lambda G(x, y) dy dx,

with f_h piecewise constant on the leaves. Entries of touching pairs (closed cubes
intersect) are the exact integrals of oracle.touching; entries of all other pairs use the
2x2x2 Gauss-Legendre point rule on both cells:

  A_{w lambda} ~ sum_{g in w} sum_{g' in lambda} w_g w_g' G(x_g, y_g').

Level-dependent near-field order (Sec. 4, the paragraph on the near-field Gauss rule: a fixed order
on the finest level, raised on each coarser level). Reading: a leaf of level l carries the tensor
Gauss-Legendre rule of n_l = 2 + (L - l) points per axis, and a non-touching near pair (w, lambda)
takes n_l(w)^3 points on w and n_l(lambda)^3 points on lambda (so the entry stays symmetric).
Far pairs keep the 2x2x2 rule: their entries are what the FMM's moments (2x2x2 rule) approximate.
apply_near_order() is that operator; apply(..., orders=...) applies the per-leaf rule to every
non-touching pair (the direct mode of the library, where every pair is near).
"""

import numpy as np

from . import _clib, touching

_XI = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))  # 2-point Gauss nodes on [0, 1]
_REF = np.array([[_XI[i], _XI[j], _XI[k]] for k in (0, 1) for j in (0, 1) for i in (0, 1)])  # (8, 3)


def leaf_geometry(leaves, L):
    """Integer lower corners and sides at level-L resolution, plus float lower corners and sides."""
    leaves = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)
    size = np.left_shift(1, L - leaves[:, 0])
    lo_int = leaves[:, 1:4] * size[:, None]
    a = np.ldexp(1.0, -leaves[:, 0].astype(np.int32))
    lo = leaves[:, 1:4] * a[:, None]
    return lo_int, size, lo, a


def gauss_points(lo, a):
    """2x2x2 Gauss points (n, 8, 3) and the common weight a^3/8 (n,) of each cube."""
    return lo[:, None, :] + a[:, None, None] * _REF[None, :, :], a ** 3 / 8.0


def point_rule(lo_t, a_t, lo_s, a_s):
    """sum_{g,g'} w_g w_g' / (4 pi |x_g - y_g'|) for arrays of cube pairs.

    The 2x2x2 points are tensor products, so per axis the differences x_g - y_g' take the
    four values (target node) - (source node); the 64 squared distances are sums of one
    squared difference per axis.
    """
    xi = np.array(_XI)
    wt = a_t ** 3 / 8.0
    ws = a_s ** 3 / 8.0
    r2 = 0.0
    for ax, shape in zip(range(3), [(-1, 4, 1, 1), (-1, 1, 4, 1), (-1, 1, 1, 4)]):
        xt = lo_t[:, ax, None] + a_t[:, None] * xi[None, :]  # (n, 2)
        xs = lo_s[:, ax, None] + a_s[:, None] * xi[None, :]
        d = (xt[:, :, None] - xs[:, None, :]).reshape(-1, 4)  # (n, 4)
        r2 = r2 + (d * d).reshape(shape)
    return wt * ws * (1.0 / np.sqrt(r2)).reshape(-1, 64).sum(axis=1) / (4.0 * np.pi)


def touching_class_index(lo_t, s_t, lo_s, s_s):
    """Touching class index per pair (0..6 in touching.TOUCH_CLASSES order) or -1 if not touching."""
    lo = np.maximum(lo_t, lo_s)
    hi = np.minimum(lo_t + s_t[:, None], lo_s + s_s[:, None])
    touch = np.all(lo <= hi, axis=1)
    n_contact = np.sum(lo == hi, axis=1)
    same = s_t == s_s
    ratio_ok = np.where(same, True, (np.maximum(s_t, s_s) == 2 * np.minimum(s_t, s_s)))
    if np.any(touch & ~ratio_ok):
        raise AssertionError("touching leaves violate 2:1 balance")
    if np.any(touch & ~same & (n_contact == 0)):
        raise AssertionError("cells of different size overlap")
    cls = np.where(same, n_contact, 3 + n_contact)
    return np.where(touch, cls, -1)


def near_gauss_orders(leaves, L, near_order):
    """Gauss points per axis of each leaf: 2 (near_order 0) or 2 + (L - level) (near_order 1)."""
    lev = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)[:, 0]
    if near_order == 0:
        return np.full(len(lev), 2, dtype=np.int32)
    if near_order != 1:
        raise ValueError("near_order must be 0 or 1")
    return (2 + (L - lev)).astype(np.int32)


_TABLES = None


def gauss_tables():
    """Gauss-Legendre nodes and weights on [0, 1]: row n holds the n-point rule (n = 1..16)."""
    global _TABLES
    if _TABLES is None:
        gx, gw = np.zeros((17, 16)), np.zeros((17, 16))
        for n in range(1, 17):
            t, w = np.polynomial.legendre.leggauss(n)
            gx[n, :n], gw[n, :n] = 0.5 * (t + 1.0), 0.5 * w
        _TABLES = (gx, gw)
    return _TABLES


def _rule_args(orders):
    """ctypes arguments (order, nodes, weights) of the C loops; NULLs for the 2x2x2 rule."""
    if orders is None:
        return None, None, None, None
    orders = np.ascontiguousarray(orders, dtype=np.int32)
    if orders.min() < 1 or orders.max() > 16:
        raise ValueError("Gauss orders must be 1..16")
    gx, gw = gauss_tables()
    keep = (orders, gx, gw)
    return keep, orders.ctypes.data, gx.ctypes.data, gw.ctypes.data


def gauss_rule(lo_t, a_t, n_t, lo_s, a_s, n_s):
    """One pair by NumPy: the n_t^3-point rule on cube t against the n_s^3-point rule on cube s."""
    def points(lo, a, n):
        t, w = np.polynomial.legendre.leggauss(n)
        t, w = 0.5 * (t + 1.0), 0.5 * w
        X = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
        W = np.einsum("i,j,k->ijk", w, w, w).ravel()
        return np.asarray(lo, dtype=np.float64) + a * X, W * a ** 3

    x, wx = points(lo_t, a_t, n_t)
    y, wy = points(lo_s, a_s, n_s)
    r = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(axis=2))
    return float(wx @ (1.0 / r) @ wy) / (4.0 * np.pi)


def _geometry_arrays(leaves, L):
    lo_int, size, lo, a = leaf_geometry(leaves, L)
    return (np.ascontiguousarray(lo_int, dtype=np.int64), np.ascontiguousarray(size, dtype=np.int64),
            np.ascontiguousarray(lo, dtype=np.float64), np.ascontiguousarray(a, dtype=np.float64))


def entries(leaves, L, ti, si, orders=None):
    """Galerkin entries A_{ti, si} for arrays of leaf-index pairs (plain-C loop, oracle/o1.c).

    orders: Gauss points per axis of each leaf for non-touching pairs (None: the 2x2x2 rule)."""
    lo_int, size, lo, a = _geometry_arrays(leaves, L)
    ti = np.ascontiguousarray(ti, dtype=np.int64)
    si = np.ascontiguousarray(si, dtype=np.int64)
    out = np.empty(len(ti))
    _keep, po, pgx, pgw = _rule_args(orders)
    if _clib.lib().o1_entries(len(ti), ti, si, lo_int, size, lo, a, touching.constants(40), po, pgx, pgw, out):
        raise AssertionError("touching leaves violate 2:1 balance")
    return out


def entries_numpy(leaves, L, ti, si):
    """The same entries as entries(), evaluated with NumPy (cross-check of the C loop)."""
    lo_int, size, lo, a = leaf_geometry(leaves, L)
    ti = np.asarray(ti)
    si = np.asarray(si)
    cls = touching_class_index(lo_int[ti], size[ti], lo_int[si], size[si])
    t = cls >= 0
    out = np.empty(len(ti))
    nt = ~t
    out[nt] = point_rule(lo[ti[nt]], a[ti[nt]], lo[si[nt]], a[si[nt]])
    if np.any(t):
        consts = touching.constants(40)
        a_small = np.minimum(a[ti[t]], a[si[t]])
        out[t] = consts[cls[t]] * a_small ** 5 / (4.0 * np.pi)
    return out


def apply(leaves, L, f, targets=None, orders=None):
    """u_t = sum over ALL leaves s of A_{ts} f_s, for the given target leaf indices (default all).

    orders: Gauss points per axis of each leaf for every non-touching pair (None: 2x2x2)."""
    leaves = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)
    n = len(leaves)
    f = np.ascontiguousarray(f, dtype=np.float64)
    targets = np.arange(n) if targets is None else np.asarray(targets)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    lo_int, size, lo, a = _geometry_arrays(leaves, L)
    u = np.empty(len(targets))
    _keep, po, pgx, pgw = _rule_args(orders)
    if _clib.lib().o1_apply(n, lo_int, size, lo, a, touching.constants(40), po, pgx, pgw, f, len(targets), targets, u):
        raise AssertionError("touching leaves violate 2:1 balance")
    return u


def apply_near_order(mesh, f, targets=None):
    """The operator with the level-dependent rule on the mesh's near pairs (w x N*(w), marked
    sources expanded to their leaves) and the 2x2x2 rule on every other non-touching pair:
    O1 plus, over each target's near pairs, (level rule - 2x2x2 rule) times f."""
    lv = mesh.leaf_array()
    L = mesh.L
    targets = np.arange(len(lv)) if targets is None else np.asarray(targets, dtype=np.int64)
    u = apply(lv, L, f, targets)
    ti, si = [], []
    for n, t in enumerate(targets):
        lev, i, j, k = mesh.leaves[t]
        for s in mesh.near_leaf_sources(lev, (i, j, k)):
            ti.append(n)
            si.append(mesh.leaf_index[s])
    ti = np.array(ti, dtype=np.int64)
    si = np.array(si, dtype=np.int64)
    tg = targets[ti]
    d = entries(lv, L, tg, si, near_gauss_orders(lv, L, 1)) - entries(lv, L, tg, si)
    return u + np.bincount(ti, weights=d * np.asarray(f)[si], minlength=len(targets))


def matrix(leaves, L):
    """The dense Galerkin matrix A (small meshes only)."""
    n = len(leaves)
    ti = np.repeat(np.arange(n), n)
    si = np.tile(np.arange(n), n)
    return entries(leaves, L, ti, si).reshape(n, n)
