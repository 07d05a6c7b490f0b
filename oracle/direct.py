"""O1: the Galerkin volume potential u = A f by direct O(N^2) evaluation (test infrastructure only).

Definition (Sec. 1.2, eq. galerkin:vol with degree p = 0 and the indicator basis; Sec. 1.1 for
the Newton potential and G = 1/(4 pi |x - y|)):

  u_w = <1_w, N f_h>_{L2(Omega)} = sum_lambda A_{w lambda} f_lambda,
  A_{w lambda} = int_w int_lambda G(x, y) dy dx,

with f_h piecewise constant on the leaves. Entries of touching pairs (closed cubes
intersect) are the exact integrals of oracle.touching; entries of all other pairs use the
2x2x2 Gauss-Legendre point rule on both cells:

  A_{w lambda} ~ sum_{g in w} sum_{g' in lambda} w_g w_g' G(x_g, y_g').
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


def _geometry_arrays(leaves, L):
    lo_int, size, lo, a = leaf_geometry(leaves, L)
    return (np.ascontiguousarray(lo_int, dtype=np.int64), np.ascontiguousarray(size, dtype=np.int64),
            np.ascontiguousarray(lo, dtype=np.float64), np.ascontiguousarray(a, dtype=np.float64))


def entries(leaves, L, ti, si):
    """Galerkin entries A_{ti, si} for arrays of leaf-index pairs (plain-C loop, oracle/o1.c)."""
    lo_int, size, lo, a = _geometry_arrays(leaves, L)
    ti = np.ascontiguousarray(ti, dtype=np.int64)
    si = np.ascontiguousarray(si, dtype=np.int64)
    out = np.empty(len(ti))
    if _clib.lib().o1_entries(len(ti), ti, si, lo_int, size, lo, a, touching.constants(40), out):
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


def apply(leaves, L, f, targets=None):
    """u_t = sum over ALL leaves s of A_{ts} f_s, for the given target leaf indices (default all)."""
    leaves = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)
    n = len(leaves)
    f = np.ascontiguousarray(f, dtype=np.float64)
    targets = np.arange(n) if targets is None else np.asarray(targets)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    lo_int, size, lo, a = _geometry_arrays(leaves, L)
    u = np.empty(len(targets))
    if _clib.lib().o1_apply(n, lo_int, size, lo, a, touching.constants(40), f, len(targets), targets, u):
        raise AssertionError("touching leaves violate 2:1 balance")
    return u


def matrix(leaves, L):
    """The dense Galerkin matrix A (small meshes only)."""
    n = len(leaves)
    ti = np.repeat(np.arange(n), n)
    si = np.tile(np.arange(n), n)
    return entries(leaves, L, ti, si).reshape(n, n)
