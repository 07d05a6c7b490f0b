"""Seeded synthetic inputs for volume-potential runs on boundary-concentrated cube meshes.

This module generates input data only: volume densities on leaves, and boundary data on the
boundary faces. It holds no part of the potential method: no quadrature of cell or face
pairs, no expansions, no translation operators. Both the CPU oracle and the GPU library
receive the data it produces, keyed by each leaf's (level, i, j, k) and each face's
(level, i, j, k, axis, side).

Density recipe (piecewise constant on leaves):
  f(x) = sum_k exp(-|x - c_k|^2 / (2 sigma_k^2)), k = 1..4,
  c_k ~ U[0,1]^3 and sigma_k ~ U[0.1, 0.3], drawn from numpy.random.default_rng(seed)
  in the order c_1..c_4 then sigma_1..sigma_4;
  f_leaf = (1/|leaf|) * (n x n x n Gauss-Legendre rule of f over the leaf), n = 2 by default.
"""

import numpy as np

__all__ = [
    "gaussian_mixture_params",
    "gaussian_mixture",
    "cell_average",
    "leaf_density",
    "ball_indicator",
    "constant_one",
    "harmonic_params",
    "harmonic",
    "face_data",
    "legendre_coefficients",
]


def gaussian_mixture_params(seed, n_terms=4):
    """Centres and widths of the seeded Gaussian mixture (centres first, then widths)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_terms, 3))
    widths = rng.uniform(0.1, 0.3, size=n_terms)
    return centres, widths


def gaussian_mixture(x, centres, widths):
    """Evaluate sum_k exp(-|x-c_k|^2/(2 sigma_k^2)) at points x of shape (..., 3)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape[:-1], dtype=np.float64)
    for c, s in zip(centres, widths):
        d2 = np.sum((x - c) ** 2, axis=-1)
        out += np.exp(-d2 / (2.0 * s * s))
    return out


def ball_indicator(centre=(0.5, 0.5, 0.5), radius=0.4):
    """Return a function x -> 1 inside the ball, 0 outside (uniform-ball density)."""
    c = np.asarray(centre, dtype=np.float64)

    def f(x):
        return (np.sum((np.asarray(x) - c) ** 2, axis=-1) <= radius * radius).astype(np.float64)

    return f


def constant_one(x):
    return np.ones(np.asarray(x).shape[:-1], dtype=np.float64)


def _gauss_legendre_unit(n):
    """Nodes and weights of the n-point Gauss-Legendre rule on [0, 1]."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def cell_average(level_ijk, func, n=2, chunk=65536):
    """Cell averages (1/|w|) int_w func over cubes of the unit-cube octree.

    level_ijk: int array (N, 4) of (level, i, j, k); the cube is [i,i+1]x[j,j+1]x[k,k+1] * 2^-level.
    func: vectorised function of points (..., 3).
    """
    lv = np.asarray(level_ijk, dtype=np.int64)
    t, w = _gauss_legendre_unit(n)
    tx, ty, tz = np.meshgrid(t, t, t, indexing="ij")
    wx, wy, wz = np.meshgrid(w, w, w, indexing="ij")
    nodes = np.stack([tx.ravel(), ty.ravel(), tz.ravel()], axis=-1)  # (n^3, 3) in [0,1]^3
    weights = (wx * wy * wz).ravel()  # sums to 1
    out = np.empty(len(lv), dtype=np.float64)
    for s in range(0, len(lv), chunk):
        blk = lv[s : s + chunk]
        a = np.ldexp(1.0, -blk[:, 0])  # side 2^-level
        lo = blk[:, 1:4] * a[:, None]
        pts = lo[:, None, :] + a[:, None, None] * nodes[None, :, :]
        out[s : s + chunk] = func(pts) @ weights
    return out


def leaf_density(level_ijk, seed=0, n=2):
    """Seeded Gaussian-mixture density projected to piecewise constants on the given leaves."""
    centres, widths = gaussian_mixture_params(seed)
    return cell_average(level_ijk, lambda x: gaussian_mixture(x, centres, widths), n=n)


# -- boundary data: traces of a harmonic function -------------------------------------------------
#
# u(x) = sum_k c_k / |x - p_k|, k = 1..4, with c_k ~ U[0.5, 1.5] and p_k = (1/2, 1/2, 1/2) + R_k d_k,
# d_k uniform on the unit sphere (normalised standard normal), R_k ~ U[1.0, 1.6] (outside the unit
# cube), drawn from numpy.random.default_rng(seed) in the order c, then d, then R. u is harmonic
# in the cube. A boundary face (level, i, j, k, axis, side) is the face of that cube normal to
# `axis` at its low (side 0) or high (side 1) end, outward normal (2 side - 1) e_axis; its data are
# the face averages (n x n Gauss-Legendre) of the Dirichlet trace g = u and of the Neumann trace
# q = du/dn.


def harmonic_params(seed, n_terms=4):
    rng = np.random.default_rng(seed)
    charges = rng.uniform(0.5, 1.5, size=n_terms)
    d = rng.standard_normal(size=(n_terms, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    radii = rng.uniform(1.0, 1.6, size=n_terms)
    return charges, 0.5 + radii[:, None] * d


def harmonic(x, charges, poles, grad=False):
    """u(x) (and its gradient if grad) at points x of shape (..., 3)."""
    x = np.asarray(x, dtype=np.float64)
    u = np.zeros(x.shape[:-1])
    g = np.zeros(x.shape)
    for c, p in zip(charges, poles):
        d = x - p
        r = np.sqrt(np.sum(d * d, axis=-1))
        u += c / r
        g -= c * d / r[..., None] ** 3
    return (u, g) if grad else u


def face_data(faces, seed=0, n=4):
    """Face averages (q, g) of du/dn and u on faces given as an int array (N, 6) of
    (level, i, j, k, axis, side)."""
    charges, poles = harmonic_params(seed)
    f = np.asarray(faces, dtype=np.int64).reshape(-1, 6)
    t, w = _gauss_legendre_unit(n)
    s_, t_ = np.meshgrid(t, t, indexing="ij")
    ww = np.outer(w, w).ravel()
    a = np.ldexp(1.0, -f[:, 0])
    lo = f[:, 1:4] * a[:, None]
    ax, side = f[:, 4], f[:, 5]
    pts = np.repeat(lo[:, None, :], n * n, axis=1)
    rows = np.arange(len(f))
    o1, o2 = (ax + 1) % 3, (ax + 2) % 3
    pts[rows, :, ax] += (side * a)[:, None]
    pts[rows, :, o1] += a[:, None] * s_.ravel()[None, :]
    pts[rows, :, o2] += a[:, None] * t_.ravel()[None, :]
    u, grad = harmonic(pts, charges, poles, grad=True)
    sign = 2.0 * side - 1.0
    dudn = sign[:, None] * grad[rows[:, None], np.arange(n * n)[None, :], ax[:, None]]
    return dudn @ ww, u @ ww


def legendre_coefficients(level_ijk, L, func, extra=4):
    """Density input for degree-p leaf bases: on each leaf (level l, side a, centre c) the coefficients
    f_alpha = <phi^alpha, func> / ||phi^alpha||^2 of the L2 projection of func onto
    phi^alpha(x) = prod_i P_{alpha_i}(2 (x_i - c_i)/a), |alpha| <= p = L - l (Legendre), by an
    (p + extra)-point Gauss-Legendre rule per axis. Returns (coefficients, offsets): leaf-major, leaf w
    owning coefficients[offsets[w]:offsets[w+1]], alpha in the graded order (total degree, then
    alpha_x descending, then alpha_y descending)."""
    lv = np.asarray(level_ijk, dtype=np.int64)
    deg = L - lv[:, 0]
    nb = (deg + 1) * (deg + 2) * (deg + 3) // 6
    offsets = np.concatenate([[0], np.cumsum(nb)]).astype(np.int64)
    out = np.empty(offsets[-1])
    for p in np.unique(deg):
        sel = np.nonzero(deg == p)[0]
        t, w = _gauss_legendre_unit(int(p) + extra)
        nodes = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
        weights = np.einsum("i,j,k->ijk", w, w, w).ravel()
        P = np.polynomial.legendre.legvander(2.0 * nodes - 1.0, int(p))  # (n^3, 3, p + 1)
        idx = [(i, j, d - i - j) for d in range(p + 1) for i in range(d, -1, -1) for j in range(d - i, -1, -1)]
        phi = np.stack([P[:, 0, i] * P[:, 1, j] * P[:, 2, k] for i, j, k in idx], axis=1)  # (n^3, nb)
        norm = np.array([(2 * i + 1) * (2 * j + 1) * (2 * k + 1) for i, j, k in idx], dtype=np.float64)
        a = np.ldexp(1.0, -lv[sel, 0].astype(np.int32))
        for c0 in range(0, len(sel), 4096):
            s = sel[c0 : c0 + 4096]
            pts = lv[s, 1:4][:, None, :] * a[c0 : c0 + 4096, None, None] + a[c0 : c0 + 4096, None, None] * nodes[None]
            vals = func(pts) * weights[None, :]  # (n, n^3)
            coef = (vals @ phi) * norm[None, :]
            for r in range(len(idx)):
                out[offsets[s] + r] = coef[:, r]
    return out, offsets
