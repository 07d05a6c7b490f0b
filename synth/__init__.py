"""Seeded synthetic inputs for volume-potential runs on boundary-concentrated cube meshes.

This module generates densities only. It holds no part of the volume-potential method:
no Green's function, no quadrature of cell pairs, no expansions. Both the CPU oracle and
the GPU library receive the densities it produces, keyed by each leaf's (level, i, j, k).

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
