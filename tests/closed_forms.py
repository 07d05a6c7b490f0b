"""Closed-form potentials used to pin the oracle (not part of the method).

Homogeneous box: the Newton potential U(p) = int_[0,1]^3 dy / (4 pi |p - y|) of the unit cube
with unit density has the classical closed form (rectangular-prism gravity formula)

  U(p) = (1/4pi) sum_{i,j,k in {0,1}} (-1)^(i+j+k+1) F(X_i, Y_j, Z_k),  X_i = i - p_x, ...
  F(x,y,z) = xy ln(z+r) + yz ln(x+r) + zx ln(y+r)
             - x^2/2 atan(yz/(xr)) - y^2/2 atan(zx/(yr)) - z^2/2 atan(xy/(zr)),  r = |(x,y,z)|,

with terms whose prefactor vanishes taken as 0. It satisfies -Laplacian U = 1 inside the cube.

Uniform ball of radius R, unit density: U(p) = R^2/2 - |p - c|^2/6 inside, R^3/(3 |p - c|) outside.
"""

import numpy as np


def _F(x, y, z):
    r = np.sqrt(x * x + y * y + z * z)
    out = np.zeros_like(r)
    with np.errstate(divide="ignore", invalid="ignore"):
        for a, b, c in ((x, y, z), (y, z, x), (z, x, y)):
            t = np.where(a * b != 0.0, a * b * np.log(np.where(c + r > 0, c + r, 1.0)), 0.0)
            out = out + t
        for a, b, c in ((x, y, z), (y, z, x), (z, x, y)):
            t = np.where(a != 0.0, 0.5 * a * a * np.arctan(b * c / np.where(a * r != 0, a * r, 1.0)), 0.0)
            out = out - t
    return out


def box_potential(p):
    """U(p) for points p of shape (..., 3): potential of the unit cube [0,1]^3, unit density."""
    p = np.asarray(p, dtype=np.float64)
    u = np.zeros(p.shape[:-1])
    for i in (0, 1):
        for j in (0, 1):
            for k in (0, 1):
                s = (-1.0) ** (i + j + k + 1)
                u = u + s * _F(i - p[..., 0], j - p[..., 1], k - p[..., 2])
    return u / (4.0 * np.pi)


def box_potential_cell_averages(level_ijk, n=6):
    """(1/|w|) int_w U for octree cells (level, i, j, k), by an n^3 Gauss rule (U is smooth inside)."""
    lv = np.asarray(level_ijk, dtype=np.int64)
    t, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    X, Y, Z = np.meshgrid(t, t, t, indexing="ij")
    W = np.einsum("i,j,k->ijk", w, w, w).ravel()
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    a = np.ldexp(1.0, -lv[:, 0].astype(np.int32))
    lo = lv[:, 1:4] * a[:, None]
    pts = lo[:, None, :] + a[:, None, None] * nodes[None]
    return box_potential(pts) @ W


def ball_potential(p, centre=(0.5, 0.5, 0.5), radius=0.4):
    d = np.linalg.norm(np.asarray(p, dtype=np.float64) - np.asarray(centre), axis=-1)
    return np.where(d <= radius, radius ** 2 / 2.0 - d * d / 6.0, radius ** 3 / (3.0 * np.maximum(d, 1e-300)))
