"""Exact Galerkin integrals of 1/|x - y| over touching cube pairs (test infrastructure only).

The paper computes singular near-field integrals with singularity-removing transforms to
hypercubes followed by tensor Gauss-Legendre rules (Sec. 3, after the translation
operators). For axis-aligned boxes this oracle uses its own reduction, written from the
mathematics rather than from the paper:

  int_A int_B 1/|x - y| dy dx = int_{R^3} prod_i c_i(u_i) / |u| du,   u = x - y,

where c_i(u) = length of [a_i, a_i + s_i] intersected with [b_i + u, b_i + t_i + u] is a
piecewise-linear function of u (elementary convolution identity). Each axis is split at the
kinks of c_i and at 0, so on every sub-box the numerator is a polynomial. Sub-boxes with the
origin as a corner are split into three Duffy pyramids (Duffy 1982), whose Jacobian t^2
cancels the 1/|u| singularity; all other sub-boxes are regular and take tensor
Gauss-Legendre directly.

Cube pairs in a 2:1 balanced octree touch in one of seven ways, with the smaller side
normalised to 1: self, face, edge, vertex (equal sides) and face, edge, vertex with the
larger side 2. The Galerkin entry of a touching pair with smaller side a is
CONSTANTS[class] * a^5 / (4 pi) (translation invariance and degree-5 homogeneity).
"""

import numpy as np

TOUCH_CLASSES = ("self", "face", "edge", "vertex", "face2", "edge2", "vertex2")


def _axis_breaks(alo, ahi, blo, bhi):
    """Kinks of c(u) = |[alo, ahi] cap [blo + u, bhi + u]|, plus 0 if inside the support."""
    pts = {alo - bhi, ahi - blo, alo - blo, ahi - bhi}
    lo, hi = alo - bhi, ahi - blo
    if lo < 0.0 < hi:
        pts.add(0.0)
    return sorted(pts)


def _axis_overlap(u, alo, ahi, blo, bhi):
    """c(u): overlap length of [alo, ahi] and [blo + u, bhi + u]."""
    return np.maximum(0.0, np.minimum(ahi, bhi + u) - np.maximum(alo, blo + u))


def _gauss01(n):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def box_pair_integral(a_lo, a_hi, b_lo, b_hi, n=30):
    """int_A int_B 1/|x-y| dy dx for axis-aligned boxes A = [a_lo, a_hi], B = [b_lo, b_hi]."""
    a_lo, a_hi, b_lo, b_hi = (np.asarray(v, dtype=np.float64) for v in (a_lo, a_hi, b_lo, b_hi))
    breaks = [_axis_breaks(a_lo[i], a_hi[i], b_lo[i], b_hi[i]) for i in range(3)]
    g, gw = _gauss01(n)
    total = 0.0
    for ix in range(len(breaks[0]) - 1):
        for iy in range(len(breaks[1]) - 1):
            for iz in range(len(breaks[2]) - 1):
                lo = np.array([breaks[0][ix], breaks[1][iy], breaks[2][iz]])
                hi = np.array([breaks[0][ix + 1], breaks[1][iy + 1], breaks[2][iz + 1]])
                total += _sub_box(lo, hi, a_lo, a_hi, b_lo, b_hi, g, gw)
    return total


def _numerator(u, a_lo, a_hi, b_lo, b_hi):
    """prod_i c_i(u_i) for points u of shape (..., 3)."""
    out = np.ones(u.shape[:-1])
    for i in range(3):
        out = out * _axis_overlap(u[..., i], a_lo[i], a_hi[i], b_lo[i], b_hi[i])
    return out


def _sub_box(lo, hi, a_lo, a_hi, b_lo, b_hi, g, gw):
    h = hi - lo
    corner_at_origin = all(lo[i] == 0.0 or hi[i] == 0.0 for i in range(3))
    if not corner_at_origin:
        # Regular integrand: plain tensor Gauss-Legendre on the sub-box.
        X, Y, Z = np.meshgrid(lo[0] + h[0] * g, lo[1] + h[1] * g, lo[2] + h[2] * g, indexing="ij")
        W = np.einsum("i,j,k->ijk", gw, gw, gw) * (h[0] * h[1] * h[2])
        u = np.stack([X, Y, Z], axis=-1)
        return float(np.sum(W * _numerator(u, a_lo, a_hi, b_lo, b_hi) / np.linalg.norm(u, axis=-1)))
    # The origin is a corner: write u = sigma * v with v in [0, h]^3, sigma = +-1 per axis.
    sigma = np.array([1.0 if lo[i] == 0.0 else -1.0 for i in range(3)])
    T, S1, S2 = np.meshgrid(g, g, g, indexing="ij")
    W = np.einsum("i,j,k->ijk", gw, gw, gw)
    total = 0.0
    for kax in range(3):
        # Pyramid where v_k / h_k is the largest normalised coordinate: v_k = h_k t,
        # v_j = h_j t s_j for the other two axes; Jacobian h1 h2 h3 t^2.
        others = [j for j in range(3) if j != kax]
        v = np.empty(T.shape + (3,))
        v[..., kax] = h[kax] * T
        v[..., others[0]] = h[others[0]] * T * S1
        v[..., others[1]] = h[others[1]] * T * S2
        u = v * sigma
        # |u| = t * sqrt(h_k^2 + (h_j s_j)^2 + (h_m s_m)^2): the t cancels against t^2.
        rho = np.sqrt(h[kax] ** 2 + (h[others[0]] * S1) ** 2 + (h[others[1]] * S2) ** 2)
        integrand = _numerator(u, a_lo, a_hi, b_lo, b_hi) * T / rho
        total += float(np.sum(W * integrand)) * h[0] * h[1] * h[2]
    return total


def class_geometry(name):
    """Canonical box pair (A, B) of a touching class, smaller side 1."""
    unit = (np.zeros(3), np.ones(3))
    if name == "self":
        return unit, unit
    if name in ("face", "edge", "vertex"):
        n_contact = {"face": 1, "edge": 2, "vertex": 3}[name]
        o = np.array([1.0] * n_contact + [0.0] * (3 - n_contact))
        return unit, (o, o + 1.0)
    if name in ("face2", "edge2", "vertex2"):
        # Big cube of side 2 on the negative side of the contact axes; the small unit cube
        # [0,1]^3 sits at a corner of the big cube's face / edge / vertex.
        n_contact = {"face2": 1, "edge2": 2, "vertex2": 3}[name]
        big_lo = np.array([-2.0] * n_contact + [0.0] * (3 - n_contact))
        return (big_lo, big_lo + 2.0), unit
    raise ValueError(name)


def touching_constant(name, n=30):
    """C_class = int_A int_B 1/|x-y| for the canonical pair of the class (smaller side 1)."""
    (alo, ahi), (blo, bhi) = class_geometry(name)
    return box_pair_integral(alo, ahi, blo, bhi, n=n)


_CACHE = {}


def constants(n=30):
    """All seven class constants, in TOUCH_CLASSES order (cached per n)."""
    if n not in _CACHE:
        _CACHE[n] = np.array([touching_constant(c, n) for c in TOUCH_CLASSES])
    return _CACHE[n]


def classify(lo_t, size_t, lo_s, size_s):
    """Touching class of two leaves given integer lower corners and sides at a common resolution.

    Returns None if the closed cubes do not intersect, else the class name. Raises if they
    touch with a size ratio other than 1 or 2 (the 2:1 balance of the mesh forbids it).
    """
    n_contact = 0
    for i in range(3):
        lo = max(lo_t[i], lo_s[i])
        hi = min(lo_t[i] + size_t, lo_s[i] + size_s)
        if lo > hi:
            return None
        if lo == hi:
            n_contact += 1
    if size_t == size_s:
        if n_contact == 0:
            if tuple(lo_t) != tuple(lo_s):
                raise AssertionError("overlapping distinct cells")
            return "self"
        return ("face", "edge", "vertex")[n_contact - 1]
    small, big = min(size_t, size_s), max(size_t, size_s)
    if big != 2 * small or n_contact == 0:
        raise AssertionError("touching cells violate 2:1 balance")
    return ("face2", "edge2", "vertex2")[n_contact - 1]


# -- polynomial weights (degree-p leaf bases) ------------------------------------------------------
#
# With tensor-product weights P(x) = prod_i P_{a_i}(.) on A and Q(y) = prod_i P_{b_i}(.) on B the
# same reduction holds with a weighted overlap per axis:
#
#   int_A int_B P(x) Q(y) / |x - y| dy dx = int_{R^3} prod_i c_i(u_i) / |u| du,
#   c_i(u) = int over [alo_i, ahi_i] cap [blo_i + u, bhi_i + u] of p_i(x) q_i(x - u) dx,
#
# and c_i is a polynomial in u between the same kinks (the limits move linearly with u), of degree
# at most deg p_i + deg q_i + 1. Each c_i(u) is itself computed by Gauss-Legendre on the overlap
# interval with enough nodes to be exact.


def legendre_table(t, p):
    """P_k(t) for k = 0..p (three-term recurrence): array (p + 1,) + t.shape."""
    t = np.asarray(t, dtype=np.float64)
    out = [np.ones_like(t), t.copy()]
    for k in range(1, p):
        out.append(((2 * k + 1) * t * out[k] - k * out[k - 1]) / (k + 1))
    return np.stack(out[: p + 1])


def _weighted_overlap(u, alo, ahi, blo, bhi, pa, pb):
    """c^{ab}(u) for all a <= pa, b <= pb at points u (any shape): array u.shape + (pa + 1, pb + 1).

    The weights are the Legendre polynomials of each box's own axis, P_a(2(x - ca)/sa) on A and
    P_b(2(y - cb)/sb) on B (y = x - u)."""
    u = np.asarray(u, dtype=np.float64)
    lo = np.maximum(alo, blo + u)
    hi = np.minimum(ahi, bhi + u)
    ln = np.maximum(hi - lo, 0.0)
    m = (pa + pb) // 2 + 1
    t, w = np.polynomial.legendre.leggauss(m)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    x = lo[..., None] + ln[..., None] * t  # u.shape + (m,)
    ca, sa = 0.5 * (alo + ahi), ahi - alo
    cb, sb = 0.5 * (blo + bhi), bhi - blo
    Pa = legendre_table(2.0 * (x - ca) / sa, pa)  # (pa+1,) + u.shape + (m,)
    Pb = legendre_table(2.0 * (x - u[..., None] - cb) / sb, pb)
    return np.einsum("a...k,b...k,k,...->...ab", Pa, Pb, w, ln)


def box_pair_poly(a_lo, a_hi, b_lo, b_hi, pa, pb, n=30):
    """int_A int_B P_alpha(x) P_beta(y) / |x - y| dy dx for all alpha in [0, pa]^3, beta in [0, pb]^3,
    with P_alpha(x) = prod_i P_{alpha_i}(2 (x_i - centre_i)/side_i) the Legendre tensor polynomial of
    each box: array (pa+1,)*3 + (pb+1,)*3 indexed [ax, ay, az, bx, by, bz]. Degree 0 is
    box_pair_integral."""
    a_lo, a_hi, b_lo, b_hi = (np.asarray(v, dtype=np.float64) for v in (a_lo, a_hi, b_lo, b_hi))
    breaks = [_axis_breaks(a_lo[i], a_hi[i], b_lo[i], b_hi[i]) for i in range(3)]
    g, gw = _gauss01(n)
    total = np.zeros((pa + 1,) * 3 + (pb + 1,) * 3)
    for ix in range(len(breaks[0]) - 1):
        for iy in range(len(breaks[1]) - 1):
            for iz in range(len(breaks[2]) - 1):
                lo = np.array([breaks[0][ix], breaks[1][iy], breaks[2][iz]])
                hi = np.array([breaks[0][ix + 1], breaks[1][iy + 1], breaks[2][iz + 1]])
                total += _sub_box_poly(lo, hi, a_lo, a_hi, b_lo, b_hi, pa, pb, g, gw)
    return total


def _sub_box_poly(lo, hi, a_lo, a_hi, b_lo, b_hi, pa, pb, g, gw):
    h = hi - lo
    ov = lambda ax, u: _weighted_overlap(u, a_lo[ax], a_hi[ax], b_lo[ax], b_hi[ax], pa, pb)  # noqa: E731
    corner_at_origin = all(lo[i] == 0.0 or hi[i] == 0.0 for i in range(3))
    if not corner_at_origin:
        u = [lo[i] + h[i] * g for i in range(3)]
        C = [ov(i, u[i]) * (gw * h[i])[:, None, None] for i in range(3)]  # (n, pa+1, pb+1) per axis
        R = 1.0 / np.sqrt(u[0][:, None, None] ** 2 + u[1][None, :, None] ** 2 + u[2][None, None, :] ** 2)
        return np.einsum("xyz,xad,ybe,zcf->abcdef", R, C[0], C[1], C[2], optimize=True)
    sigma = np.array([1.0 if lo[i] == 0.0 else -1.0 for i in range(3)])
    out = np.zeros((pa + 1,) * 3 + (pb + 1,) * 3)
    for kax in range(3):
        # Duffy pyramid with axis kax largest: v_k = h_k t, v_j = h_j t s_j; Jacobian h1 h2 h3 t^2,
        # |u| = t rho(s), so the integrand is t * numerator / rho.
        j1, j2 = [j for j in range(3) if j != kax]
        Ck = ov(kax, sigma[kax] * h[kax] * g) * (gw * g * h[0] * h[1] * h[2])[:, None, None]  # (t, a, b)
        C1 = ov(j1, sigma[j1] * h[j1] * g[:, None] * g[None, :]) * gw[None, :, None, None]  # (t, s1, a, b)
        C2 = ov(j2, sigma[j2] * h[j2] * g[:, None] * g[None, :]) * gw[None, :, None, None]  # (t, s2, a, b)
        rho = np.sqrt(h[kax] ** 2 + (h[j1] * g[:, None]) ** 2 + (h[j2] * g[None, :]) ** 2)  # (s1, s2)
        T = np.einsum("uv,tab,tucd,tvef->acebdf", 1.0 / rho, Ck, C1, C2, optimize=True)
        # T is indexed [a_k, a_j1, a_j2, b_k, b_j1, b_j2]: put the axes back in x, y, z order
        perm = np.argsort([kax, j1, j2])
        out += T.transpose(list(perm) + [3 + q for q in perm])
    return out
