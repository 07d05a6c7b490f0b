/*
 * Direct O(N^2) Galerkin sums for the VtV volume potential -- TEST INFRASTRUCTURE ONLY.
 * Part of the CPU oracle (see oracle/__init__.py); never linked into the product library.
 *
 * u_t = sum_s A_ts f_s with (Sec. 1.2, Galerkin projection with degree 0, indicator basis):
 *   A_ts = C_class * a_small^5 / (4 pi)          if the closed cubes t and s intersect,
 *   A_ts = sum_{g in t} sum_{g' in s} w_g w_g' / (4 pi |x_g - y_g'|)   otherwise,
 * with the 2x2x2 Gauss-Legendre rule on each cube (w_g = a^3 / 8).
 * The seven class constants are passed in (computed by oracle/touching.py).
 *
 * Level-dependent near-field order (Sec. 4, the near-field quadrature paragraph: fixed order on the
 * finest level, raised on coarser levels): when an order array is given, a non-touching pair takes
 * the n_t^3-point Gauss rule on t and the n_s^3-point rule on s, n = order[leaf], with nodes and
 * weights on [0, 1] passed in (row n of two 17 x 16 tables, from numpy's Gauss-Legendre routine).
 *
 * Leaves are described by integer lower corners and sides at level-L resolution (for the
 * touching test, exact) and by floating lower corners and sides (for the point rule).
 * Plain loops; OpenMP over targets only (each target's sum is one thread's fixed-order loop).
 */
#include <math.h>
#include <stdint.h>

static double node(int g) { return g == 0 ? 0.5 - 0.5 / sqrt(3.0) : 0.5 + 0.5 / sqrt(3.0); }

/* Touching class: -1 not touching; 0 self, 1 face, 2 edge, 3 vertex (equal sides);
 * 4 face, 5 edge, 6 vertex (sides in ratio 2); -2 if the pair breaks 2:1 balance. */
int o1_touch_class(const int64_t *lo_t, int64_t s_t, const int64_t *lo_s, int64_t s_s)
{
    int contact = 0;
    for (int i = 0; i < 3; ++i) {
        int64_t lo = lo_t[i] > lo_s[i] ? lo_t[i] : lo_s[i];
        int64_t ht = lo_t[i] + s_t, hs = lo_s[i] + s_s;
        int64_t hi = ht < hs ? ht : hs;
        if (lo > hi) return -1;
        if (lo == hi) ++contact;
    }
    if (s_t == s_s) return contact; /* 0 = self (same cell) */
    int64_t big = s_t > s_s ? s_t : s_s, small = s_t > s_s ? s_s : s_t;
    if (big != 2 * small || contact == 0) return -2;
    return 3 + contact;
}

double o1_point_rule(const double *lo_t, double a_t, const double *lo_s, double a_s)
{
    double sum = 0.0;
    for (int gz = 0; gz < 2; ++gz)
        for (int gy = 0; gy < 2; ++gy)
            for (int gx = 0; gx < 2; ++gx)
                for (int hz = 0; hz < 2; ++hz)
                    for (int hy = 0; hy < 2; ++hy)
                        for (int hx = 0; hx < 2; ++hx) {
                            double dx = (lo_t[0] + a_t * node(gx)) - (lo_s[0] + a_s * node(hx));
                            double dy = (lo_t[1] + a_t * node(gy)) - (lo_s[1] + a_s * node(hy));
                            double dz = (lo_t[2] + a_t * node(gz)) - (lo_s[2] + a_s * node(hz));
                            sum += 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
                        }
    double wt = a_t * a_t * a_t / 8.0, ws = a_s * a_s * a_s / 8.0;
    return wt * ws * sum / (4.0 * M_PI);
}

/* sum_{g in t} sum_{g' in s} w_g w_g' / (4 pi |x_g - y_g'|), tensor rules of n_t and n_s points per axis. */
double o1_gauss_rule(const double *lo_t, double a_t, int n_t, const double *lo_s, double a_s, int n_s,
                     const double *gx, const double *gw)
{
    const double *xt = gx + 16 * n_t, *wt = gw + 16 * n_t, *xs = gx + 16 * n_s, *ws = gw + 16 * n_s;
    double sum = 0.0;
    for (int i3 = 0; i3 < n_t; ++i3)
        for (int i2 = 0; i2 < n_t; ++i2)
            for (int i1 = 0; i1 < n_t; ++i1) {
                double inner = 0.0;
                for (int j3 = 0; j3 < n_s; ++j3)
                    for (int j2 = 0; j2 < n_s; ++j2)
                        for (int j1 = 0; j1 < n_s; ++j1) {
                            double dx = (lo_t[0] + a_t * xt[i1]) - (lo_s[0] + a_s * xs[j1]);
                            double dy = (lo_t[1] + a_t * xt[i2]) - (lo_s[1] + a_s * xs[j2]);
                            double dz = (lo_t[2] + a_t * xt[i3]) - (lo_s[2] + a_s * xs[j3]);
                            inner += ws[j1] * ws[j2] * ws[j3] / sqrt(dx * dx + dy * dy + dz * dz);
                        }
                sum += wt[i1] * wt[i2] * wt[i3] * inner;
            }
    return sum * (a_t * a_t * a_t) * (a_s * a_s * a_s) / (4.0 * M_PI);
}

/* Gauss orders per leaf (NULL: the 2x2x2 rule everywhere) and the node / weight tables. */
typedef struct {
    const int32_t *order;
    const double *gx, *gw;
} rule_t;

static double entry(int64_t t, int64_t s, const int64_t *lo_int, const int64_t *size,
                    const double *lo, const double *a, const double *consts, const rule_t *r, int *bad)
{
    int c = o1_touch_class(lo_int + 3 * t, size[t], lo_int + 3 * s, size[s]);
    if (c == -2) { *bad = 1; return 0.0; }
    if (c >= 0) {
        double as = a[t] < a[s] ? a[t] : a[s];
        return consts[c] * as * as * as * as * as / (4.0 * M_PI);
    }
    if (r->order && (r->order[t] != 2 || r->order[s] != 2))
        return o1_gauss_rule(lo + 3 * t, a[t], r->order[t], lo + 3 * s, a[s], r->order[s], r->gx, r->gw);
    return o1_point_rule(lo + 3 * t, a[t], lo + 3 * s, a[s]);
}

/* out[p] = A_{ti[p], si[p]} for n pairs. Returns 0, or 1 if a touching pair breaks 2:1 balance.
 * order, gx, gw: see rule_t (order may be NULL). */
int o1_entries(int64_t n, const int64_t *ti, const int64_t *si, const int64_t *lo_int,
               const int64_t *size, const double *lo, const double *a, const double *consts,
               const int32_t *order, const double *gx, const double *gw, double *out)
{
    const rule_t r = {order, gx, gw};
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t p = 0; p < n; ++p) {
        int b = 0;
        out[p] = entry(ti[p], si[p], lo_int, size, lo, a, consts, &r, &b);
        bad |= b;
    }
    return bad;
}

/* u[k] = sum over all n leaves s of A_{targets[k], s} f[s]. Returns 0, or 1 on a 2:1 violation. */
int o1_apply(int64_t n, const int64_t *lo_int, const int64_t *size, const double *lo, const double *a,
             const double *consts, const int32_t *order, const double *gx, const double *gw,
             const double *f, int64_t n_targets, const int64_t *targets, double *u)
{
    const rule_t r = {order, gx, gw};
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (int64_t k = 0; k < n_targets; ++k) {
        int b = 0;
        double acc = 0.0;
        for (int64_t s = 0; s < n; ++s)
            acc += entry(targets[k], s, lo_int, size, lo, a, consts, &r, &b) * f[s];
        u[k] = acc;
        bad |= b;
    }
    return bad;
}

/* Potential sums of the degree-p leaf bases (oracle/basis.py): out[g] = sum_h q[h] / |x_g - y_h|
 * for nx points x and ny weighted source points (y_h, q_h), 3 coordinates per point. Plain loop,
 * OpenMP over the target points (each sum in a fixed order). */
void o1_point_potential(int64_t nx, const double *x, int64_t ny, const double *y, const double *q, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < nx; ++g) {
        double acc = 0.0;
        for (int64_t h = 0; h < ny; ++h) {
            const double d0 = x[3 * g] - y[3 * h], d1 = x[3 * g + 1] - y[3 * h + 1], d2 = x[3 * g + 2] - y[3 * h + 2];
            acc += q[h] / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        }
        out[g] = acc;
    }
}
