/*
 * Galerkin entries of touching cells of a mapped (curved) mesh -- TEST INFRASTRUCTURE ONLY.
 * Part of the CPU oracle (see oracle/__init__.py and oracle/mapped.py); never linked into the
 * product library.
 *
 * A mapped mesh is the BC cube octree of [0,1]^3 pushed through a map Phi; a leaf w is Phi(c_w)
 * for a reference cube c_w, and the entry of two leaves (Sec. 1.2, degree 0, indicator basis) is
 *   A_ts = int_{c_t} int_{c_s} G(Phi(xi), Phi(eta)) J(xi) J(eta) d eta d xi,  J = |det D Phi|,
 * G = 1/(4 pi |x - y|). Maps: 0 = identity, 1 = the analytic cube-to-sphere map (the volume form of
 * the mapping reviewed by Zucker and Higashi, "Cube-to-sphere projections for procedural texturing
 * and beyond", JCGT 7(2), 2018): with u = 2 xi - 1,
 *   y_i = u_i sqrt(1 - u_j^2/2 - u_k^2/2 + u_j^2 u_k^2/3),  Phi(xi) = (1 + y)/2,
 * which takes [0,1]^3 onto the ball of centre (1/2,1/2,1/2) and radius 1/2; D Phi(xi) = D y(u).
 *
 * Touching cubes of equal side a (lower corners lo_t, lo_s, delta = (lo_s - lo_t)/a in {-1,0,1}^3):
 * with xi = lo_t + a s, eta = lo_s + a t and z = delta + t - s (so eta - xi = a z),
 *   A = a^6 int dz int_{B(z)} F(s, s + z - delta) ds,  B(z) = [0,1]^3 cap (delta - z + [0,1]^3).
 * The z range [delta_i - 1, delta_i + 1] of each axis is cut at delta_i into two unit segments, so z
 * runs over 8 unit boxes; on each box B(z) is a box whose ends are linear in z. A box with z = 0 as
 * a corner carries the singularity of G there: it is split into 3 pyramids by the largest of
 * |z_1|, |z_2|, |z_3| (Duffy: |z_k| = lambda, the other two lambda mu_1, lambda mu_2, Jacobian
 * lambda^2, which cancels 1/|z|); the other boxes take a tensor Gauss rule in z. Inside, s runs over
 * B(z) with a tensor Gauss rule. Orders: n_lam (lambda), n_mu (mu_1, mu_2), n_z, n_s.
 * Sides in ratio 2 (the larger cube's 8 children have the smaller side): children that touch the
 * smaller cube take the rule above; the others the n_r^3 x n_r^3 tensor Gauss rule.
 * Gauss-Legendre nodes and weights on [0, 1] come in as a table (row n: the n-point rule, 16 wide).
 */
#include <math.h>
#include <stdint.h>

static void map_point(int kind, const double *x, double *p, double *jac)
{
    if (kind == 0) {
        p[0] = x[0], p[1] = x[1], p[2] = x[2];
        *jac = 1.0;
        return;
    }
    double u[3], s[3], d[3][3];
    for (int i = 0; i < 3; ++i) u[i] = 2.0 * x[i] - 1.0;
    for (int i = 0; i < 3; ++i) {
        int j = (i + 1) % 3, k = (i + 2) % 3;
        double uj2 = u[j] * u[j], uk2 = u[k] * u[k];
        s[i] = sqrt(1.0 - 0.5 * uj2 - 0.5 * uk2 + uj2 * uk2 / 3.0);
        p[i] = 0.5 + 0.5 * u[i] * s[i];
        /* d y_i / d u_m */
        d[i][i] = s[i];
        d[i][j] = u[i] * u[j] * (-1.0 + 2.0 * uk2 / 3.0) / (2.0 * s[i]);
        d[i][k] = u[i] * u[k] * (-1.0 + 2.0 * uj2 / 3.0) / (2.0 * s[i]);
    }
    double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) - d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                 d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
    *jac = fabs(det);
}

void om_map(int kind, int64_t n, const double *x, double *p, double *jac)
{
    for (int64_t i = 0; i < n; ++i) map_point(kind, x + 3 * i, p + 3 * i, jac + i);
}

/* F(s, t) = G(Phi(lo_t + a s), Phi(lo_s + a t)) J J, without the a^6. */
static double integrand(int kind, const double *lo_t, const double *lo_s, double a, const double *s, const double *t)
{
    double x[3], y[3], px[3], py[3], jx, jy;
    for (int i = 0; i < 3; ++i) x[i] = lo_t[i] + a * s[i], y[i] = lo_s[i] + a * t[i];
    map_point(kind, x, px, &jx);
    map_point(kind, y, py, &jy);
    double dx = px[0] - py[0], dy = px[1] - py[1], dz = px[2] - py[2];
    return jx * jy / (4.0 * M_PI * sqrt(dx * dx + dy * dy + dz * dz));
}

/* int_{B(z)} F(s, s + z - delta) ds by the n_s^3 tensor rule. */
static double inner(int kind, const double *lo_t, const double *lo_s, double a, const int *delta, const double *z,
                    int ns, const double *gx, const double *gw)
{
    double b0[3], len[3];
    for (int i = 0; i < 3; ++i) {
        double lo = delta[i] - z[i] > 0.0 ? delta[i] - z[i] : 0.0;
        double hi = 1.0 + delta[i] - z[i] < 1.0 ? 1.0 + delta[i] - z[i] : 1.0;
        b0[i] = lo;
        len[i] = hi - lo;
    }
    if (len[0] <= 0.0 || len[1] <= 0.0 || len[2] <= 0.0) return 0.0;
    const double *x = gx + 16 * ns, *w = gw + 16 * ns;
    double sum = 0.0;
    for (int c = 0; c < ns; ++c)
        for (int b = 0; b < ns; ++b)
            for (int q = 0; q < ns; ++q) {
                double s[3] = {b0[0] + len[0] * x[q], b0[1] + len[1] * x[b], b0[2] + len[2] * x[c]};
                double t[3] = {s[0] + z[0] - delta[0], s[1] + z[1] - delta[1], s[2] + z[2] - delta[2]};
                sum += w[q] * w[b] * w[c] * integrand(kind, lo_t, lo_s, a, s, t);
            }
    return sum * len[0] * len[1] * len[2];
}

/* Equal sides, closed cubes touching (or equal). */
double om_touch_same(int kind, const double *lo_t, const double *lo_s, double a, int n_lam, int n_mu, int n_z, int ns,
                     const double *gx, const double *gw)
{
    int delta[3];
    for (int i = 0; i < 3; ++i) delta[i] = (int)lround((lo_s[i] - lo_t[i]) / a);
    double total = 0.0;
    for (int box = 0; box < 8; ++box) {
        double g0[3];  /* segment [g0, g0 + 1] per axis */
        int corner = 1;
        double sg[3];  /* z_i = sg_i v_i, v_i in [0, 1], on a box with corner 0 */
        for (int i = 0; i < 3; ++i) {
            int upper = (box >> i) & 1;
            g0[i] = upper ? (double)delta[i] : (double)(delta[i] - 1);
            if (g0[i] == 0.0)
                sg[i] = 1.0;
            else if (g0[i] == -1.0)
                sg[i] = -1.0;
            else
                corner = 0;
        }
        if (corner) {
            const double *xl = gx + 16 * n_lam, *wl = gw + 16 * n_lam, *xm = gx + 16 * n_mu, *wm = gw + 16 * n_mu;
            for (int k = 0; k < 3; ++k) {
                int j1 = (k + 1) % 3, j2 = (k + 2) % 3;
                for (int il = 0; il < n_lam; ++il)
                    for (int i1 = 0; i1 < n_mu; ++i1)
                        for (int i2 = 0; i2 < n_mu; ++i2) {
                            double lam = xl[il];
                            double z[3];
                            z[k] = sg[k] * lam;
                            z[j1] = sg[j1] * lam * xm[i1];
                            z[j2] = sg[j2] * lam * xm[i2];
                            double wgt = wl[il] * wm[i1] * wm[i2] * lam * lam;
                            total += wgt * inner(kind, lo_t, lo_s, a, delta, z, ns, gx, gw);
                        }
            }
        } else {
            const double *xz = gx + 16 * n_z, *wz = gw + 16 * n_z;
            for (int c = 0; c < n_z; ++c)
                for (int b = 0; b < n_z; ++b)
                    for (int q = 0; q < n_z; ++q) {
                        double z[3] = {g0[0] + xz[q], g0[1] + xz[b], g0[2] + xz[c]};
                        total += wz[q] * wz[b] * wz[c] * inner(kind, lo_t, lo_s, a, delta, z, ns, gx, gw);
                    }
        }
    }
    double a3 = a * a * a;
    return total * a3 * a3;
}

/* Tensor rule n^3 x n^3 on two cubes (lower corners, sides). */
double om_regular(int kind, const double *lo_t, double a_t, const double *lo_s, double a_s, int n, const double *gx,
                  const double *gw)
{
    const double *x = gx + 16 * n, *w = gw + 16 * n;
    double sum = 0.0;
    for (int i = 0; i < n * n * n; ++i) {
        double xi[3] = {lo_t[0] + a_t * x[i % n], lo_t[1] + a_t * x[(i / n) % n], lo_t[2] + a_t * x[i / (n * n)]};
        double wi = w[i % n] * w[(i / n) % n] * w[i / (n * n)];
        double px[3], jx;
        map_point(kind, xi, px, &jx);
        for (int m = 0; m < n * n * n; ++m) {
            double eta[3] = {lo_s[0] + a_s * x[m % n], lo_s[1] + a_s * x[(m / n) % n], lo_s[2] + a_s * x[m / (n * n)]};
            double wm = w[m % n] * w[(m / n) % n] * w[m / (n * n)];
            double py[3], jy;
            map_point(kind, eta, py, &jy);
            double dx = px[0] - py[0], dy = px[1] - py[1], dz = px[2] - py[2];
            sum += wi * wm * jx * jy / sqrt(dx * dx + dy * dy + dz * dz);
        }
    }
    double vt = a_t * a_t * a_t, vs = a_s * a_s * a_s;
    return sum * vt * vs / (4.0 * M_PI);
}

static int cubes_touch(const double *lo1, double a1, const double *lo2, double a2)
{
    for (int i = 0; i < 3; ++i) {
        double lo = lo1[i] > lo2[i] ? lo1[i] : lo2[i];
        double hi = lo1[i] + a1 < lo2[i] + a2 ? lo1[i] + a1 : lo2[i] + a2;
        if (lo > hi) return 0;
    }
    return 1;
}

/* Entry of a touching pair: equal sides, or sides in ratio 2 (the larger split into children). */
double om_touch_entry(int kind, const double *lo_t, double a_t, const double *lo_s, double a_s, int n_lam, int n_mu,
                      int n_z, int ns, int n_r, const double *gx, const double *gw)
{
    if (a_t == a_s) return om_touch_same(kind, lo_t, lo_s, a_t, n_lam, n_mu, n_z, ns, gx, gw);
    int big_is_t = a_t > a_s;
    const double *lo_b = big_is_t ? lo_t : lo_s, *lo_m = big_is_t ? lo_s : lo_t;
    double a = big_is_t ? a_s : a_t;
    double sum = 0.0;
    for (int c = 0; c < 8; ++c) {
        double lo_c[3] = {lo_b[0] + a * (c & 1), lo_b[1] + a * ((c >> 1) & 1), lo_b[2] + a * ((c >> 2) & 1)};
        const double *t = big_is_t ? lo_c : lo_m, *s = big_is_t ? lo_m : lo_c;
        if (cubes_touch(lo_c, a, lo_m, a))
            sum += om_touch_same(kind, t, s, a, n_lam, n_mu, n_z, ns, gx, gw);
        else
            sum += om_regular(kind, t, a, s, a, n_r, gx, gw);
    }
    return sum;
}

/* A batch of touching entries (OpenMP over pairs). lo_t, lo_s: 3 per pair; a_t, a_s: 1 per pair. */
void om_touch_entries(int kind, int64_t n, const double *lo_t, const double *a_t, const double *lo_s, const double *a_s,
                      int n_lam, int n_mu, int n_z, int ns, int n_r, const double *gx, const double *gw, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i)
        out[i] = om_touch_entry(kind, lo_t + 3 * i, a_t[i], lo_s + 3 * i, a_s[i], n_lam, n_mu, n_z, ns, n_r, gx, gw);
}

/* A batch of regular entries (OpenMP over pairs). */
void om_regular_entries(int kind, int64_t n, const double *lo_t, const double *a_t, const double *lo_s,
                        const double *a_s, int n_r, const double *gx, const double *gw, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) out[i] = om_regular(kind, lo_t + 3 * i, a_t[i], lo_s + 3 * i, a_s[i], n_r, gx, gw);
}
