// Exact Galerkin integrals of 1/|x - y| with Legendre weights over touching cube pairs: the
// singular near-field blocks of the degree-p leaf bases (Sec. 1.2, the finite element space with
// polynomials of degree p_w per leaf; Sec. 3 integrates such singular pairs by transforms to smooth
// integrals, here the self-similarity of the cube does it, as for the degree-0 classes).
//
// Local coordinates of a cube of side s and centre c: xi = (x - c)/s in [-1/2, 1/2]^3. Monomial
// table of a pair (A, B):  I[alpha][beta] = int_A int_B xi^alpha eta^beta / |x - y| dy dx,
// |alpha|, |beta| <= P, in the graded multi-index order of multiindex.hpp. Unit pairs at integer
// offset o (B = A + o) touch when |o|_inf <= 1. Halving both cubes of a unit pair gives 64 pairs of
// side 1/2 at offsets (in half units) 2o + v - u, u, v in {0,1}^3 the child positions; on child u,
//     xi = xi_u / 2 + s_u / 4,  s_u = 2u - 1,  so  xi^alpha = sum_{alpha' <= alpha} E_u[alpha][alpha'] xi_u^alpha',
//     E_u[alpha][alpha'] = prod_i C(alpha_i, alpha'_i) 2^-alpha'_i (s_i / 4)^(alpha_i - alpha'_i),
// and a pair of side 1/2 is 2^-5 times the unit pair at the same offset (degree-5 homogeneity;
// xi is scale free):
//     I_o = 2^-5 sum_{u, v} (E_u x E_v) J_{2o + v - u},
// with J the touching table where the child pair touches and a regular unit-pair integral (6-D
// Gauss-Legendre on the host) otherwise. The four canonical offsets (0,0,0), (0,0,1), (0,1,1),
// (1,1,1) solve this system by fixed-point iteration: its degree-0 part is the 4x4 system of the
// class constants (contraction factor 1/4), the higher degrees contract faster. Every other offset
// follows from a canonical one by a signed permutation of the axes. A side-2 cube is 8 unit cubes,
// so the pairs of sides 1 and 2 are sums of unit pairs: I = sum_k (1 x E_k) J_{b + k}. Finally the
// Legendre weights P_a(2 xi) replace the monomials (their coefficients, per axis).
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "multiindex.hpp"

namespace bcv {

void gauss_legendre01(int n, double *x, double *w);

namespace {

using Off = std::array<int, 3>;

struct Index {  // multi-indices of total degree <= P in the graded order
    int P, nb;
    std::vector<std::array<int, 3>> e;
    explicit Index(int p) : P(p), nb(ncoef(p))
    {
        for (int d = 0; d <= P; ++d)
            for (int i = d; i >= 0; --i)
                for (int j = d - i; j >= 0; --j) e.push_back({i, j, d - i - j});
    }
    int with(int a, int axis, int v) const  // position of e[a] with component `axis` set to v
    {
        std::array<int, 3> m = e[a];
        m[axis] = v;
        return mi_index(m[0], m[1], m[2]);
    }
};

using Table = std::vector<double>;  // [alpha][beta], nb x nb

// out[.][.] = sum over the 1-D matrix m (lower triangular, (P+1) x (P+1)) applied on `axis` of the
// alpha index (side 0) or the beta index (side 1).
void axis_pass(const Index &ix, const Table &in, Table &out, int side, int axis, const double *m)
{
    const int nb = ix.nb, P1 = ix.P + 1;
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
            const int r = side == 0 ? a : b;
            const int top = ix.e[r][axis];
            double s = 0.0;
            for (int k = 0; k <= top; ++k) {
                const double c = m[top * P1 + k];
                if (c == 0.0) continue;
                const int rk = ix.with(r, axis, k);
                s += c * (side == 0 ? in[(size_t)rk * nb + b] : in[(size_t)a * nb + rk]);
            }
            out[(size_t)a * nb + b] = s;
        }
}

// The child expansion matrix e_s[a][a'] = C(a, a') 2^-a' (s/4)^(a - a'), s = +-1.
std::vector<double> child_matrix(int P, int s)
{
    std::vector<double> m((P + 1) * (P + 1), 0.0);
    for (int a = 0; a <= P; ++a) {
        double binom = 1.0;
        for (int k = 0; k <= a; ++k) {
            if (k > 0) binom = binom * (a - k + 1) / k;
            m[a * (P + 1) + k] = binom * std::ldexp(1.0, -k) * std::pow(0.25 * s, a - k);
        }
    }
    return m;
}

// Monomial coefficients of P_a(2 xi): l[a][g] (three-term recurrence in t = 2 xi).
std::vector<double> legendre_matrix(int P)
{
    std::vector<double> t((P + 1) * (P + 1), 0.0);  // coefficients in t
    t[0] = 1.0;
    if (P >= 1) t[(P + 1) + 1] = 1.0;
    for (int a = 1; a < P; ++a)
        for (int g = 0; g <= a + 1; ++g) {
            double v = -(double)a * (g <= a - 1 ? t[(a - 1) * (P + 1) + g] : 0.0);
            if (g >= 1) v += (2.0 * a + 1.0) * t[a * (P + 1) + g - 1];
            t[(a + 1) * (P + 1) + g] = v / (a + 1.0);
        }
    for (int a = 0; a <= P; ++a)
        for (int g = 0; g <= a; ++g) t[a * (P + 1) + g] *= std::ldexp(1.0, g);  // t^g = 2^g xi^g
    return t;
}

// Canonical form of an offset: |o| sorted ascending, with perm[k] = the axis of the k-th smallest
// |o_i| and sign[k] its sign (+1 for 0).
Off canonical(const Off &o, int perm[3], int sign[3])
{
    int ax[3] = {0, 1, 2};
    std::stable_sort(ax, ax + 3, [&](int a, int b) { return std::abs(o[a]) < std::abs(o[b]); });
    Off c;
    for (int k = 0; k < 3; ++k) {
        perm[k] = ax[k];
        sign[k] = o[ax[k]] < 0 ? -1 : 1;
        c[k] = std::abs(o[ax[k]]);
    }
    return c;
}

// T_o from the canonical table: T_o[alpha][beta] = prod_k sign_k^(alpha_perm(k) + beta_perm(k)) T_c[alpha'][beta'],
// alpha'_k = alpha_perm(k) (the distance is invariant under the signed permutation).
void from_canonical(const Index &ix, const Table &tc, const int perm[3], const int sign[3], Table &out)
{
    const int nb = ix.nb;
    std::vector<int> pos(nb);
    std::vector<int> par(nb);
    for (int a = 0; a < nb; ++a) {
        const auto &m = ix.e[a];
        pos[a] = mi_index(m[perm[0]], m[perm[1]], m[perm[2]]);
        int odd = 0;
        for (int k = 0; k < 3; ++k)
            if (sign[k] < 0) odd += m[perm[k]];
        par[a] = odd & 1;
    }
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
            out[(size_t)a * nb + b] = ((par[a] ^ par[b]) ? -1.0 : 1.0) * tc[(size_t)pos[a] * nb + pos[b]];
}

// Regular unit pair at canonical offset c (|c|_inf >= 2): n-point Gauss-Legendre per axis on both
// cubes, summed axis by axis (z innermost).
Table regular_pair(const Index &ix, const Off &c, int n)
{
    const int P = ix.P, P1 = P + 1, nb = ix.nb;
    std::vector<double> x(n), w(n);
    gauss_legendre01(n, x.data(), w.data());
    std::vector<double> pw(n * P1);  // (node - 1/2)^e
    for (int g = 0; g < n; ++g) {
        double v = 1.0;
        for (int e = 0; e <= P; ++e, v *= x[g] - 0.5) pw[g * P1 + e] = v;
    }
    // Y[gx][hx][ay][by][az][bz]
    const size_t ysz = (size_t)P1 * P1 * P1 * P1;
    std::vector<double> Y((size_t)n * n * ysz, 0.0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int gh = 0; gh < n * n; ++gh) {
        const int gx = gh / n, hx = gh % n;
        const double dx = (x[gx] - x[hx]) - c[0];
        double *y = &Y[(size_t)gh * ysz];
        std::vector<double> Z(P1 * P1), T(P1);
        for (int gy = 0; gy < n; ++gy)
            for (int hy = 0; hy < n; ++hy) {
                const double dy = (x[gy] - x[hy]) - c[1];
                const double dxy = dx * dx + dy * dy;
                std::fill(Z.begin(), Z.end(), 0.0);
                for (int gz = 0; gz < n; ++gz) {
                    std::fill(T.begin(), T.end(), 0.0);
                    for (int hz = 0; hz < n; ++hz) {
                        const double dz = (x[gz] - x[hz]) - c[2];
                        const double k = w[hz] / std::sqrt(dxy + dz * dz);
                        for (int bz = 0; bz <= P; ++bz) T[bz] += k * pw[hz * P1 + bz];
                    }
                    for (int az = 0; az <= P; ++az) {
                        const double s = w[gz] * pw[gz * P1 + az];
                        for (int bz = 0; bz <= P; ++bz) Z[az * P1 + bz] += s * T[bz];
                    }
                }
                const double wyy = w[gy] * w[hy];
                for (int ay = 0; ay <= P; ++ay)
                    for (int by = 0; by <= P; ++by) {
                        const double s = wyy * pw[gy * P1 + ay] * pw[hy * P1 + by];
                        double *yy = y + (size_t)(ay * P1 + by) * P1 * P1;
                        for (int k = 0; k < P1 * P1; ++k) yy[k] += s * Z[k];
                    }
            }
    }
    Table R((size_t)nb * nb, 0.0);
#pragma omp parallel for schedule(static)
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
            const auto &ea = ix.e[a], &eb = ix.e[b];
            double s = 0.0;
            for (int gx = 0; gx < n; ++gx)
                for (int hx = 0; hx < n; ++hx)
                    s += w[gx] * w[hx] * pw[gx * P1 + ea[0]] * pw[hx * P1 + eb[0]] *
                         Y[(size_t)(gx * n + hx) * ysz + (size_t)((ea[1] * P1 + eb[1]) * P1 + ea[2]) * P1 + eb[2]];
            R[(size_t)a * nb + b] = s;
        }
    return R;
}

struct Solver {
    Index ix;
    int n_gauss;
    std::vector<double> E[2];  // child matrices for s = -1 (index 0) and s = +1 (index 1)
    std::map<Off, Table> regular;  // by canonical offset
    Table touch[4];                // canonical (0,0,0), (0,0,1), (0,1,1), (1,1,1): monomials

    explicit Solver(int P) : ix(P), n_gauss(14 + (P + 1) / 2)
    {
        E[0] = child_matrix(P, -1);
        E[1] = child_matrix(P, 1);
    }

    static int touch_class(const Off &c) { return c[0] + c[1] + c[2]; }  // canonical, |c|_inf <= 1

    // The table of the unit pair at offset o (touching: the current iterate; else regular).
    void unit_pair(const Off &o, Table &out)
    {
        int perm[3], sign[3];
        const Off c = canonical(o, perm, sign);
        const Table &tc = c[2] <= 1 ? touch[touch_class(c)] : regular.at(c);
        from_canonical(ix, tc, perm, sign, out);
    }

    // out += scale (E_u x E_v) J  (u or v may be null: identity on that side)
    void expand_add(const Table &J, const int *u, const int *v, double scale, Table &out)
    {
        Table a = J, b(J.size());
        for (int ax = 0; ax < 3; ++ax) {
            if (u) {
                axis_pass(ix, a, b, 0, ax, E[u[ax]].data());
                a.swap(b);
            }
            if (v) {
                axis_pass(ix, a, b, 1, ax, E[v[ax]].data());
                a.swap(b);
            }
        }
        for (size_t k = 0; k < out.size(); ++k) out[k] += scale * a[k];
    }

    void solve()
    {
        const int nb = ix.nb;
        // regular unit pairs needed by the equal-size equations and the 1:2 pairs
        for (int a = 0; a <= 3; ++a)
            for (int b = a; b <= 3; ++b)
                for (int c = b; c <= 3; ++c)
                    if (c >= 2) regular[{a, b, c}] = regular_pair(ix, {a, b, c}, n_gauss);
        const Off canon[4] = {{0, 0, 0}, {0, 0, 1}, {0, 1, 1}, {1, 1, 1}};
        Table rhs[4];
        for (int k = 0; k < 4; ++k) {
            touch[k].assign((size_t)nb * nb, 0.0);
            rhs[k].assign((size_t)nb * nb, 0.0);
        }
        Table J((size_t)nb * nb);
        for (int k = 0; k < 4; ++k)  // the regular child pairs: fixed part of every equation
            for (int uc = 0; uc < 8; ++uc)
                for (int vc = 0; vc < 8; ++vc) {
                    const int u[3] = {uc & 1, (uc >> 1) & 1, (uc >> 2) & 1};
                    const int v[3] = {vc & 1, (vc >> 1) & 1, (vc >> 2) & 1};
                    const Off o = {2 * canon[k][0] + v[0] - u[0], 2 * canon[k][1] + v[1] - u[1],
                                   2 * canon[k][2] + v[2] - u[2]};
                    if (std::max({std::abs(o[0]), std::abs(o[1]), std::abs(o[2])}) <= 1) continue;
                    unit_pair(o, J);
                    expand_add(J, u, v, 1.0 / 32.0, rhs[k]);
                }
        for (int it = 0; it < 80; ++it) {
            Table next[4];
            double change = 0.0, size = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(max : change, size)
            for (int k = 0; k < 4; ++k) {
                next[k] = rhs[k];
                Table Jt((size_t)nb * nb);
                for (int uc = 0; uc < 8; ++uc)
                    for (int vc = 0; vc < 8; ++vc) {
                        const int u[3] = {uc & 1, (uc >> 1) & 1, (uc >> 2) & 1};
                        const int v[3] = {vc & 1, (vc >> 1) & 1, (vc >> 2) & 1};
                        const Off o = {2 * canon[k][0] + v[0] - u[0], 2 * canon[k][1] + v[1] - u[1],
                                       2 * canon[k][2] + v[2] - u[2]};
                        if (std::max({std::abs(o[0]), std::abs(o[1]), std::abs(o[2])}) > 1) continue;
                        unit_pair(o, Jt);
                        expand_add(Jt, u, v, 1.0 / 32.0, next[k]);
                    }
                for (size_t e = 0; e < next[k].size(); ++e) {
                    change = std::max(change, std::fabs(next[k][e] - touch[k][e]));
                    size = std::max(size, std::fabs(next[k][e]));
                }
            }
            for (int k = 0; k < 4; ++k) touch[k].swap(next[k]);
            if (change <= 1e-17 * size) break;
        }
    }

    // Pair with sides 1 (target, at the origin) and 2 (source, lower corner b in unit steps).
    Table small_big(const Off &b)
    {
        Table out((size_t)ix.nb * ix.nb, 0.0), J((size_t)ix.nb * ix.nb);
        for (int kc = 0; kc < 8; ++kc) {
            const int k[3] = {kc & 1, (kc >> 1) & 1, (kc >> 2) & 1};
            unit_pair({b[0] + k[0], b[1] + k[1], b[2] + k[2]}, J);
            expand_add(J, nullptr, k, 1.0, out);
        }
        return out;
    }

    void to_legendre(Table &t)
    {
        const std::vector<double> l = legendre_matrix(ix.P);
        Table b(t.size());
        for (int side = 0; side < 2; ++side)
            for (int ax = 0; ax < 3; ++ax) {
                axis_pass(ix, t, b, side, ax, l.data());
                t.swap(b);
            }
    }
};

}  // namespace

const BasisTouchTable &basis_touch_table(int P)
{
    static std::mutex mu;
    static std::map<int, BasisTouchTable> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(P);
    if (it != cache.end()) return it->second;
    BCV_REQUIRE(P >= 0 && P <= kMaxBasisDegree, BCV_EINVAL, "basis degree out of range");
    Solver sv(P);
    sv.solve();
    BasisTouchTable tab;
    tab.P = P;
    tab.nb = sv.ix.nb;
    const size_t blk = (size_t)tab.nb * tab.nb;
    tab.equal.assign(27 * blk, 0.0);
    tab.small_big.assign(64 * blk, 0.0);
    Table legc[4];
    for (int k = 0; k < 4; ++k) {
        legc[k] = sv.touch[k];
        sv.to_legendre(legc[k]);
    }
    Table t(blk);
    for (int o2 = -1; o2 <= 1; ++o2)
        for (int o1 = -1; o1 <= 1; ++o1)
            for (int o0 = -1; o0 <= 1; ++o0) {
                int perm[3], sign[3];
                const Off c = canonical({o0, o1, o2}, perm, sign);
                from_canonical(sv.ix, legc[Solver::touch_class(c)], perm, sign, t);
                std::copy(t.begin(), t.end(), tab.equal.begin() + (size_t)((o0 + 1) + 3 * (o1 + 1) + 9 * (o2 + 1)) * blk);
            }
    for (int b2 = -2; b2 <= 1; ++b2)
        for (int b1 = -2; b1 <= 1; ++b1)
            for (int b0 = -2; b0 <= 1; ++b0) {
                const bool inside = (b0 == -1 || b0 == 0) && (b1 == -1 || b1 == 0) && (b2 == -1 || b2 == 0);
                if (inside) continue;  // the unit cube would lie inside the side-2 cube
                Table sb = sv.small_big({b0, b1, b2});
                sv.to_legendre(sb);
                std::copy(sb.begin(), sb.end(),
                          tab.small_big.begin() + (size_t)((b0 + 2) + 4 * (b1 + 2) + 16 * (b2 + 2)) * blk);
            }
    return cache.emplace(P, std::move(tab)).first->second;
}

}  // namespace bcv
