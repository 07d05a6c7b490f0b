// Derivative tables of the Laplace kernel for the interaction (M2L) phase.
//
// The far field of Sec. 3 needs D^gamma g at integer offsets o (in units of the cell side) with
// g(r) = 1/(4 pi |r|) and |gamma| <= q. With a_k(r) = (d^k (1/|r|))(r) / k!, the Cartesian Taylor
// coefficients of the Coulomb kernel satisfy the three-term recurrence (Duan & Krasny, 2001)
//
//     |k| |r|^2 a_k + (2|k| - 1) sum_i r_i a_{k - e_i} + (|k| - 1) sum_i a_{k - 2 e_i} = 0,
//
// with a_0 = 1/|r| and terms with a negative index absent. It is evaluated in long double and
// converted to D^k g = k! a_k / (4 pi).
#include <cmath>
#include <vector>

#include "multiindex.hpp"

namespace bcv {

void derivative_table(int q, const int o[3], double *out)
{
    const int K = ncoef(q);
    std::vector<long double> a(K, 0.0L);
    const long double r[3] = {(long double)o[0], (long double)o[1], (long double)o[2]};
    const long double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    a[0] = 1.0L / std::sqrt(r2);
    for (int d = 1; d <= q; ++d)
        for (int i = d; i >= 0; --i)
            for (int j = d - i; j >= 0; --j) {
                const int k[3] = {i, j, d - i - j};
                long double s1 = 0.0L, s2 = 0.0L;
                for (int ax = 0; ax < 3; ++ax) {
                    int m[3] = {k[0], k[1], k[2]};
                    if (m[ax] >= 1) {
                        --m[ax];
                        s1 += r[ax] * a[mi_index(m[0], m[1], m[2])];
                        if (m[ax] >= 1) {
                            --m[ax];
                            s2 += a[mi_index(m[0], m[1], m[2])];
                        }
                    }
                }
                a[mi_index(i, j, d - i - j)] = -((2 * d - 1) * s1 + (d - 1) * s2) / (d * r2);
            }
    const long double inv4pi = 1.0L / (4.0L * 3.141592653589793238462643383279502884L);
    for (int d = 0; d <= q; ++d)
        for (int i = d; i >= 0; --i)
            for (int j = d - i; j >= 0; --j) {
                const int k[3] = {i, j, d - i - j};
                long double fact = 1.0L;
                for (int ax = 0; ax < 3; ++ax)
                    for (int t = 2; t <= k[ax]; ++t) fact *= t;
                const int n = mi_index(k[0], k[1], k[2]);
                out[n] = (double)(fact * a[n] * inv4pi);
            }
}

}  // namespace bcv
