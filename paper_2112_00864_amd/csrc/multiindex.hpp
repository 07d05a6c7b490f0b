// Multi-indices alpha = (a0, a1, a2) with |alpha| <= Q in graded order, as compile-time tables.
//
// Position of alpha with d = |alpha|: d(d+1)(d+2)/6 entries of lower degree come first; within
// degree d, a0 runs from d down to 0 and, for each a0, a1 from d-a0 down to 0. Hence every
// alpha with |alpha| <= m occupies exactly the first ncoef(m) positions.
#pragma once
#include <algorithm>

namespace bcv {

constexpr int ncoef(int q) { return (q + 1) * (q + 2) * (q + 3) / 6; }

constexpr int mi_index(int i, int j, int k)
{
    const int d = i + j + k;
    return d * (d + 1) * (d + 2) / 6 + (d - i) * (d - i + 1) / 2 + (d - i - j);
}

template <int Q>
struct MultiIndex {
    static constexpr int K = ncoef(Q);
    int e[K][3];
    int deg[K];
    constexpr MultiIndex() : e{}, deg{}
    {
        int n = 0;
        for (int d = 0; d <= Q; ++d)
            for (int i = d; i >= 0; --i)
                for (int j = d - i; j >= 0; --j) {
                    e[n][0] = i;
                    e[n][1] = j;
                    e[n][2] = d - i - j;
                    deg[n] = d;
                    ++n;
                }
    }
    // Position of alpha + beta (both given by position); only meaningful if |alpha|+|beta| <= Q.
    constexpr int sum(int a, int b) const
    {
        return mi_index(e[a][0] + e[b][0], e[a][1] + e[b][1], e[a][2] + e[b][2]);
    }
};

// The multi-indices with a2 <= 1, |alpha| <= Q, in the same graded order: 2d + 1 of degree d, so
// those of degree <= m occupy the first (m + 1)^2 positions. A homogeneous harmonic polynomial of
// degree d is fixed by these 2d + 1 of its coefficients; the harmonic reduction of the interaction
// phase (kernels.hip) works in this index set.
constexpr int nreduced(int q) { return (q + 1) * (q + 1); }

template <int Q>
struct ReducedIndex {
    static constexpr int R = nreduced(Q);
    int e[R][3];
    int deg[R];
    int full[R];  // position in the full graded order
    constexpr ReducedIndex() : e{}, deg{}, full{}
    {
        int n = 0;
        for (int d = 0; d <= Q; ++d)
            for (int i = d; i >= 0; --i)
                for (int j = d - i; j >= 0; --j) {
                    if (d - i - j > 1) continue;
                    e[n][0] = i;
                    e[n][1] = j;
                    e[n][2] = d - i - j;
                    deg[n] = d;
                    full[n] = mi_index(i, j, d - i - j);
                    ++n;
                }
    }
    // Full position of alpha + beta (both given by reduced position).
    constexpr int sum(int a, int b) const
    {
        return mi_index(e[a][0] + e[b][0], e[a][1] + e[b][1], e[a][2] + e[b][2]);
    }
    // Reduced position of the multi-index (i, d - i - k, k), k <= 1, of degree d: within a degree,
    // a0 = d has one entry (a2 = 0) and every smaller a0 two (a2 = 0, then 1).
    static constexpr int index(int i, int k, int d)
    {
        int n = d * d;  // entries of lower degree
        for (int a = d; a > i; --a) n += (a == d ? 1 : 2);
        return n + k;
    }
};

// Harmonic folding of moments onto the multi-indices with b_z <= 1 (see the M2L section of
// kernels.hip): Mr^b = sum_t c[b][t] M^{src[b][t]} over the (Q + 1)^2 reduced b, with
//     Mr^b = sum_k (-1)^k sum_{i + j = k} C(k, i) M^{b - 2i e_x - 2j e_y + 2k e_z}.
template <int Q>
struct FoldTable {  // Mr^b = sum_t c[b][t] M^{src[b][t]} (full positions)
    static constexpr int fold_terms()
    {
        int best = 1;
        for (int bx = 0; bx <= Q; ++bx)
            for (int by = 0; bx + by <= Q; ++by) best = std::max(best, (bx / 2 + 1) * (by / 2 + 1));
        return best;
    }
    static constexpr int R = nreduced(Q), kTerms = fold_terms();
    int n[R], src[R][kTerms];
    double c[R][kTerms];
    constexpr FoldTable() : n{}, src{}, c{}
    {
        constexpr ReducedIndex<Q> ri{};
        for (int b = 0; b < R; ++b) {
            const int bx = ri.e[b][0], by = ri.e[b][1], bz = ri.e[b][2];
            int cnt = 0;
            double sign = 1.0;
            for (int k = 0; 2 * k <= bx + by; ++k, sign = -sign) {
                double binom = 1.0;  // C(k, i)
                for (int i = 0; i <= k; ++i) {
                    if (i > 0) binom = binom * (k - i + 1) / i;
                    const int j = k - i;
                    if (2 * i > bx || 2 * j > by) continue;
                    src[b][cnt] = mi_index(bx - 2 * i, by - 2 * j, bz + 2 * k);
                    c[b][cnt] = sign * binom;
                    ++cnt;
                }
            }
            n[b] = cnt;
        }
    }
};

// Local coefficients of the harmonic reduction expanded to every multi-index (see the M2L section of
// kernels.hip): Lambda^a for a_z >= 2 from the reduced ones (a_z <= 1), with k = floor(a_z / 2),
//     Lambda^a = (-1)^k sum_{i + j = k} C(k, i) Lambda^{a - 2k e_z + 2i e_x + 2j e_y}.
template <int Q>
struct ExpandTable {  // Lambda^a = sum_t c[a][t] Lambda~^{src[a][t]} (reduced positions), a full
    static constexpr int K = ncoef(Q), kTerms = Q / 2 + 1;
    int n[K], src[K][kTerms];
    double c[K][kTerms];
    constexpr ExpandTable() : n{}, src{}, c{}
    {
        constexpr MultiIndex<Q> mi{};
        for (int a = 0; a < K; ++a) {
            const int ax = mi.e[a][0], az = mi.e[a][2], k = az / 2;
            const double sign = (k & 1) ? -1.0 : 1.0;
            double binom = 1.0;
            for (int i = 0; i <= k; ++i) {
                if (i > 0) binom = binom * (k - i + 1) / i;
                src[a][i] = ReducedIndex<Q>::index(ax + 2 * i, az - 2 * k, mi.deg[a]);
                c[a][i] = sign * binom;
            }
            n[a] = k + 1;
        }
    }
};

}  // namespace bcv
