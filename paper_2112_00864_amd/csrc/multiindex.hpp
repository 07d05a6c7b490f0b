// Multi-indices alpha = (a0, a1, a2) with |alpha| <= Q in graded order, as compile-time tables.
//
// Position of alpha with d = |alpha|: d(d+1)(d+2)/6 entries of lower degree come first; within
// degree d, a0 runs from d down to 0 and, for each a0, a1 from d-a0 down to 0. Hence every
// alpha with |alpha| <= m occupies exactly the first ncoef(m) positions.
#pragma once

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

}  // namespace bcv
