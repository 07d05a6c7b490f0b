// Exact Galerkin integrals of 1/|x - y| over touching cube pairs (the singular near field).
//
// The paper integrates singular near-field pairs with singularity-removing transforms
// (Sec. 3, after the translation operators). On an axis-aligned 2:1-balanced cube octree the
// touching pairs fall into seven classes, each fixed up to the factor a_small^5 by translation
// invariance and degree-5 homogeneity, so seven numbers suffice. They are obtained here from the
// self-similarity of the cube: splitting both unit cubes of an equal-size class into 8 half
// cubes gives 64 half-size pairs, each 1/32 of a unit pair at integer offset 2o + d - c, so
//
//     32 C_o = sum_{c, d in {0,1}^3} J(2o + d - c),
//
// where J(delta) is one of the four equal-size class integrals when the unit cubes at offset
// delta touch and a regular integral otherwise. This is a 4x4 linear system for the self,
// face, edge and vertex classes. A side-2 cube is 8 unit cubes, so the three classes with
// sides 1:2 are sums of unit-pair integrals. The regular integrals use a 6-D Gauss-Legendre rule
// on the GPU (kernels.hip).
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace bcv {

// Gauss-Legendre nodes and weights on [0, 1] (Newton iteration on P_n in long double).
void gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        long double z = std::cos(3.141592653589793238462643383279502884L * (i + 0.75L) / (n + 0.5L));
        long double dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) p0 = 1.0L;
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            const long double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-19L) break;
        }
        // recompute the derivative at the converged node
        long double p0 = 1.0L, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0L);
        x[i] = (double)(0.5L * (1.0L - z));
        w[i] = (double)(1.0L / ((1.0L - z * z) * dp * dp));  // 2/((1-z^2)P'^2) scaled by 1/2
    }
}

namespace {

using Off = std::array<int, 3>;

Off canonical(const Off &d)  // symmetry of the cube pair: |d_i| sorted
{
    Off a = {std::abs(d[0]), std::abs(d[1]), std::abs(d[2])};
    std::sort(a.begin(), a.end());
    return a;
}

bool touches(const Off &d) { return std::abs(d[0]) <= 1 && std::abs(d[1]) <= 1 && std::abs(d[2]) <= 1; }

int contacts(const Off &d) { return (d[0] != 0) + (d[1] != 0) + (d[2] != 0); }

// Unit-pair offsets of one equation: the 64 half-cube pairs of class o (ratio 1), or the 8
// unit sub-cubes of the big cube against the unit cube (ratio 2, n_contact axes).
std::vector<Off> equal_class_terms(int n_contact)
{
    std::vector<Off> v;
    for (int c = 0; c < 8; ++c)
        for (int d = 0; d < 8; ++d) {
            Off o;
            for (int ax = 0; ax < 3; ++ax)
                o[ax] = 2 * (ax < n_contact ? 1 : 0) + ((d >> ax) & 1) - ((c >> ax) & 1);
            v.push_back(o);
        }
    return v;
}

std::vector<Off> ratio2_terms(int n_contact)
{
    std::vector<Off> v;
    for (int c = 0; c < 8; ++c) {
        Off o;  // unit cube [0,1]^3 minus sub-cube lower corner (-2 on contact axes) + c
        for (int ax = 0; ax < 3; ++ax) o[ax] = -((ax < n_contact ? -2 : 0) + ((c >> ax) & 1));
        v.push_back(o);
    }
    return v;
}

void compute(int device, double out[kTouchClasses])
{
    BCV_HIP(hipSetDevice(device));
    std::map<Off, double> regular;
    for (int k = 0; k < 4; ++k)
        for (const Off &o : equal_class_terms(k))
            if (!touches(o)) regular[canonical(o)] = 0.0;
    for (int k = 1; k <= 3; ++k)
        for (const Off &o : ratio2_terms(k))
            if (!touches(o)) regular[canonical(o)] = 0.0;
    std::vector<int> deltas;
    for (const auto &kv : regular) deltas.insert(deltas.end(), kv.first.begin(), kv.first.end());
    std::vector<double> vals(regular.size());
    regular_cube_pairs(deltas.data(), (int)regular.size(), 12, vals.data());
    size_t n = 0;
    for (auto &kv : regular) kv.second = vals[n++];

    // 32 C_k - sum_{touching terms} C_{contacts} = sum_{regular terms} J, k = 0..3.
    double A[4][5] = {};
    for (int k = 0; k < 4; ++k) {
        A[k][k] += 32.0;
        for (const Off &o : equal_class_terms(k)) {
            if (touches(o))
                A[k][contacts(o)] -= 1.0;
            else
                A[k][4] += regular[canonical(o)];
        }
    }
    for (int col = 0; col < 4; ++col) {  // Gaussian elimination with partial pivoting
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
        for (int c2 = 0; c2 < 5; ++c2) std::swap(A[col][c2], A[piv][c2]);
        for (int r = 0; r < 4; ++r) {
            if (r == col) continue;
            const double f = A[r][col] / A[col][col];
            for (int c2 = col; c2 < 5; ++c2) A[r][c2] -= f * A[col][c2];
        }
    }
    double C[4];
    for (int k = 0; k < 4; ++k) C[k] = A[k][4] / A[k][k];
    for (int k = 0; k < 4; ++k) out[k] = C[k];
    for (int k = 1; k <= 3; ++k) {
        double s = 0.0;
        for (const Off &o : ratio2_terms(k)) s += touches(o) ? C[contacts(o)] : regular[canonical(o)];
        out[3 + k] = s;
    }
}

}  // namespace

void touching_integrals(int device, double out[kTouchClasses])
{
    static std::mutex mu;
    static std::map<int, std::array<double, kTouchClasses>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(device);
    if (it == cache.end()) {
        std::array<double, kTouchClasses> v{};
        compute(device, v.data());
        it = cache.emplace(device, v).first;
    }
    std::copy(it->second.begin(), it->second.end(), out);
}

}  // namespace bcv
