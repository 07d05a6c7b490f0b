// Exact single- and double-layer integrals of touching (cell, boundary face) pairs, for the near
// field of the BtV calculation (Algorithm 3).
//
// A boundary face is a face of a level-L cell lying on the boundary of the unit cube, and every
// cell that meets it is a level-L leaf of the same size a (a cell meeting the boundary has a face
// on it and is refined down to level L). So a touching pair is a cube [0, 1]^3 (in units of a)
// and the face, normal to axis `ax` on the low (side 0) or high (side 1) end, of the cube at
// integer offset o in {-1, 0, 1}^3 that meets it: 108 configurations. Their integrals
//
//     V = int_cube int_face 1 / (4 pi |x - y|) dS_y dx              (degree-4 homogeneous)
//     K = int_cube int_face n . (x - y) / (4 pi |x - y|^3) dS_y dx    (degree-3 homogeneous)
//
// follow from self-similarity: halving the cube into 8 cubes and the face into 4 faces gives 32
// half-size pairs; a half-size pair that touches is one of the 108 configurations scaled by 2^-4
// (V) or 2^-3 (K), and one that does not is a regular 5-D integral. So
//
//     V_c - 2^-4 sum_{touching sub-pairs} V_c' = sum_{regular sub-pairs} V   (likewise K, 2^-3),
//
// a 108 x 108 linear system whose touching-count matrix has spectral radius 4, well below 8 and
// 16. The regular integrals use a tensor Gauss-Legendre rule (10 points per dimension; the
// closest regular sub-pairs are one half-cell apart).
#include <array>
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace bcv {

void gauss_legendre01(int n, double *x, double *w);

namespace {

constexpr double kInv4Pi = 0.079577471545947667884;

struct FaceConfig {
    int o[3];
    int ax, side;
};

// Closed unit cube [0,1]^3 against the face of the unit cube at offset o: do they meet?
bool meets(const int o[3], int ax, int side)
{
    for (int d = 0; d < 3; ++d) {
        const int lo = d == ax ? o[d] + side : o[d], hi = d == ax ? o[d] + side : o[d] + 1;
        if (std::max(lo, 0) > std::min(hi, 1)) return false;
    }
    return true;
}

// Regular integral (V or K, without the 1/(4 pi)) of the cube [c, c + s]^3 against the face of the
// cube at fc (side s) normal to ax on `side`, by an n-point tensor Gauss rule.
void regular_pair(const double c[3], const double fc[3], double s, int ax, int side, int n, const double *x,
                  const double *w, double &V, double &K)
{
    const int o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
    const double sign = 2.0 * side - 1.0, plane = fc[ax] + side * s;
    double sv = 0.0, sk = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                const double p[3] = {c[0] + s * x[i], c[1] + s * x[j], c[2] + s * x[k]};
                const double wp = w[i] * w[j] * w[k];
                double tv = 0.0, tk = 0.0;
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) {
                        double d[3];
                        d[ax] = p[ax] - plane;
                        d[o1] = p[o1] - (fc[o1] + s * x[a]);
                        d[o2] = p[o2] - (fc[o2] + s * x[b]);
                        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        const double ir = 1.0 / std::sqrt(r2);
                        tv += w[a] * w[b] * ir;
                        tk += w[a] * w[b] * sign * d[ax] * ir * ir * ir;
                    }
                sv += wp * tv;
                sk += wp * tk;
            }
    const double jac = s * s * s * s * s;
    V = sv * jac;
    K = sk * jac;
}

void solve(std::vector<double> &A, std::vector<double> &b, int n)  // Gaussian elimination, partial pivoting
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + col]) > std::fabs(A[(size_t)piv * n + col])) piv = r;
        if (piv != col) {
            for (int c2 = 0; c2 < n; ++c2) std::swap(A[(size_t)col * n + c2], A[(size_t)piv * n + c2]);
            std::swap(b[col], b[piv]);
        }
        for (int r = col + 1; r < n; ++r) {
            const double f = A[(size_t)r * n + col] / A[(size_t)col * n + col];
            if (f == 0.0) continue;
            for (int c2 = col; c2 < n; ++c2) A[(size_t)r * n + c2] -= f * A[(size_t)col * n + c2];
            b[r] -= f * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c2 = r + 1; c2 < n; ++c2) s -= A[(size_t)r * n + c2] * b[c2];
        b[r] = s / A[(size_t)r * n + r];
    }
}

void compute(double *V_out, double *K_out)
{
    std::vector<FaceConfig> cfg;
    std::array<int, kFaceClasses> index;
    index.fill(-1);
    for (int ax = 0; ax < 3; ++ax)
        for (int o0 = -1; o0 <= 1; ++o0)
            for (int o1 = -1; o1 <= 1; ++o1)
                for (int o2 = -1; o2 <= 1; ++o2)
                    for (int side = 0; side < 2; ++side) {
                        const int o[3] = {o0, o1, o2};
                        if (!meets(o, ax, side)) continue;
                        index[face_class(o, ax, side)] = (int)cfg.size();
                        cfg.push_back(FaceConfig{{o0, o1, o2}, ax, side});
                    }
    const int n = (int)cfg.size();
    constexpr int kGauss = 10;
    double x[kGauss], w[kGauss];
    gauss_legendre01(kGauss, x, w);
    std::vector<double> AV((size_t)n * n, 0.0), AK((size_t)n * n, 0.0), bV(n, 0.0), bK(n, 0.0);
    bool ok = true;
#pragma omp parallel for schedule(dynamic, 1) reduction(&& : ok)
    for (int i = 0; i < n; ++i) {
        const FaceConfig &f = cfg[i];
        const int o1 = (f.ax + 1) % 3, o2 = (f.ax + 2) % 3;
        AV[(size_t)i * n + i] += 1.0;
        AK[(size_t)i * n + i] += 1.0;
        for (int c = 0; c < 8; ++c)        // half cubes of the unit cube (half units: cube at cc, side 1)
            for (int h = 0; h < 4; ++h) {  // half faces
                const int cc[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
                int fc[3];
                fc[f.ax] = 2 * f.o[f.ax] + f.side;  // the half cube whose `side` face holds the half face
                fc[o1] = 2 * f.o[o1] + (h & 1);
                fc[o2] = 2 * f.o[o2] + (h >> 1);
                const int rel[3] = {fc[0] - cc[0], fc[1] - cc[1], fc[2] - cc[2]};
                const bool near = std::abs(rel[0]) <= 1 && std::abs(rel[1]) <= 1 && std::abs(rel[2]) <= 1;
                if (near && meets(rel, f.ax, f.side)) {
                    const int j = index[face_class(rel, f.ax, f.side)];
                    ok = ok && j >= 0;
                    if (j >= 0) {
                        AV[(size_t)i * n + j] -= 1.0 / 16.0;
                        AK[(size_t)i * n + j] -= 1.0 / 8.0;
                    }
                } else {
                    // the sub-pair in unit-cube coordinates: half cube at cc/2, half face of the cube at fc/2
                    const double c0[3] = {0.5 * cc[0], 0.5 * cc[1], 0.5 * cc[2]};
                    const double f0[3] = {0.5 * fc[0], 0.5 * fc[1], 0.5 * fc[2]};
                    double V, K;
                    regular_pair(c0, f0, 0.5, f.ax, f.side, kGauss, x, w, V, K);
                    bV[i] += V;
                    bK[i] += K;
                }
            }
    }
    if (!ok) fail(BCV_ESTATE, "internal: boundary touching configuration missing");
    solve(AV, bV, n);
    solve(AK, bK, n);
    for (int c = 0; c < kFaceClasses; ++c) {
        V_out[c] = index[c] >= 0 ? bV[index[c]] * kInv4Pi : 0.0;
        K_out[c] = index[c] >= 0 ? bK[index[c]] * kInv4Pi : 0.0;
    }
}

}  // namespace

void boundary_touching_integrals(double V[kFaceClasses], double K[kFaceClasses])
{
    static std::mutex mu;
    static bool done = false;
    static std::array<double, kFaceClasses> sv, sk;
    std::lock_guard<std::mutex> lock(mu);
    if (!done) {
        compute(sv.data(), sk.data());
        done = true;
    }
    std::copy(sv.begin(), sv.end(), V);
    std::copy(sk.begin(), sk.end(), K);
}

}  // namespace bcv
