// High-order quadrature of the Galerkin integral of 1/|x - y| over two axis-aligned boxes.
//
// This generates the training data of the touching-pair surrogate and checks its predictions
// (Sec. 3 computes singular near-field entries with singularity-removing transforms followed by
// tensor Gauss rules; this is a scheme of the same kind for boxes). With u = x - y,
//
//     int_A int_B 1/|x - y| dy dx = int_{R^3} prod_i c_i(u_i) / |u| du,
//     c_i(u) = | [alo_i, ahi_i] cap [blo_i + u, bhi_i + u] |,
//
// and c_i is piecewise linear with kinks at alo-bhi, alo-blo, ahi-bhi, ahi-blo. Splitting each
// axis at the kinks (and at 0) gives a lattice of cells on which the numerator is a polynomial and
// the origin, the only singular point, is a lattice vertex. Cells with the origin as a corner are
// cut to aspect ratio <= 2 and mapped by the three Duffy pyramids (the Jacobian t^2 cancels 1/|u|);
// every other cell is halved along its longest side until that side is no longer than its distance
// to the origin, and then takes a tensor Gauss-Legendre rule. All in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "quadrature.hpp"

namespace bcv {

void gauss_legendre01(int n, double *x, double *w);

namespace {

constexpr int kQThreads = 256;
constexpr int kQMaxBoxes = 768;
constexpr int kQStack = 96;

struct QRule {
    double x[kQMaxGauss], w[kQMaxGauss];
    int n;
};

struct QBox {
    double lo[3], hi[3];
    int duffy;  // 1: the origin is a corner (Duffy pyramids), 0: regular tensor rule
};

__device__ __forceinline__ double overlap(double u, double alo, double ahi, double blo, double bhi)
{
    return fmax(0.0, fmin(ahi, bhi + u) - fmax(alo, blo + u));
}

__device__ __forceinline__ double numerator(const double u[3], const double *g)  // g: alo, ahi, blo, bhi (3 each)
{
    return overlap(u[0], g[0], g[3], g[6], g[9]) * overlap(u[1], g[1], g[4], g[7], g[10]) *
           overlap(u[2], g[2], g[5], g[8], g[11]);
}

// Work space of the list builder (LDS; used by one thread).
struct QScratch {
    double br[3][5], v[5];
    int nb[3];
    QBox stack[kQStack];
};

// Builds the cell list of one pair (one thread). Returns the number of cells, or -1 if a list
// overflows.
__device__ int build_boxes(const double *g, QBox *out, QScratch &w)
{
    double(*br)[5] = w.br;
    int *nb = w.nb;
    for (int i = 0; i < 3; ++i) {
        const double alo = g[i], ahi = g[3 + i], blo = g[6 + i], bhi = g[9 + i];
        double *v = w.v;
        v[0] = alo - bhi, v[1] = ahi - blo, v[2] = alo - blo, v[3] = ahi - bhi, v[4] = 0.0;
        const int m = (alo - bhi < 0.0 && 0.0 < ahi - blo) ? 5 : 4;
        for (int a = 1; a < m; ++a)  // insertion sort
            for (int b = a; b > 0 && v[b] < v[b - 1]; --b) {
                const double t = v[b];
                v[b] = v[b - 1];
                v[b - 1] = t;
            }
        int k = 0;
        for (int a = 0; a < m; ++a)
            if (k == 0 || v[a] != br[i][k - 1]) br[i][k++] = v[a];
        nb[i] = k;
    }
    QBox *stack = w.stack;
    int sp = 0, n = 0;
    for (int ix = 0; ix + 1 < nb[0]; ++ix)
        for (int iy = 0; iy + 1 < nb[1]; ++iy)
            for (int iz = 0; iz + 1 < nb[2]; ++iz) {
                QBox b;
                b.lo[0] = br[0][ix], b.hi[0] = br[0][ix + 1];
                b.lo[1] = br[1][iy], b.hi[1] = br[1][iy + 1];
                b.lo[2] = br[2][iz], b.hi[2] = br[2][iz + 1];
                b.duffy = 0;
                // skip cells where the numerator vanishes (outside the support of some c_i)
                const double mid[3] = {0.5 * (b.lo[0] + b.hi[0]), 0.5 * (b.lo[1] + b.hi[1]), 0.5 * (b.lo[2] + b.hi[2])};
                if (numerator(mid, g) <= 0.0) continue;
                if (sp == kQStack) return -1;
                stack[sp++] = b;
                while (sp > 0) {
                    QBox c = stack[--sp];
                    double s[3], smax = 0.0, smin = 1e300, d2 = 0.0;
                    int jmax = 0;
                    bool corner = true;
                    for (int i = 0; i < 3; ++i) {
                        s[i] = c.hi[i] - c.lo[i];
                        if (s[i] > smax) smax = s[i], jmax = i;
                        smin = fmin(smin, s[i]);
                        const double di = c.lo[i] > 0.0 ? c.lo[i] : (c.hi[i] < 0.0 ? -c.hi[i] : 0.0);
                        d2 += di * di;
                        corner = corner && (c.lo[i] == 0.0 || c.hi[i] == 0.0);
                    }
                    QBox p = c, q = c;  // the two halves if c is split
                    if (corner) {
                        if (smax <= 2.0 * smin) {
                            if (n == kQMaxBoxes) return -1;
                            c.duffy = 1;
                            out[n++] = c;
                            continue;
                        }
                        // cut the longest side at 2 * smin from the origin
                        const double cut = c.lo[jmax] == 0.0 ? 2.0 * smin : -2.0 * smin;
                        if (c.lo[jmax] == 0.0) p.hi[jmax] = cut, q.lo[jmax] = cut;
                        else p.lo[jmax] = cut, q.hi[jmax] = cut;
                    } else {
                        if (smax * smax <= d2) {
                            if (n == kQMaxBoxes) return -1;
                            out[n++] = c;
                            continue;
                        }
                        const double mid_j = 0.5 * (c.lo[jmax] + c.hi[jmax]);
                        p.hi[jmax] = mid_j;
                        q.lo[jmax] = mid_j;
                    }
                    if (sp + 2 > kQStack) return -1;
                    stack[sp++] = p;
                    stack[sp++] = q;
                }
            }
    return n;
}

// One block per pair: thread 0 lists the cells, all threads share the quadrature points.
__global__ __launch_bounds__(kQThreads) void box_pair_kernel(int64_t n_pairs, const double *__restrict__ geom,
                                                             QRule rule, double *__restrict__ out)
{
    __shared__ QBox boxes[kQMaxBoxes];
    __shared__ QScratch scratch;
    __shared__ int n_boxes;
    __shared__ double part[kQThreads];
    __shared__ double g[12];
    const int64_t pair = blockIdx.x;
    if (pair >= n_pairs) return;
    if (threadIdx.x < 12) g[threadIdx.x] = geom[pair * 12 + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) n_boxes = build_boxes(g, boxes, scratch);
    __syncthreads();
    const int n = rule.n, n3 = n * n * n;
    double acc = 0.0;
    for (int b = 0; b < n_boxes; ++b) {
        const QBox c = boxes[b];
        const double h[3] = {c.hi[0] - c.lo[0], c.hi[1] - c.lo[1], c.hi[2] - c.lo[2]};
        if (!c.duffy) {
            for (int p = threadIdx.x; p < n3; p += kQThreads) {
                const int i0 = p % n, i1 = (p / n) % n, i2 = p / (n * n);
                const double u[3] = {c.lo[0] + h[0] * rule.x[i0], c.lo[1] + h[1] * rule.x[i1],
                                     c.lo[2] + h[2] * rule.x[i2]};
                const double r = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                acc += rule.w[i0] * rule.w[i1] * rule.w[i2] * h[0] * h[1] * h[2] * numerator(u, g) / r;
            }
        } else {
            // u = sigma * v, v in [0, h]^3; pyramid k: v_k = h_k t, v_j = h_j t s_j (j != k)
            const double sg[3] = {c.lo[0] == 0.0 ? 1.0 : -1.0, c.lo[1] == 0.0 ? 1.0 : -1.0,
                                  c.lo[2] == 0.0 ? 1.0 : -1.0};
            for (int p = threadIdx.x; p < 3 * n3; p += kQThreads) {
                const int k = p / n3, q = p % n3;
                const int it = q % n, i1 = (q / n) % n, i2 = q / (n * n);
                const int j1 = (k + 1) % 3, j2 = (k + 2) % 3;
                const double t = rule.x[it], s1 = rule.x[i1], s2 = rule.x[i2];
                double u[3];
                u[k] = sg[k] * h[k] * t;
                u[j1] = sg[j1] * h[j1] * t * s1;
                u[j2] = sg[j2] * h[j2] * t * s2;
                const double rho = sqrt(h[k] * h[k] + h[j1] * h[j1] * s1 * s1 + h[j2] * h[j2] * s2 * s2);
                acc += rule.w[it] * rule.w[i1] * rule.w[i2] * h[0] * h[1] * h[2] * numerator(u, g) * t / rho;
            }
        }
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kQThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[pair] = n_boxes < 0 ? nan("") : part[0];
}

}  // namespace

void box_pair_integrals_device(int64_t n, const double *geom_dev, int n_gauss, double *out_dev, hipStream_t st)
{
    BCV_REQUIRE(n_gauss >= 1 && n_gauss <= kQMaxGauss, BCV_EINVAL, "Gauss order must be 1..16");
    if (n == 0) return;
    QRule rule;
    gauss_legendre01(n_gauss, rule.x, rule.w);
    rule.n = n_gauss;
    box_pair_kernel<<<(unsigned)n, kQThreads, 0, st>>>(n, geom_dev, rule, out_dev);
    BCV_HIP(hipGetLastError());
}

void box_pair_integrals(int device, int64_t n, const double *geom_host, int n_gauss, double *out_host)
{
    BCV_REQUIRE(n >= 0, BCV_EINVAL, "negative pair count");
    BCV_HIP(hipSetDevice(device));
    double *d_geom = nullptr, *d_out = nullptr;
    const size_t gb = (size_t)std::max<int64_t>(n, 1) * 12 * sizeof(double), ob = (size_t)std::max<int64_t>(n, 1) * sizeof(double);
    if (hipMalloc(&d_geom, gb) != hipSuccess) fail(BCV_ENOMEM, "hipMalloc failed");
    if (hipMalloc(&d_out, ob) != hipSuccess) {
        (void)hipFree(d_geom);
        fail(BCV_ENOMEM, "hipMalloc failed");
    }
    try {
        BCV_HIP(hipMemcpy(d_geom, geom_host, (size_t)n * 12 * sizeof(double), hipMemcpyHostToDevice));
        box_pair_integrals_device(n, d_geom, n_gauss, d_out, nullptr);
        BCV_HIP(hipMemcpy(out_host, d_out, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    } catch (...) {
        (void)hipFree(d_geom);
        (void)hipFree(d_out);
        throw;
    }
    (void)hipFree(d_geom);
    (void)hipFree(d_out);
}

}  // namespace bcv
