// Mapped (curved) meshes: the BC octree of the reference cube pushed through the cube-to-ball map
// (ballmap.hpp). Algorithm 1 is unchanged in structure (same near and interaction lists, decided on
// the reference cubes), but the cells are curved:
//   * a cell's expansion centre is the image of its reference centre, so the translations of Sec. 3
//     act between arbitrary centres: M2M and L2L take each child's own shift, and the interaction
//     phase computes the derivatives of G for every (target, source) pair from the pair's offset
//     (m2l_pairs_kernel) instead of reading a table per lattice offset;
//   * P2M and the evaluation use each leaf's own moment row kappa_w^b = sum_g w_g ((x_g - x_w)/a)^b / b!
//     over its 2x2x2 mapped Gauss points x_g = Phi(xi_g) with weights w_g = (a^3 / 8) J(xi_g);
//   * the near field is assembled at plan time: non-touching pairs by the mapped point rule, touching
//     pairs (the closed reference cubes meet) by a singular rule in the relative coordinate
//     (ball_touch_kernel).
// Cube meshes of a forest that also holds ball meshes take the same kernels with the identity map;
// their touching entries keep the exact class values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <utility>

#include "ballmap.hpp"
#include "internal.hpp"
#include "kernels.hpp"
#include "multiindex.hpp"

namespace bcv {

void gauss_legendre01(int n, double *x, double *w);

namespace {

void check_launch()
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(BCV_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
}

constexpr int kW = 64;
constexpr double kInv4PiM = 0.079577471545947667884;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum_m(double v)
{
#pragma unroll
    for (int off = kW / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kW);
    return v;
}

// Tables read with indices known only at run time live in constant memory.
template <int Q>
__constant__ constexpr MultiIndex<Q> kMiM{};
template <int Q>
__constant__ constexpr FoldTable<Q> kFoldM{};
template <int Q>
__constant__ constexpr ExpandTable<Q> kExM{};

// Degree of the graded position j (|b| of the multi-index at position j).
__device__ __forceinline__ int degree_of(int j)
{
    int d = 0;
    while ((d + 1) * (d + 2) * (d + 3) / 6 <= j) ++d;
    return d;
}

// ---- near-field entries ----------------------------------------------------------------------------
// Non-touching entries of mapped target leaves: sum over the 8 x 8 mapped points (x, y, z, weight).
// Touching entries are left to ball_touch_kernel. One wave per near unit.
__global__ __launch_bounds__(256) void mapped_assemble_kernel(int64_t n_units, const NearUnit *__restrict__ units,
                                                              const uint32_t *__restrict__ col,
                                                              const double4 *__restrict__ pts,
                                                              const uint8_t *__restrict__ leaf_mapped,
                                                              double *__restrict__ val)
{
    const int lane = threadIdx.x & (kW - 1);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kW) + (threadIdx.x / kW);
    if (w >= n_units) return;
    const NearUnit un = units[w];
    const int32_t t = un.target;
    if (!leaf_mapped[t]) return;  // uniform per wave
    double4 pt[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) pt[g] = pts[8 * (int64_t)t + g];
    for (int64_t e = un.begin + lane; e < un.end; e += kW) {
        const uint32_t c = col[e];
        if (c >> 28) continue;
        const int32_t s = (int32_t)(c & 0x0FFFFFFFu);
        double acc = 0.0;
        for (int h = 0; h < 8; ++h) {
            const double4 ps = pts[8 * (int64_t)s + h];
            double in = 0.0;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const double dx = pt[g].x - ps.x, dy = pt[g].y - ps.y, dz = pt[g].z - ps.z;
                in = fma(pt[g].w, 1.0 / sqrt(dx * dx + dy * dy + dz * dz), in);
            }
            acc = fma(ps.w, in, acc);
        }
        val[e] = acc * kInv4PiM;
    }
}

// Gauss-Legendre rules on [0, 1] of the singular rule: lambda (radial Duffy variable), mu (the two
// Duffy directions), z (relative-coordinate boxes away from the singularity), s (the inner box), r
// (regular sub-pairs of a ratio-2 pair).
constexpr int kRuleMax = 8;
struct SingRule {
    double xl[kRuleMax], wl[kRuleMax], xm[kRuleMax], wm[kRuleMax], xz[kRuleMax], wz[kRuleMax], xs[kRuleMax],
        ws[kRuleMax], xr[kRuleMax], wr[kRuleMax];
    int nl, nm, nz, ns, nr;
};

// G(Phi(lo_t + a s), Phi(lo_s + a t)) J J over the inner box B(z) of the relative coordinate z:
// s in [0,1]^3 with s + z - delta in [0,1]^3, by the n_s^3 tensor rule (a box whose ends are linear
// in z on each of the 8 unit boxes of z).
__device__ double inner_box(const double *lo_t, const double *lo_s, double a, const int *delta, const double *z,
                            const SingRule &R)
{
    double b0[3], len[3];
    for (int i = 0; i < 3; ++i) {
        const double lo = fmax(0.0, delta[i] - z[i]);
        const double hi = fmin(1.0, 1.0 + delta[i] - z[i]);
        b0[i] = lo;
        len[i] = hi - lo;
    }
    if (len[0] <= 0.0 || len[1] <= 0.0 || len[2] <= 0.0) return 0.0;
    double sum = 0.0;
    for (int c = 0; c < R.ns; ++c)
        for (int b = 0; b < R.ns; ++b)
            for (int q = 0; q < R.ns; ++q) {
                const double s[3] = {b0[0] + len[0] * R.xs[q], b0[1] + len[1] * R.xs[b], b0[2] + len[2] * R.xs[c]};
                double x[3], y[3], px[3], py[3], jx, jy;
                for (int i = 0; i < 3; ++i) {
                    x[i] = lo_t[i] + a * s[i];
                    y[i] = lo_s[i] + a * (s[i] + z[i] - delta[i]);
                }
                ball_map(x, px, &jx);
                ball_map(y, py, &jy);
                const double dx = px[0] - py[0], dy = px[1] - py[1], dz = px[2] - py[2];
                sum += R.ws[q] * R.ws[b] * R.ws[c] * jx * jy / sqrt(dx * dx + dy * dy + dz * dz);
            }
    return sum * len[0] * len[1] * len[2];
}

// This thread's share of the singular rule for two touching cubes of equal side a (reference
// coordinates of the mesh, lower corners lo_t and lo_s): z = delta + t - s runs over the 8 unit boxes
// [g_i, g_i + 1] (g_i = delta_i - 1 or delta_i); a box with z = 0 as a corner is split into 3 Duffy
// pyramids (|z_k| = lambda largest, the others lambda mu_1, lambda mu_2, weight lambda^2), the others
// take the n_z^3 tensor rule. Without the factor a^6 / (4 pi).
__device__ double touch_same_part(const double *lo_t, const double *lo_s, double a, const SingRule &R, int tid,
                                  int nthreads)
{
    int delta[3];
    for (int i = 0; i < 3; ++i) delta[i] = (int)rint((lo_s[i] - lo_t[i]) / a);
    const int n_corner = 3 * R.nl * R.nm * R.nm, n_far = R.nz * R.nz * R.nz;
    int count[8];
    int total = 0, corners = 0;  // bit box: the box has z = 0 as a corner
    for (int box = 0; box < 8; ++box) {
        bool corner = true;
        for (int i = 0; i < 3; ++i) {
            const int g0 = ((box >> i) & 1) ? delta[i] : delta[i] - 1;
            corner = corner && (g0 == 0 || g0 == -1);
        }
        corners |= corner ? 1 << box : 0;
        count[box] = corner ? n_corner : n_far;
        total += count[box];
    }
    double sum = 0.0;
    for (int o = tid; o < total; o += nthreads) {
        int box = 0, r = o;
        while (r >= count[box]) r -= count[box++];
        double g0[3], sg[3];
        for (int i = 0; i < 3; ++i) {
            g0[i] = ((box >> i) & 1) ? delta[i] : delta[i] - 1;
            sg[i] = g0[i] == 0.0 ? 1.0 : -1.0;
        }
        double z[3], wgt;
        if ((corners >> box) & 1) {
            const int k = r / (R.nl * R.nm * R.nm);
            int rr = r - k * R.nl * R.nm * R.nm;
            const int il = rr / (R.nm * R.nm);
            rr -= il * R.nm * R.nm;
            const int i1 = rr / R.nm, i2 = rr - i1 * R.nm;
            const int j1 = k == 2 ? 0 : k + 1, j2 = k == 0 ? 2 : k - 1;
            const double lam = R.xl[il];
            z[k] = sg[k] * lam;
            z[j1] = sg[j1] * lam * R.xm[i1];
            z[j2] = sg[j2] * lam * R.xm[i2];
            wgt = R.wl[il] * R.wm[i1] * R.wm[i2] * lam * lam;
        } else {
            const int q = r % R.nz, b = (r / R.nz) % R.nz, c = r / (R.nz * R.nz);
            z[0] = g0[0] + R.xz[q];
            z[1] = g0[1] + R.xz[b];
            z[2] = g0[2] + R.xz[c];
            wgt = R.wz[q] * R.wz[b] * R.wz[c];
        }
        sum += wgt * inner_box(lo_t, lo_s, a, delta, z, R);
    }
    return sum;
}

// This thread's share of the n_r^3 x n_r^3 tensor rule on two cubes of side a. Without a^6 / (4 pi).
__device__ double regular_part(const double *lo_t, const double *lo_s, double a, const SingRule &R, int tid,
                               int nthreads)
{
    const int n3 = R.nr * R.nr * R.nr;
    double sum = 0.0;
    for (int o = tid; o < n3 * n3; o += nthreads) {
        const int i = o / n3, m = o - i * n3;
        const int i0 = i % R.nr, i1 = (i / R.nr) % R.nr, i2 = i / (R.nr * R.nr);
        const int m0 = m % R.nr, m1 = (m / R.nr) % R.nr, m2 = m / (R.nr * R.nr);
        const double x[3] = {lo_t[0] + a * R.xr[i0], lo_t[1] + a * R.xr[i1], lo_t[2] + a * R.xr[i2]};
        const double y[3] = {lo_s[0] + a * R.xr[m0], lo_s[1] + a * R.xr[m1], lo_s[2] + a * R.xr[m2]};
        double px[3], py[3], jx, jy;
        ball_map(x, px, &jx);
        ball_map(y, py, &jy);
        const double dx = px[0] - py[0], dy = px[1] - py[1], dz = px[2] - py[2];
        sum += R.wr[i0] * R.wr[i1] * R.wr[i2] * R.wr[m0] * R.wr[m1] * R.wr[m2] * jx * jy /
               sqrt(dx * dx + dy * dy + dz * dz);
    }
    return sum;
}

// This thread's share of the singular rule for the touching cubes (lower corner, side) t and s of one
// mesh's reference cube, without the factor a^6 / (4 pi) (a the smaller side, returned): equal sides,
// the rule above; sides in ratio 2, the larger cube's 8 children against the smaller one, by the rule
// where they touch and the tensor rule elsewhere.
__device__ double pair_part(const double *lt, double at, const double *ls, double as, const SingRule &R, int tid,
                            int nthreads, double *a_small)
{
    double sum = 0.0;
    if (at == as) {
        *a_small = at;
        return touch_same_part(lt, ls, at, R, tid, nthreads);
    }
    const bool big_t = at > as;
    const double a = big_t ? as : at;
    *a_small = a;
    const double *lb = big_t ? lt : ls, *lm = big_t ? ls : lt;
    for (int c = 0; c < 8; ++c) {
        const double lc[3] = {lb[0] + a * (c & 1), lb[1] + a * ((c >> 1) & 1), lb[2] + a * ((c >> 2) & 1)};
        bool touch = true;
        for (int i = 0; i < 3; ++i) touch = touch && fmax(lc[i], lm[i]) <= fmin(lc[i] + a, lm[i] + a);
        const double *pt = big_t ? lc : lm, *ps = big_t ? lm : lc;
        sum += touch ? touch_same_part(pt, ps, a, R, tid, nthreads) : regular_part(pt, ps, a, R, tid, nthreads);
    }
    return sum;
}

// Sum of the block's shares (256 threads), times a^6 / (4 pi), in thread 0.
__device__ double block_entry(double part, double a, double *red)
{
    red[threadIdx.x] = part;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double a3 = a * a * a;
    const double v = red[0] * a3 * a3 * kInv4PiM;
    __syncthreads();
    return v;
}

// Touching entries of mapped leaves: one block per listed entry (its index, target leaf and the
// index of its mirror (s, t) or -1, written with the same value: the rule is symmetric); the source
// comes from the entry's column. Geometry: lower corners and sides of the leaves in the forest's
// reference frame (mesh m in [4m, 4m + 1) x [0,1)^2); the map acts on the mesh's own reference cube.
__global__ __launch_bounds__(256) void ball_touch_kernel(int64_t n, const int64_t *__restrict__ entry,
                                                         const int32_t *__restrict__ target,
                                                         const int64_t *__restrict__ mirror,
                                                         const uint32_t *__restrict__ col,
                                                         const double4 *__restrict__ geom, SingRule R,
                                                         double *__restrict__ val)
{
    __shared__ double red[256];
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        const int64_t e = entry[k];
        const int32_t t = target[k], s = (int32_t)(col[e] & 0x0FFFFFFFu);
        const double4 gt = geom[t], gs = geom[s];
        const double shift = 4.0 * floor(gt.x * 0.25);  // the mesh's offset along x
        const double lt[3] = {gt.x - shift, gt.y, gt.z}, ls[3] = {gs.x - shift, gs.y, gs.z};
        double a;
        const double part = pair_part(lt, gt.w, ls, gs.w, R, threadIdx.x, blockDim.x, &a);
        const double v = block_entry(part, a, red);
        if (threadIdx.x == 0) {
            val[e] = v;
            if (mirror[k] >= 0) val[mirror[k]] = v;
        }
    }
}

// The same rule on explicit pairs: pair k is the cube (gt[k].xyz, gt[k].w) against (gs[k].xyz,
// gs[k].w) of the reference cube [0,1]^3.
__global__ __launch_bounds__(256) void ball_pair_kernel(int64_t n, const double4 *__restrict__ gt,
                                                        const double4 *__restrict__ gs, SingRule R,
                                                        double *__restrict__ out)
{
    __shared__ double red[256];
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        const double4 t = gt[k], s = gs[k];
        const double lt[3] = {t.x, t.y, t.z}, ls[3] = {s.x, s.y, s.z};
        double a;
        const double part = pair_part(lt, t.w, ls, s.w, R, threadIdx.x, blockDim.x, &a);
        const double v = block_entry(part, a, red);
        if (threadIdx.x == 0) out[k] = v;
    }
}

SingRule make_rule(const int orders[5])
{
    SingRule R{};
    for (int k = 0; k < 5; ++k)
        BCV_REQUIRE(orders[k] >= 1 && orders[k] <= kRuleMax, BCV_EINVAL, "singular-rule orders: 1..8");
    R.nl = orders[0], R.nm = orders[1], R.nz = orders[2], R.ns = orders[3], R.nr = orders[4];
    gauss_legendre01(R.nl, R.xl, R.wl);
    gauss_legendre01(R.nm, R.xm, R.wm);
    gauss_legendre01(R.nz, R.xz, R.wz);
    gauss_legendre01(R.ns, R.xs, R.ws);
    gauss_legendre01(R.nr, R.xr, R.wr);
    return R;
}

// ---- P2M and evaluation from the leaves' moment rows -------------------------------------------
// M^b = f (-1)^|b| kappa^b (full rows, FP64) and the folded row Mr = f kappar (kappar: the folded,
// signed kappa). One thread per (leaf, j); K = ncoef(Q) is a compile-time constant, so splitting the
// thread index is a multiplication, not a 64-bit division.
template <int Q, class TR>
__global__ __launch_bounds__(256) void mapped_p2m_kernel(int64_t n_leaves, const int32_t *__restrict__ leaf_cell,
                                                         const double *__restrict__ kap,
                                                         const double *__restrict__ kapr,
                                                         const double *__restrict__ f, double *__restrict__ M,
                                                         TR *__restrict__ Mr, int ldk, int ldr)
{
    constexpr int K = ncoef(Q), R = (Q + 1) * (Q + 1);
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)n_leaves * K) return;
    const int64_t l = (int64_t)(i / K);
    const int j = (int)(i - (uint64_t)l * K);
    const int32_t c = leaf_cell[l];
    const double fl = f[l];
    const double v = fl * kap[i];
    M[(int64_t)c * ldk + j] = (degree_of(j) & 1) ? -v : v;
    if (j < R) Mr[(int64_t)c * ldr + j] = (TR)(fl * kapr[l * R + j]);
}

// u_w += sum_a kappa_w^a Lambda_w^a. 8 lanes per leaf: lane j of a group takes a = j, j + 8, ...
template <int Q>
__global__ __launch_bounds__(256) void mapped_eval_kernel(int64_t n_leaves, const int32_t *__restrict__ leaf_cell,
                                                          const double *__restrict__ kap,
                                                          const double *__restrict__ Lam, int ldk,
                                                          double *__restrict__ u)
{
    constexpr int K = ncoef(Q);
    const int64_t l = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int j = threadIdx.x & 7;
    double s = 0.0;
    if (l < n_leaves) {
        const double *__restrict__ lam = Lam + (int64_t)leaf_cell[l] * ldk;
        const double *__restrict__ kr = kap + l * K;
#pragma unroll
        for (int a = j; a < K; a += 8) s = fma(kr[a], lam[a], s);
    }
    s += __shfl_xor(s, 1, kW);
    s += __shfl_xor(s, 2, kW);
    s += __shfl_xor(s, 4, kW);
    if (l < n_leaves && j == 0) u[l] += s;
}

// val[entry[k]] <-> vals[k] (to_val: scatter the cached values; else gather them).
__global__ void touch_copy_kernel(int64_t n, const int64_t *__restrict__ entry, double *__restrict__ vals,
                                  double *__restrict__ val, int to_val)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        if (to_val)
            val[entry[k]] = vals[k];
        else
            vals[k] = val[entry[k]];
    }
}

__global__ void zero_kernel(int64_t n, double *__restrict__ u)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        u[i] = 0.0;
}

// ---- M2M and L2L with each child's own shift --------------------------------------------------------
// tau_c = (x_c - x_P) / a_P (arbitrary now). With the scaled coefficients
//   M2M  M_P^b  = sum_c sum_{g <= b} prod_i (-tau_ci)^(b_i - g_i)/(b_i - g_i)! 2^-g_i M_c^g
//   L2L  Lam_c^a = prod_i 2^-a_i sum_{b_i >= a_i} tau_ci^(b_i - a_i)/(b_i - a_i)! Lam_P^b
// Both are products of three 1-D operators that keep |b| <= Q, applied child by child: one pass
// per axis over the K coefficients (lane l takes l, l + 64, ...), each a sum of at most Q + 1 terms
// run as a fixed-length loop with the terms outside the range masked, so the lanes of a wave stay
// in step. One wave per marked cell; the rows and the 1-D factors in LDS.
constexpr int kTreeWaves = 4;

// Scratch rows of one wave: the two ping-pong rows of the passes.
template <int Q>
struct PassRows {
    double r[2][ncoef(Q)];
};

// The terms of a lane's passes do not depend on the child, so their positions are worked out once
// per wave: code[ax][n][k] for the lane's n-th coefficient b = lane + 64 n, term k along axis ax, is
// (position of the term's row entry) << 4 | (the exponent the term scales by), or -1 out of range.
template <int Q>
struct PassCodes {
    static constexpr int NB = (ncoef(Q) + kW - 1) / kW;
    int code[3][NB][Q + 1];
};

// M2M: term k of b is in[b - k e_ax] times w[k] 2^-(b_ax - k), for k <= b_ax.
template <int Q>
__device__ __forceinline__ void m2m_codes(PassCodes<Q> &pc, int lane)
{
    constexpr auto &mi = kMiM<Q>;
#pragma unroll
    for (int n = 0; n < PassCodes<Q>::NB; ++n) {
        const int b = lane + kW * n;
        const int e0 = b < ncoef(Q) ? mi.e[b][0] : 0, e1 = b < ncoef(Q) ? mi.e[b][1] : 0,
                  e2 = b < ncoef(Q) ? mi.e[b][2] : 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int bx = ax == 0 ? e0 : (ax == 1 ? e1 : e2);
#pragma unroll
            for (int k = 0; k <= Q; ++k) {
                const int g = bx - k;  // the source's component along ax
                const int j = ax == 0 ? mi_index(g, e1, e2) : (ax == 1 ? mi_index(e0, g, e2) : mi_index(e0, e1, g));
                pc.code[ax][n][k] = b < ncoef(Q) && k <= bx ? (j << 4) | g : -1;
            }
        }
    }
}

// L2L: term k of a is in[a + k e_ax] times w[k] (the pass then scales by 2^-a_ax), for k <= Q - |a|.
template <int Q>
__device__ __forceinline__ void l2l_codes(PassCodes<Q> &pc, int lane)
{
    constexpr auto &mi = kMiM<Q>;
#pragma unroll
    for (int n = 0; n < PassCodes<Q>::NB; ++n) {
        const int a = lane + kW * n;
        const int e0 = a < ncoef(Q) ? mi.e[a][0] : 0, e1 = a < ncoef(Q) ? mi.e[a][1] : 0,
                  e2 = a < ncoef(Q) ? mi.e[a][2] : 0;
        const int room = Q - (e0 + e1 + e2);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int ea = ax == 0 ? e0 : (ax == 1 ? e1 : e2);
#pragma unroll
            for (int k = 0; k <= Q; ++k) {
                const int j = ax == 0 ? mi_index(e0 + k, e1, e2) : (ax == 1 ? mi_index(e0, e1 + k, e2) : mi_index(e0, e1, e2 + k));
                pc.code[ax][n][k] = a < ncoef(Q) && k <= room ? (j << 4) | ea : -1;
            }
        }
    }
}

// out[b] = sum_k w[k] 2^-(b_ax - k) in[b - k e_ax]   (M2M direction)
template <int Q, int AX>
__device__ __forceinline__ void m2m_pass(const double *in, double *out, const double *w, const PassCodes<Q> &pc,
                                         int lane)
{
#pragma unroll
    for (int n = 0; n < PassCodes<Q>::NB; ++n) {
        if (lane + kW * n >= ncoef(Q)) continue;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k <= Q; ++k) {
            const int code = pc.code[AX][n][k];
            if (code >= 0) acc = fma(ldexp(w[k], -(code & 15)), in[code >> 4], acc);
        }
        out[lane + kW * n] = acc;
    }
}

// out[a] = 2^-a_ax sum_k w[k] in[a + k e_ax]   (L2L direction)
template <int Q, int AX>
__device__ __forceinline__ void l2l_pass(const double *in, double *out, const double *w, const PassCodes<Q> &pc,
                                         int lane)
{
#pragma unroll
    for (int n = 0; n < PassCodes<Q>::NB; ++n) {
        if (lane + kW * n >= ncoef(Q)) continue;
        double acc = 0.0;
        int ea = 0;
#pragma unroll
        for (int k = 0; k <= Q; ++k) {
            const int code = pc.code[AX][n][k];
            if (code >= 0) {
                acc = fma(w[k], in[code >> 4], acc);
                ea = code & 15;
            }
        }
        out[lane + kW * n] = ldexp(acc, -ea);
    }
}

// 1-D factors of child c along ax: w[k] = (s tau)^k / k!, s = -1 (M2M) or +1 (L2L).
__device__ __forceinline__ void shift_factors(double *w, const double4 &cc, const double4 &cp, int ax, double sign, int q)
{
    const double d = ax == 0 ? cc.x - cp.x : (ax == 1 ? cc.y - cp.y : cc.z - cp.z);
    const double t = sign * d / cp.w;
    double v = 1.0;
    for (int k = 0; k <= q; ++k) {
        w[k] = v;
        v *= t / (k + 1);
    }
}

template <int Q, class TR>
__global__ __launch_bounds__(kW *kTreeWaves) void mapped_m2m_kernel(int n_par, const int32_t *__restrict__ parents,
                                                                     const double4 *__restrict__ centre,
                                                                     double *__restrict__ M, TR *__restrict__ Mr,
                                                                     int ldk, int ldr)
{
    constexpr int K = ncoef(Q), R = nreduced(Q);
    constexpr auto &fold = kFoldM<Q>;
    __shared__ double sm[kTreeWaves][8][K];
    __shared__ double pw[kTreeWaves][8][3][Q + 1];
    __shared__ PassRows<Q> rows[kTreeWaves];
    const int wv = threadIdx.x / kW, lane = threadIdx.x & (kW - 1);
    const int w = blockIdx.x * kTreeWaves + wv;
    if (w >= n_par) return;  // uniform per wave; only wave-level synchronisation below
    const int32_t par = parents[2 * w], first = parents[2 * w + 1];
    const double4 cp = centre[par];
    {
        constexpr int NL = (8 * K + kW - 1) / kW;
        double v[NL];  // every load issued before the first LDS store
#pragma unroll
        for (int n = 0; n < NL; ++n) {
            const int i = lane + kW * n;
            v[n] = i < 8 * K ? M[(int64_t)(first + i / K) * ldk + i % K] : 0.0;
        }
        if (lane < 24) shift_factors(pw[wv][lane / 3][lane % 3], centre[first + lane / 3], cp, lane % 3, -1.0, Q);
#pragma unroll
        for (int n = 0; n < NL; ++n)
            if (lane + kW * n < 8 * K) sm[wv][(lane + kW * n) / K][(lane + kW * n) % K] = v[n];
    }
    wave_sync();
    PassCodes<Q> pc;
    m2m_codes<Q>(pc, lane);
    double acc[(K + kW - 1) / kW] = {};
    for (int c = 0; c < 8; ++c) {
        m2m_pass<Q, 0>(sm[wv][c], rows[wv].r[0], pw[wv][c][0], pc, lane);
        wave_sync();
        m2m_pass<Q, 1>(rows[wv].r[0], rows[wv].r[1], pw[wv][c][1], pc, lane);
        wave_sync();
        m2m_pass<Q, 2>(rows[wv].r[1], rows[wv].r[0], pw[wv][c][2], pc, lane);
        wave_sync();
#pragma unroll
        for (int s = 0; s < (K + kW - 1) / kW; ++s)
            if (lane + s * kW < K) acc[s] += rows[wv].r[0][lane + s * kW];
        wave_sync();
    }
#pragma unroll
    for (int s = 0; s < (K + kW - 1) / kW; ++s)
        if (lane + s * kW < K) {
            rows[wv].r[1][lane + s * kW] = acc[s];
            M[(int64_t)par * ldk + lane + s * kW] = acc[s];
        }
    wave_sync();
    for (int r = lane; r < R; r += kW) {
        double v = 0.0;
        for (int t = 0; t < fold.n[r]; ++t) v = fma(fold.c[r][t], rows[wv].r[1][fold.src[r][t]], v);
        Mr[(int64_t)par * ldr + r] = (TR)v;
    }
}

template <int Q>
__global__ __launch_bounds__(kW *kTreeWaves) void mapped_l2l_kernel(int n_par, const int32_t *__restrict__ parents,
                                                                     const double4 *__restrict__ centre,
                                                                     double *__restrict__ Lam, int ldk)
{
    constexpr int K = ncoef(Q);
    __shared__ double lp[kTreeWaves][K];
    __shared__ double pw[kTreeWaves][8][3][Q + 1];
    __shared__ PassRows<Q> rows[kTreeWaves];
    const int wv = threadIdx.x / kW, lane = threadIdx.x & (kW - 1);
    const int w = blockIdx.x * kTreeWaves + wv;
    if (w >= n_par) return;
    const int32_t par = parents[2 * w], first = parents[2 * w + 1];
    const double4 cp = centre[par];
    constexpr int NA = (K + kW - 1) / kW;
    double old[8][NA];  // the children's own locals, read while the passes run
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int n = 0; n < NA; ++n)
            old[c][n] = lane + kW * n < K ? Lam[(int64_t)(first + c) * ldk + lane + kW * n] : 0.0;
    for (int i = lane; i < K; i += kW) lp[wv][i] = Lam[(int64_t)par * ldk + i];
    if (lane < 24) shift_factors(pw[wv][lane / 3][lane % 3], centre[first + lane / 3], cp, lane % 3, 1.0, Q);
    wave_sync();
    PassCodes<Q> pc;
    l2l_codes<Q>(pc, lane);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        l2l_pass<Q, 2>(lp[wv], rows[wv].r[0], pw[wv][c][2], pc, lane);
        wave_sync();
        l2l_pass<Q, 1>(rows[wv].r[0], rows[wv].r[1], pw[wv][c][1], pc, lane);
        wave_sync();
        l2l_pass<Q, 0>(rows[wv].r[1], rows[wv].r[0], pw[wv][c][0], pc, lane);
        wave_sync();
#pragma unroll
        for (int n = 0; n < NA; ++n)
            if (lane + kW * n < K)
                Lam[(int64_t)(first + c) * ldk + lane + kW * n] = old[c][n] + rows[wv].r[0][lane + kW * n];
        wave_sync();
    }
}

// ---- interaction phase with per-pair derivatives ----------------------------------------------
// Lambda^a = a^-1 sum_{b_z <= 1} D^{a+b} g(o) Mr^b over the reduced a (a_z <= 1), then expanded to
// every a (the harmonic reduction of the lattice kernel), with o = (x_t - x_s) / a the pair's scaled
// offset, now arbitrary. D^g g for g_z <= 2 (all a + b need) from the recurrence of the Taylor
// coefficients of 1/|r| (Duan and Krasny, 2001), written for D^g g = g! a_g / (4 pi):
//   |g| |o|^2 D_g = -(2|g| - 1) sum_i g_i o_i D_{g - e_i} - (|g| - 1) sum_i g_i (g_i - 1) D_{g - 2e_i},
// which stays inside g_z <= 2. Derivatives in FP64, the contraction in T.
template <int Q>
struct PairTables {
    static constexpr int count()
    {
        int n = 0;
        for (int d = 0; d <= Q; ++d)
            for (int i = d; i >= 0; --i)
                for (int j = d - i; j >= 0; --j)
                    if (d - i - j <= 2) ++n;
        return n;
    }
    static constexpr int N = count(), R = nreduced(Q);
    int e[N][3], deg[N], m1[N][3], m2[N][3];
    int sum[R][R];  // position of a + b (reduced a, b) in this set, -1 where |a| + |b| > Q
    constexpr int pos(int x, int y, int z) const
    {
        for (int k = 0; k < N; ++k)
            if (e[k][0] == x && e[k][1] == y && e[k][2] == z) return k;
        return -1;
    }
    constexpr PairTables() : e{}, deg{}, m1{}, m2{}, sum{}
    {
        int n = 0;
        for (int d = 0; d <= Q; ++d)
            for (int i = d; i >= 0; --i)
                for (int j = d - i; j >= 0; --j)
                    if (d - i - j <= 2) {
                        e[n][0] = i, e[n][1] = j, e[n][2] = d - i - j, deg[n] = d;
                        ++n;
                    }
        for (int k = 0; k < N; ++k)
            for (int ax = 0; ax < 3; ++ax) {
                int g1[3] = {e[k][0], e[k][1], e[k][2]}, g2[3] = {e[k][0], e[k][1], e[k][2]};
                g1[ax] -= 1;
                g2[ax] -= 2;
                m1[k][ax] = g1[ax] >= 0 ? pos(g1[0], g1[1], g1[2]) : -1;
                m2[k][ax] = g2[ax] >= 0 ? pos(g2[0], g2[1], g2[2]) : -1;
            }
        constexpr ReducedIndex<Q> ri{};
        for (int a = 0; a < R; ++a)
            for (int b = 0; b < R; ++b)
                sum[a][b] = ri.deg[a] + ri.deg[b] <= Q
                                ? pos(ri.e[a][0] + ri.e[b][0], ri.e[a][1] + ri.e[b][1], ri.e[a][2] + ri.e[b][2])
                                : -1;
    }
};

template <int Q>
struct PairT {
    static constexpr PairTables<Q> t{};
};

// D_g for g_z = 2 follows from harmonicity, D_{(i, j, 2)} = -D_{(i + 2, j, 0)} - D_{(i, j + 2, 0)} (both
// of the same degree and earlier in the order); the others from the recurrence, with 1/|g| a
// compile-time factor (a multiplication, not a division per entry).
template <int Q, int k>
__device__ __forceinline__ void deriv_step(double *D, const double *o, double inv_r2)
{
    constexpr auto &pt = PairT<Q>::t;
    constexpr int n = pt.deg[k];
    if constexpr (pt.e[k][2] == 2) {
        constexpr int kx = pt.pos(pt.e[k][0] + 2, pt.e[k][1], 0), ky = pt.pos(pt.e[k][0], pt.e[k][1] + 2, 0);
        static_assert(kx >= 0 && kx < k && ky >= 0 && ky < k, "harmonic partners come first");
        D[k] = -D[kx] - D[ky];
    } else {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (pt.m1[k][ax] >= 0) s1 = fma((double)pt.e[k][ax] * o[ax], D[pt.m1[k][ax] >= 0 ? pt.m1[k][ax] : 0], s1);
            if (pt.m2[k][ax] >= 0)
                s2 = fma((double)(pt.e[k][ax] * (pt.e[k][ax] - 1)), D[pt.m2[k][ax] >= 0 ? pt.m2[k][ax] : 0], s2);
        }
        constexpr double inv_n = 1.0 / n;
        D[k] = (-(double)(2 * n - 1) * s1 - (double)(n - 1) * s2) * (inv_r2 * inv_n);
    }
}

template <int Q, int... Ks>
__device__ __forceinline__ void derivatives(double *D, const double *o, std::integer_sequence<int, Ks...>)
{
    const double r2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
    D[0] = kInv4PiM / sqrt(r2);
    const double inv_r2 = 1.0 / r2;
    (deriv_step<Q, Ks + 1>(D, o, inv_r2), ...);
}

template <int Q, class T, int B, int... As>
__device__ __forceinline__ void pair_column(T *acc, const T *D, T mb, std::integer_sequence<int, As...>)
{
    constexpr auto &pt = PairT<Q>::t;
    ((acc[As] = fma(D[pt.sum[As][B] >= 0 ? pt.sum[As][B] : 0], mb, acc[As])), ...);
}

// The source's folded moments are read column by column (not held all at once); D: the derivatives
// in the contraction's type (converted once per pair).
template <int Q, class T, int... Bs>
__device__ __forceinline__ void pair_contract(T *acc, const T *D, const T *__restrict__ m,
                                              std::integer_sequence<int, Bs...>)
{
    constexpr ReducedIndex<Q> ri{};
    (pair_column<Q, T, Bs>(acc, D, m[Bs],
                           std::make_integer_sequence<int, nreduced(Q - ri.deg[Bs])>{}),
     ...);
}

template <int Q, class T, int... Fs>
__device__ __forceinline__ void pair_store(const T *acc, double scale, double *__restrict__ dst,
                                           std::integer_sequence<int, Fs...>)
{
    constexpr auto &ex = kExM<Q>;
    auto one = [&](int a) {
        double v = 0.0;
        for (int t = 0; t < ex.n[a]; ++t) v += ex.c[a][t] * (double)acc[ex.src[a][t]];
        return v;
    };
    ((dst[Fs] = scale * one(Fs)), ...);
}

// One thread per listed target cell (CSR lists of source cells).
template <int Q, class T>
__global__ __launch_bounds__(kW) void m2l_pairs_kernel(const int32_t *__restrict__ tgt, int32_t n,
                                                       const int64_t *__restrict__ off,
                                                       const int32_t *__restrict__ src,
                                                       const double4 *__restrict__ centre,
                                                       const T *__restrict__ Mr, double *__restrict__ Lam, int ldr,
                                                       int ldk)
{
    constexpr int R = nreduced(Q), N = PairTables<Q>::N, K = ncoef(Q);
    const int32_t i = (int32_t)(blockIdx.x * kW + threadIdx.x);
    if (i >= n) return;
    const int32_t t = tgt[i];
    const double4 ct = centre[t];
    const double inv_a = 1.0 / ct.w;
    T acc[R];
#pragma unroll
    for (int a = 0; a < R; ++a) acc[a] = T(0);
    const int64_t e1 = off[i + 1];
    for (int64_t e = off[i]; e < e1; ++e) {
        const int32_t s = src[e];
        const double4 cs = centre[s];
        const double o[3] = {(ct.x - cs.x) * inv_a, (ct.y - cs.y) * inv_a, (ct.z - cs.z) * inv_a};
        double D[N];
        derivatives<Q>(D, o, std::make_integer_sequence<int, N - 1>{});
        T Dt[N];
#pragma unroll
        for (int k = 0; k < N; ++k) Dt[k] = (T)D[k];
        pair_contract<Q, T>(acc, Dt, Mr + (int64_t)s * ldr, std::make_integer_sequence<int, R>{});
    }
    pair_store<Q, T>(acc, inv_a, Lam + (int64_t)t * ldk, std::make_integer_sequence<int, K>{});
}

template <int Q>
void mapped_passes(const bcv_plan_s &p, const double *f, int phase, hipStream_t st)
{
    const bool mixed = p.precision != BCV_FP64;
    if (phase == 0) {  // P2M
        if (p.K != ncoef(Q) || p.R != (Q + 1) * (Q + 1)) fail(BCV_ESTATE, "mapped P2M: row lengths");
        const int64_t n = p.n_leaves * p.K;
        const unsigned blocks = (unsigned)((n + 255) / 256);
        if (mixed)
            mapped_p2m_kernel<Q, float><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, p.d_kap, p.d_kapr, f,
                                                                p.d_M, p.d_M32, p.K, p.R);
        else
            mapped_p2m_kernel<Q, double><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, p.d_kap, p.d_kapr, f,
                                                                 p.d_M, p.d_Mr, p.K, p.R);
        check_launch();
    } else if (phase == 1) {  // M2M, finest parents first
        const auto *cen = reinterpret_cast<const double4 *>(p.d_centre);
        for (int lev = p.L - 1; lev >= 0; --lev) {
            const int n_par = p.parent_begin[lev + 1] - p.parent_begin[lev];
            if (n_par == 0) continue;
            const unsigned blocks = (unsigned)((n_par + kTreeWaves - 1) / kTreeWaves);
            const int32_t *par = p.d_parents + 2 * p.parent_begin[lev];
            if (mixed)
                mapped_m2m_kernel<Q, float><<<blocks, kW * kTreeWaves, 0, st>>>(n_par, par, cen, p.d_M, p.d_M32, p.K, p.R);
            else
                mapped_m2m_kernel<Q, double><<<blocks, kW * kTreeWaves, 0, st>>>(n_par, par, cen, p.d_M, p.d_Mr, p.K, p.R);
            check_launch();
        }
    } else if (phase == 2) {  // interaction phase of the ball cells of levels >= 2
        const auto *cen = reinterpret_cast<const double4 *>(p.d_centre);
        const int32_t n = (int32_t)p.n_ilist_targets;
        if (n > 0) {
            const unsigned blocks = (unsigned)((n + kW - 1) / kW);
            if (mixed)
                m2l_pairs_kernel<Q, float><<<blocks, kW, 0, st>>>(p.d_ilist_tgt, n, p.d_ilist_off, p.d_ilist_src, cen,
                                                                  p.d_M32, p.d_Lam, p.R, p.K);
            else
                m2l_pairs_kernel<Q, double><<<blocks, kW, 0, st>>>(p.d_ilist_tgt, n, p.d_ilist_off, p.d_ilist_src, cen,
                                                                   p.d_Mr, p.d_Lam, p.R, p.K);
            check_launch();
        }
    } else {  // L2L, coarsest parents first (levels 2 .. L - 1; levels 0 and 1 have no interaction list)
        const auto *cen = reinterpret_cast<const double4 *>(p.d_centre);
        for (int lev = 2; lev < p.L; ++lev) {
            const int n_par = p.parent_begin[lev + 1] - p.parent_begin[lev];
            if (n_par == 0) continue;
            const unsigned blocks = (unsigned)((n_par + kTreeWaves - 1) / kTreeWaves);
            mapped_l2l_kernel<Q><<<blocks, kW * kTreeWaves, 0, st>>>(n_par, p.d_parents + 2 * p.parent_begin[lev], cen,
                                                                     p.d_Lam, p.K);
            check_launch();
        }
    }
}

}  // namespace

void launch_mapped_phase(const bcv_plan_s &p, const double *f, int phase, hipStream_t st)
{
    switch (p.q) {
    case 4: mapped_passes<4>(p, f, phase, st); break;
    case 6: mapped_passes<6>(p, f, phase, st); break;
    case 8: mapped_passes<8>(p, f, phase, st); break;
    default: fail(BCV_ENOTSUP, "mapped meshes: q must be 4, 6 or 8");
    }
}

void launch_mapped_eval(const bcv_plan_s &p, double *u, hipStream_t st)
{
    const unsigned blocks = (unsigned)((p.n_leaves + 31) / 32);  // 8 lanes per leaf
    switch (p.q) {
    case 4: mapped_eval_kernel<4><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, p.d_kap, p.d_Lam, p.K, u); break;
    case 6: mapped_eval_kernel<6><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, p.d_kap, p.d_Lam, p.K, u); break;
    case 8: mapped_eval_kernel<8><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, p.d_kap, p.d_Lam, p.K, u); break;
    default: fail(BCV_ENOTSUP, "mapped meshes: q must be 4, 6 or 8");
    }
    check_launch();
}

void launch_mapped_zero(const bcv_plan_s &p, double *u, hipStream_t st)
{
    zero_kernel<<<(unsigned)std::min<int64_t>((p.n_leaves + 255) / 256, 4096), 256, 0, st>>>(p.n_leaves, u);
    check_launch();
}

// Plan time: the near entries of mapped target leaves (point rule), then their touching entries
// (singular rule), into p.d_val. touch_entry/touch_target list every touching entry of a ball leaf;
// the rule runs on the pairs of `work` (entry, target, mirror entry or -1) and writes both entries of
// a pair. cache: the touching values in list order, reused if it has the list's length, else filled.
// Synchronous.
void launch_mapped_assemble(const bcv_plan_s &p, const std::vector<int64_t> &touch_entry,
                            const std::vector<int64_t> &work_entry, const std::vector<int32_t> &work_target,
                            const std::vector<int64_t> &work_mirror, const int rule_orders[5],
                            std::vector<double> &cache)
{
    if (p.n_units > 0) {
        mapped_assemble_kernel<<<(unsigned)((p.n_units + 3) / 4), 256>>>(
            p.n_units, p.d_units, p.d_col, reinterpret_cast<const double4 *>(p.d_leaf_pts), p.d_leaf_mapped, p.d_val);
        check_launch();
    }
    const int64_t n = (int64_t)touch_entry.size();
    if (n == 0) {
        BCV_HIP(hipDeviceSynchronize());
        return;
    }
    int64_t *d_list = nullptr;
    double *d_vals = nullptr;
    BCV_HIP(hipMalloc(&d_list, n * sizeof(int64_t)));
    BCV_HIP(hipMalloc(&d_vals, n * sizeof(double)));
    BCV_HIP(hipMemcpy(d_list, touch_entry.data(), n * sizeof(int64_t), hipMemcpyHostToDevice));
    const unsigned cblocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    if ((int64_t)cache.size() == n) {
        BCV_HIP(hipMemcpy(d_vals, cache.data(), n * sizeof(double), hipMemcpyHostToDevice));
        touch_copy_kernel<<<cblocks, 256>>>(n, d_list, d_vals, p.d_val, 1);
        check_launch();
    } else {
        const SingRule R = make_rule(rule_orders);
        const int64_t nw = (int64_t)work_entry.size();
        int64_t *d_e = nullptr, *d_m = nullptr;
        int32_t *d_t = nullptr;
        BCV_HIP(hipMalloc(&d_e, nw * sizeof(int64_t)));
        BCV_HIP(hipMalloc(&d_m, nw * sizeof(int64_t)));
        BCV_HIP(hipMalloc(&d_t, nw * sizeof(int32_t)));
        BCV_HIP(hipMemcpy(d_e, work_entry.data(), nw * sizeof(int64_t), hipMemcpyHostToDevice));
        BCV_HIP(hipMemcpy(d_m, work_mirror.data(), nw * sizeof(int64_t), hipMemcpyHostToDevice));
        BCV_HIP(hipMemcpy(d_t, work_target.data(), nw * sizeof(int32_t), hipMemcpyHostToDevice));
        ball_touch_kernel<<<(unsigned)std::min<int64_t>(nw, 1 << 20), 256>>>(
            nw, d_e, d_t, d_m, p.d_col, reinterpret_cast<const double4 *>(p.d_leaf_geom), R, p.d_val);
        check_launch();
        touch_copy_kernel<<<cblocks, 256>>>(n, d_list, d_vals, p.d_val, 0);
        check_launch();
        cache.resize(n);
        BCV_HIP(hipMemcpy(cache.data(), d_vals, n * sizeof(double), hipMemcpyDeviceToHost));
        BCV_HIP(hipFree(d_e));
        BCV_HIP(hipFree(d_m));
        BCV_HIP(hipFree(d_t));
    }
    BCV_HIP(hipDeviceSynchronize());
    BCV_HIP(hipFree(d_list));
    BCV_HIP(hipFree(d_vals));
}

// The singular rule of `orders` on explicit pairs (host arrays of 4 doubles per cube: lower corner in
// the reference cube [0,1]^3 and side); results into out (host). Synchronous.
void mapped_rule_values(int64_t n, const double *geom_t, const double *geom_s, const int orders[5], double *out)
{
    if (n <= 0) return;
    const SingRule R = make_rule(orders);
    double *d = nullptr;
    BCV_HIP(hipMalloc(&d, (size_t)n * 9 * sizeof(double)));
    double *dt = d, *ds = d + 4 * n, *dv = d + 8 * n;
    BCV_HIP(hipMemcpy(dt, geom_t, (size_t)n * 4 * sizeof(double), hipMemcpyHostToDevice));
    BCV_HIP(hipMemcpy(ds, geom_s, (size_t)n * 4 * sizeof(double), hipMemcpyHostToDevice));
    ball_pair_kernel<<<(unsigned)std::min<int64_t>(n, 1 << 20), 256>>>(n, reinterpret_cast<const double4 *>(dt),
                                                                      reinterpret_cast<const double4 *>(ds), R, dv);
    check_launch();
    BCV_HIP(hipMemcpy(out, dv, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    BCV_HIP(hipFree(d));
}

}  // namespace bcv
