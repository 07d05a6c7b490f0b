// Device kernels of the VtV apply (Algorithm 1 of the paper) for gfx950, FP64.
//
// Expansion coefficients are stored scaled so that every translation is level independent.
// For a cell w of side a and centre x_w, with the moments m^b and local coefficients lambda^a
// of Sec. 3 (translation operators):
//     M^b      = (-1)^|b| m^b / (b! a^|b|)          (moments)
//     Lambda^a = lambda^a  a! a^|a|                 (local coefficients)
// Then, with tau = (x_child - x_parent)/a_parent in {-1/4, +1/4}^3 and o = (x_w - x_w')/a:
//     P2M  M^b       = f a^3 kappa_b,  kappa_b = (1/8) sum_g xi_g^b / b!  (2x2x2 Gauss nodes xi_g)
//     M2M  M_P^b     = sum_c sum_{g<=b} (-tau_c)^(b-g)/(b-g)! 2^-|g| M_c^g
//     M2L  Lambda^a += a^-1 sum_{|b|<=q-|a|} D^{a+b}g(o) M^b,  g = 1/(4 pi |.|)
//     L2L  Lambda_c^a += 2^-|a| sum_{b>=a} tau_c^(b-a)/(b-a)! Lambda_P^b
//     L2P  u_w      += a^3 sum_a kappa_a Lambda^a
// The near field adds, per leaf w, sum over N*(w) of A_{w s} f_s, with A_{w s} the exact
// touching integral C_class a_small^5/(4 pi) or the 2x2x2 x 2x2x2 point rule.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "kernels.hpp"
#include "multiindex.hpp"

namespace bcv {
namespace {

constexpr int kWave = 64;
constexpr double kNode0 = 0.21132486540518711775;  // 1/2 - 1/(2 sqrt 3): 2-point Gauss on [0,1]
constexpr double kNode1 = 0.78867513459481288225;  // 1/2 + 1/(2 sqrt 3)
constexpr double kInv4Pi = 0.079577471545947667884;

// Expansion sizes per level (level-dependent orders) and the row strides of the coefficient arrays.
struct LevelOrders {
    int32_t k[kMaxLevel + 1];  // ncoef(q_l)
    int32_t r[kMaxLevel + 1];  // (q_l + 1)^2, folded rows
    int32_t ldk, ldr;          // row strides of the moment / local arrays and of the folded rows
};

// Level of a cell from its side a = 2^-l (the exponent field of the double).
__device__ __forceinline__ int level_of_side(double a)
{
    return 1023 - (int)((__double_as_longlong(a) >> 52) & 0x7FF);
}

// mu(e)/e! per axis, mu(e) = (1/2)(xi^e + (-xi)^e), xi = 1/(2 sqrt 3) so xi^2 = 1/12.
constexpr double kappa_axis_ce(int e)
{
    if (e & 1) return 0.0;
    double v = 1.0;
    for (int t = 2; t <= e; t += 2) v /= 12.0;
    for (int t = 2; t <= e; ++t) v /= (double)t;
    return v;
}

template <int Q>
struct KappaTable {  // kappa_a = prod_i mu(a_i)/a_i! for every multi-index of order <= Q
    double v[MultiIndex<Q>::K];
    constexpr KappaTable() : v{}
    {
        constexpr MultiIndex<Q> mi{};
        for (int a = 0; a < MultiIndex<Q>::K; ++a)
            v[a] = kappa_axis_ce(mi.e[a][0]) * kappa_axis_ce(mi.e[a][1]) * kappa_axis_ce(mi.e[a][2]);
    }
};

template <int Q>
struct Tables {
    static constexpr MultiIndex<Q> mi{};
};

template <int Q>
__constant__ constexpr KappaTable<Q> kKappa{};

// Boundary moments (BtV, Algorithm 3). The 2x2 Gauss points of a face of a cell, relative to the
// cell centre in units of its side a, are s = side - 1/2 along the face's normal axis n and
// +-1/(2 sqrt 3) in the face. With m^b = int_face (y - x_w)^b q - d/dn (y - x_w)^b g (q and g
// constant on the face) and the scaled moments M^b = (-1)^|b| m^b / (b! a^|b|):
//     M^b = a^2 q phi^b - a g psi^b,
//     phi^b = (-1)^|b| s^{b_n}/b_n! kappa(b_1) kappa(b_2),
//     psi^b = sign (-1)^|b| s^{b_n - 1}/(b_n - 1)! kappa(b_1) kappa(b_2)   (0 if b_n = 0),
// with b_1, b_2 the in-face components, kappa the per-axis factor of P2M and sign = 2 side - 1 the
// outward normal. Face type = 2 axis + side.
template <int Q>
struct FaceKappaTable {
    double phi[6][MultiIndex<Q>::K], psi[6][MultiIndex<Q>::K];
    constexpr FaceKappaTable() : phi{}, psi{}
    {
        constexpr MultiIndex<Q> mi{};
        for (int type = 0; type < 6; ++type) {
            const int ax = type >> 1, side = type & 1;
            const double s = side ? 0.5 : -0.5, sign = side ? 1.0 : -1.0;
            for (int b = 0; b < MultiIndex<Q>::K; ++b) {
                double in_face = 1.0;
                for (int d = 0; d < 3; ++d)
                    if (d != ax) in_face *= kappa_axis_ce(mi.e[b][d]);
                const int bn = mi.e[b][ax];
                const double par = (mi.deg[b] & 1) ? -1.0 : 1.0;
                double p_bn = 1.0, p_bn1 = 1.0;  // s^bn / bn!, s^(bn-1) / (bn-1)!
                for (int k = 1; k <= bn; ++k) p_bn *= s / k;
                for (int k = 1; k <= bn - 1; ++k) p_bn1 *= s / k;
                phi[type][b] = par * p_bn * in_face;
                psi[type][b] = bn >= 1 ? sign * par * p_bn1 * in_face : 0.0;
            }
        }
    }
};

template <int Q>
__constant__ constexpr FaceKappaTable<Q> kFaceKappa{};

// Harmonic folding of the moments (see the M2L section): Mr^b = sum_t c[b][t] M^{src[b][t]} over the
// (Q + 1)^2 multi-indices b with b_z <= 1. The writers of the moments (P2M, the boundary P2M, M2M)
// also write the folded rows the interaction phase reads; for the leaf moments this is the folded
// kappa table.
template <int Q>
struct FoldedKappaTable {
    double v[nreduced(Q)];
    constexpr FoldedKappaTable() : v{}
    {
        constexpr KappaTable<Q> kap{};
        constexpr FoldTable<Q> fo{};
        for (int b = 0; b < nreduced(Q); ++b)
            for (int t = 0; t < fo.n[b]; ++t) v[b] += fo.c[b][t] * kap.v[fo.src[b][t]];
    }
};

template <int Q>
struct FoldedFaceKappaTable {
    double phi[6][nreduced(Q)], psi[6][nreduced(Q)];
    constexpr FoldedFaceKappaTable() : phi{}, psi{}
    {
        constexpr FaceKappaTable<Q> fk{};
        constexpr FoldTable<Q> fo{};
        for (int type = 0; type < 6; ++type)
            for (int b = 0; b < nreduced(Q); ++b)
                for (int t = 0; t < fo.n[b]; ++t) {
                    phi[type][b] += fo.c[b][t] * fk.phi[type][fo.src[b][t]];
                    psi[type][b] += fo.c[b][t] * fk.psi[type][fo.src[b][t]];
                }
    }
};

template <int Q>
__constant__ constexpr FoldTable<Q> kFold{};
template <int Q>
__constant__ constexpr FoldedKappaTable<Q> kFoldedKappa{};
template <int Q>
__constant__ constexpr FoldedFaceKappaTable<Q> kFoldedFaceKappa{};

// Moments of a parent whose 8 children are leaves with densities f_c (side a each): the children's
// moments f_c a^3 kappa translated by M2M (separable per axis) give
//     M_P^b = a^3 sum_c f_c W[c][b],   W[c][b] = prod_i w1(c_i, b_i),
//     w1(s, e) = sum_{g <= e} (+-1/4)^(e-g)/(e-g)! 2^-g kappa1(g)   (+ for the lower child, s = 0),
// and the folded row likewise with Wr = fold(W).
template <int Q>
struct LeafParentTable {
    double W[8][ncoef(Q)], Wr[8][nreduced(Q)];
    constexpr LeafParentTable() : W{}, Wr{}
    {
        constexpr MultiIndex<Q> mi{};
        constexpr FoldTable<Q> fo{};
        double w1[2][Q + 1] = {};
        for (int side = 0; side < 2; ++side)
            for (int e = 0; e <= Q; ++e)
                for (int g = 0; g <= e; ++g) {
                    double t = kappa_axis_ce(g);
                    for (int k = 1; k <= e - g; ++k) t *= (side ? -0.25 : 0.25) / k;
                    for (int k = 0; k < g; ++k) t *= 0.5;
                    w1[side][e] += t;
                }
        for (int c = 0; c < 8; ++c) {
            for (int b = 0; b < ncoef(Q); ++b)
                W[c][b] = w1[c & 1][mi.e[b][0]] * w1[(c >> 1) & 1][mi.e[b][1]] * w1[(c >> 2) & 1][mi.e[b][2]];
            for (int r = 0; r < nreduced(Q); ++r)
                for (int t = 0; t < fo.n[r]; ++t) Wr[c][r] += fo.c[r][t] * W[c][fo.src[r][t]];
        }
    }
};
template <int Q>
__constant__ constexpr LeafParentTable<Q> kLeafParent{};

// The evaluation of a parent's local expansion at its 8 leaf children, through their L2L: child c
// (c = x + 2y + 4z, bit 0 on an axis = the lower half, tau = -1/4 there and +1/4 above) gets
//   sum_a kappa_a Lambda_c^a = sum_a kappa_a 2^-|a| sum_{b >= a} prod_i tau_i^(b_i-a_i)/(b_i-a_i)! Lambda_P^b
//                            = sum_b E[c][b] Lambda_P^b,
// E[c][b] = prod_i e1[side_i][b_i], e1[side][e] = sum_{g <= e} kappa_axis(g) 2^-g tau^(e-g)/(e-g)!
// (kappa and the shift are products over the axes; a <= b keeps |a| <= |b| <= Q, so nothing the L2L
// truncates is lost).
template <int Q>
struct LeafEvalTable {
    double E[8][ncoef(Q)];
    constexpr LeafEvalTable() : E{}
    {
        constexpr MultiIndex<Q> mi{};
        double e1[2][Q + 1] = {};
        for (int side = 0; side < 2; ++side)
            for (int e = 0; e <= Q; ++e)
                for (int g = 0; g <= e; ++g) {
                    double t = kappa_axis_ce(g);
                    for (int k = 1; k <= e - g; ++k) t *= (side ? 0.25 : -0.25) / k;
                    for (int k = 0; k < g; ++k) t *= 0.5;
                    e1[side][e] += t;
                }
        for (int c = 0; c < 8; ++c)
            for (int b = 0; b < ncoef(Q); ++b)
                E[c][b] = e1[c & 1][mi.e[b][0]] * e1[(c >> 1) & 1][mi.e[b][1]] * e1[(c >> 2) & 1][mi.e[b][2]];
    }
};
template <int Q>
__constant__ constexpr LeafEvalTable<Q> kLeafEval{};

// (1/4)^k / k! for k = 0..kMaxOrder (translation coefficients; the sign (-1)^k is applied by the caller).
constexpr int kMaxOrder = 12;
struct QuarterTable {
    double v[kMaxOrder + 1];
    constexpr QuarterTable() : v{}
    {
        v[0] = 1.0;
        for (int k = 1; k <= kMaxOrder; ++k) v[k] = v[k - 1] * 0.25 / k;
    }
};
__constant__ constexpr QuarterTable kQuarter{};


__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

struct TouchValues {
    double v[kTouchClasses];  // C_class / (4 pi), smaller side 1
};

// 1/sqrt(x) for finite x > 0: the hardware estimate (relative error about 5e-8) refined by one
// Newton step y <- y + y (1 - x y^2) / 2 (relative error below 5e-15, measured on gfx950).
__device__ __forceinline__ double rsqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(0.5 * y, e, y);
}

// sum_{g in t} sum_{g' in s} w_g w_g' G(x_g, y_g') with the 2x2x2 rule on both cubes.
__device__ __forceinline__ double point_rule(const double4 gt, const double4 gs)
{
    double d2[3][4];
    const double lt[3] = {gt.x, gt.y, gt.z}, ls[3] = {gs.x, gs.y, gs.z};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double x0 = lt[ax] + gt.w * kNode0, x1 = lt[ax] + gt.w * kNode1;
        const double y0 = ls[ax] + gs.w * kNode0, y1 = ls[ax] + gs.w * kNode1;
        const double d[4] = {x0 - y0, x0 - y1, x1 - y0, x1 - y1};
#pragma unroll
        for (int m = 0; m < 4; ++m) d2[ax][m] = d[m] * d[m];
    }
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const double xy = d2[0][a] + d2[1][b];
#pragma unroll
            for (int c = 0; c < 4; ++c) s += rsqrt_pos(xy + d2[2][c]);
        }
    const double wt = gt.w * gt.w * gt.w * 0.125, ws = gs.w * gs.w * gs.w * 0.125;
    return s * wt * ws * kInv4Pi;
}

// The same point rule with the 64 kernel evaluations in FP32: per-axis differences are formed in
// FP64 (exact inputs, so their rounding is relative to the gap, not to the coordinates), then
// squared and summed in FP32 with the hardware reciprocal square root (about 1 ulp).
__device__ __forceinline__ double point_rule_f32(const double4 gt, const double4 gs)
{
    float d2[3][4];
    const double lt[3] = {gt.x, gt.y, gt.z}, ls[3] = {gs.x, gs.y, gs.z};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double x0 = lt[ax] + gt.w * kNode0, x1 = lt[ax] + gt.w * kNode1;
        const double y0 = ls[ax] + gs.w * kNode0, y1 = ls[ax] + gs.w * kNode1;
        const float d[4] = {(float)(x0 - y0), (float)(x0 - y1), (float)(x1 - y0), (float)(x1 - y1)};
#pragma unroll
        for (int m = 0; m < 4; ++m) d2[ax][m] = d[m] * d[m];
    }
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float xy = d2[0][a] + d2[1][b];
#pragma unroll
            for (int c = 0; c < 4; ++c) s += __builtin_amdgcn_rsqf(xy + d2[2][c]);
        }
    const double wt = gt.w * gt.w * gt.w * 0.125, ws = gs.w * gs.w * gs.w * 0.125;
    return (double)s * wt * ws * kInv4Pi;
}

__device__ __forceinline__ double near_entry(uint32_t code, const double4 gt, const double4 *__restrict__ geom,
                                             const TouchValues &tv)
{
    const int32_t s = (int32_t)(code & 0x0FFFFFFFu);
    const uint32_t cls = code >> 28;
    const double4 gs = geom[s];
    if (cls) {
        const double a = fmin(gt.w, gs.w);
        return tv.v[(cls & 7u) - 1] * (a * a) * (a * a) * a;
    }
    return point_rule(gt, gs);
}

// Lane k's value, in every lane (k wave-uniform).
__device__ __forceinline__ int lane_value(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ double lane_value(double v, int k)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, k), hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// ---- P2M: M^b = f a^3 kappa_b on every leaf, and the folded row Mr = f a^3 fold(kappa) ------------
// Q: the largest order of any level; a level-l leaf writes its ncoef(q_l) and (q_l + 1)^2 leading
// coefficients (the tables are graded, so those are the order-q_l tables).
// Leaves of level skip_level write only their folded rows (their parents' moments come from
// m2m_leaves_kernel); -1 = none. One wave per 64 consecutive leaves: lane l reads leaf l's density,
// side and cell, then the wave writes the leaves' rows one after the other, lanes over coefficients.
template <int Q, class TR>
__global__ __launch_bounds__(256) void p2m_kernel(int64_t n_leaves, const int32_t *__restrict__ leaf_cell,
                                                  const double4 *__restrict__ geom, const double *__restrict__ f,
                                                  double *__restrict__ M, TR *__restrict__ Mr, const LevelOrders lo,
                                                  int skip_level)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t base = ((int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave;
    if (base >= n_leaves) return;  // uniform per wave
    const int cnt = (int)min((int64_t)kWave, n_leaves - base);
    double sl = 0.0;
    int cl = 0, levl = 0;
    if (lane < cnt) {
        const double a = geom[base + lane].w;
        levl = level_of_side(a);
        sl = f[base + lane] * (a * a * a);
        cl = leaf_cell[base + lane];
    }
    for (int k = 0; k < cnt; ++k) {
        const double sk = lane_value(sl, k);
        const int64_t c = lane_value(cl, k);
        const int lev = lane_value(levl, k);
        for (int j = lane; j < lo.r[lev]; j += kWave) Mr[c * lo.ldr + j] = (TR)(sk * kFoldedKappa<Q>.v[j]);
        if (lev != skip_level)
            for (int b = lane; b < lo.k[lev]; b += kWave) M[c * lo.ldk + b] = sk * kKappa<Q>.v[b];
    }
}

// M2M for parents whose 8 children are leaves, straight from the children's densities (see
// LeafParentTable). One wave per 64 parents: lane l gathers parent l's 8 densities, then the wave
// writes the parents' rows one after the other, lanes over coefficients (each lane keeps the table
// entries of its coefficients in registers).
template <int Q, class TR>
__global__ __launch_bounds__(256) void m2m_leaves_kernel(int n_par, const int32_t *__restrict__ parents,
                                                         const int32_t *__restrict__ cell_leaf,
                                                         const double4 *__restrict__ geom,
                                                         const double *__restrict__ f, double *__restrict__ M,
                                                         TR *__restrict__ Mr, int32_t ldk, int32_t ldr)
{
    constexpr int K = MultiIndex<Q>::K, R = nreduced(Q), NK = (K + kWave - 1) / kWave, NR = (R + kWave - 1) / kWave;
    const int lane = threadIdx.x % kWave;
    const int base = (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave;
    if (base >= n_par) return;  // uniform per wave
    const int cnt = min(kWave, n_par - base);
    double fl[8] = {}, a3l = 0.0;
    int celll = 0;
    if (lane < cnt) {
        celll = parents[2 * (base + lane)];
        const int32_t child0 = parents[2 * (base + lane) + 1];
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int32_t leaf = cell_leaf[child0 + c];
            fl[c] = f[leaf];
            a = geom[leaf].w;
        }
        a3l = a * a * a;
    }
    double w[NK][8], wr[NR][8];
#pragma unroll
    for (int n = 0; n < NK; ++n)
#pragma unroll
        for (int c = 0; c < 8; ++c) w[n][c] = lane + kWave * n < K ? kLeafParent<Q>.W[c][lane + kWave * n] : 0.0;
#pragma unroll
    for (int n = 0; n < NR; ++n)
#pragma unroll
        for (int c = 0; c < 8; ++c) wr[n][c] = lane + kWave * n < R ? kLeafParent<Q>.Wr[c][lane + kWave * n] : 0.0;
    for (int k = 0; k < cnt; ++k) {
        double fc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) fc[c] = lane_value(fl[c], k);
        const double a3 = lane_value(a3l, k);
        const int64_t cell = lane_value(celll, k);
#pragma unroll
        for (int n = 0; n < NK; ++n) {
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c) v = fma(fc[c], w[n][c], v);
            if (lane + kWave * n < K) M[cell * ldk + lane + kWave * n] = v * a3;
        }
#pragma unroll
        for (int n = 0; n < NR; ++n) {
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c) v = fma(fc[c], wr[n][c], v);
            if (lane + kWave * n < R) Mr[cell * ldr + lane + kWave * n] = (TR)(v * a3);
        }
    }
}

// ---- M2M and L2L: one wave per marked cell, separable per-axis shifts through LDS -----------------
// Both translations are tensor products of 1-D shifts, and stay inside |b| <= Q axis by axis:
//   M2M  M_P^b  = sum_c prod_i [ sum_{g_i <= b_i} (-tau_i)^(b_i-g_i)/(b_i-g_i)! 2^-g_i ] M_c^g
//   L2L  Lam_c^a = 2^-|a| prod_i [ sum_{b_i >= a_i} tau_i^(b_i-a_i)/(b_i-a_i)! ] Lam_P^b
// so the 8 children are combined pairwise along x, then y, then z (M2M), and the parent is
// expanded along z, then y, then x (L2L): 14 one-dimensional passes per parent instead of 8 full
// three-dimensional sums. Lane l owns the coefficients l, l + 64, ...: their multi-indices are read
// once, and within a pass the index and weight of every term are shared by all the vectors the pass
// treats. The 1-D weights come from a small LDS table.
// Parents per block (one wave each).
template <int Q>
constexpr int tree_waves()
{
    return 4;
}

// w[e][g] = (1/4)^(e-g)/(e-g)! 2^-g for g <= e (M2M); the L2L weights are w[k][0] = (1/4)^k/k!.
template <int Q>
__device__ __forceinline__ void fill_shift_weights(double (*w)[Q + 1])
{
    for (int i = threadIdx.x; i < (Q + 1) * (Q + 1); i += blockDim.x) {
        const int e = i / (Q + 1), g = i % (Q + 1);
        w[e][g] = g <= e ? kQuarter.v[e - g] * ldexp(1.0, -g) : 0.0;
    }
}

// Children rows hold moments up to their own order (zero beyond): the parent's order Q covers them.
template <int Q, class TR>
__global__ __launch_bounds__(kWave *tree_waves<Q>()) void m2m_kernel(int n_par, const int32_t *__restrict__ parents,
                                                                      double *__restrict__ M, TR *__restrict__ Mr,
                                                                      int32_t ldk, int32_t ldr)
{
    constexpr int K = MultiIndex<Q>::K, R = nreduced(Q), NB = (K + kWave - 1) / kWave;
    constexpr auto &mi = Tables<Q>::mi;
    __shared__ double buf[tree_waves<Q>()][8][K];
    __shared__ double w[Q + 1][Q + 1];
    fill_shift_weights<Q>(w);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int pi = blockIdx.x * tree_waves<Q>() + wave;
    const bool active = pi < n_par;
    double(*B)[K] = buf[wave];
    int ex[NB], ey[NB], ez[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) {
        const int b = lane + kWave * n;
        ex[n] = b < K ? mi.e[b][0] : 0;
        ey[n] = b < K ? mi.e[b][1] : 0;
        ez[n] = b < K ? mi.e[b][2] : 0;
    }
    int32_t cell = 0;
    if (active) {
        cell = parents[2 * pi];
        const double *__restrict__ src = M + (int64_t)parents[2 * pi + 1] * ldk;  // 8 consecutive children
        constexpr int NL = (8 * K + kWave - 1) / kWave;
        double v[NL];  // every load issued before the first LDS store
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int n = lane + kWave * i;
            v[i] = n < 8 * K ? src[(int64_t)(n / K) * ldk + n % K] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < NL; ++i)
            if (lane + kWave * i < 8 * K) B[(lane + kWave * i) / K][(lane + kWave * i) % K] = v[i];
    }
    __syncthreads();
    // x: children (0,y,z) + (1,y,z) -> 4 vectors indexed by y + 2z (lower child: -tau = +1/4)
    double xo[NB][4] = {};
    if (active)
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            if (lane + kWave * n >= K) continue;
            for (int g = 0; g <= ex[n]; ++g) {
                const int idx = mi_index(g, ey[n], ez[n]);
                const double wt = w[ex[n]][g], sg = ((ex[n] - g) & 1) ? -wt : wt;
#pragma unroll
                for (int yz = 0; yz < 4; ++yz) xo[n][yz] += wt * B[2 * yz][idx] + sg * B[2 * yz + 1][idx];
            }
        }
    __syncthreads();
    if (active)
#pragma unroll
        for (int n = 0; n < NB; ++n)
            if (lane + kWave * n < K)
#pragma unroll
                for (int yz = 0; yz < 4; ++yz) B[yz][lane + kWave * n] = xo[n][yz];
    __syncthreads();
    // y: vectors (0,z) + (1,z) -> 2 vectors indexed by z
    double yo[NB][2] = {};
    if (active)
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            if (lane + kWave * n >= K) continue;
            for (int g = 0; g <= ey[n]; ++g) {
                const int idx = mi_index(ex[n], g, ez[n]);
                const double wt = w[ey[n]][g], sg = ((ey[n] - g) & 1) ? -wt : wt;
#pragma unroll
                for (int z = 0; z < 2; ++z) yo[n][z] += wt * B[2 * z][idx] + sg * B[2 * z + 1][idx];
            }
        }
    __syncthreads();
    if (active)
#pragma unroll
        for (int n = 0; n < NB; ++n)
            if (lane + kWave * n < K)
#pragma unroll
                for (int z = 0; z < 2; ++z) B[z][lane + kWave * n] = yo[n][z];
    __syncthreads();
    // z: vectors 0 + 1 -> the parent's moments; slot 2 keeps them for the folded row
    if (active)
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int b = lane + kWave * n;
            if (b >= K) continue;
            double acc = 0.0;
            for (int g = 0; g <= ez[n]; ++g) {
                const int idx = mi_index(ex[n], ey[n], g);
                const double wt = w[ez[n]][g], sg = ((ez[n] - g) & 1) ? -wt : wt;
                acc += wt * B[0][idx] + sg * B[1][idx];
            }
            M[(int64_t)cell * ldk + b] = acc;
            B[2][b] = acc;
        }
    __syncthreads();
    if (active)  // the folded row
        for (int r = lane; r < R; r += kWave) {
            double v = 0.0;
            for (int t = 0; t < kFold<Q>.n[r]; ++t) v = fma(kFold<Q>.c[r][t], B[2][kFold<Q>.src[r][t]], v);
            Mr[(int64_t)cell * ldr + r] = (TR)v;
        }
}

// Q: the parent's order; the children keep their first k_child coefficients (their own order).
template <int Q>
__global__ __launch_bounds__(kWave *tree_waves<Q>()) void l2l_kernel(int n_par, const int32_t *__restrict__ parents,
                                                                      double *__restrict__ Lam, int32_t ldk,
                                                                      int32_t k_child)
{
    constexpr int K = MultiIndex<Q>::K, NB = (K + kWave - 1) / kWave;
    constexpr auto &mi = Tables<Q>::mi;
    __shared__ double buf[tree_waves<Q>()][7][K];
    __shared__ double w[Q + 1][Q + 1];
    fill_shift_weights<Q>(w);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int pi = blockIdx.x * tree_waves<Q>() + wave;
    const bool active = pi < n_par;
    double(*B)[K] = buf[wave];
    int ex[NB], ey[NB], ez[NB], dg[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) {
        const int a = lane + kWave * n;
        ex[n] = a < K ? mi.e[a][0] : 0;
        ey[n] = a < K ? mi.e[a][1] : 0;
        ez[n] = a < K ? mi.e[a][2] : 0;
        dg[n] = ex[n] + ey[n] + ez[n];
    }
    int32_t child0 = 0;
    double old[NB][8];  // the children's own locals, read while the passes run
    if (active) {
        child0 = parents[2 * pi + 1];
        const double *__restrict__ src = Lam + (int64_t)parents[2 * pi] * ldk;
        const double *__restrict__ dst = Lam + (int64_t)child0 * ldk;  // 8 consecutive children
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int c = 0; c < 8; ++c)
                old[n][c] = lane + kWave * n < k_child ? dst[(int64_t)c * ldk + lane + kWave * n] : 0.0;
        for (int n = lane; n < K; n += kWave) B[0][n] = src[n];
    }
    __syncthreads();
    // out_lo[a] = sum_{b >= a_AX} (-1/4)^(b-a)/(b-a)! in[.., b, ..], out_hi the same with +1/4
    if (active)  // z: slot 0 -> slots 1 + z
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int a = lane + kWave * n;
            if (a >= K) continue;
            double lo = 0.0, hi = 0.0;
            for (int b = ez[n]; b <= Q - dg[n] + ez[n]; ++b) {
                const double v = B[0][mi_index(ex[n], ey[n], b)] * w[b - ez[n]][0];
                hi += v;
                lo += ((b - ez[n]) & 1) ? -v : v;
            }
            B[1][a] = lo;
            B[2][a] = hi;
        }
    __syncthreads();
    if (active)  // y: slots 1 + z -> slots 3 + y + 2z
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int a = lane + kWave * n;
            if (a >= K) continue;
            double lo[2] = {0.0, 0.0}, hi[2] = {0.0, 0.0};
            for (int b = ey[n]; b <= Q - dg[n] + ey[n]; ++b) {
                const int idx = mi_index(ex[n], b, ez[n]);
                const double wt = w[b - ey[n]][0], sg = ((b - ey[n]) & 1) ? -wt : wt;
#pragma unroll
                for (int z = 0; z < 2; ++z) {
                    hi[z] += wt * B[1 + z][idx];
                    lo[z] += sg * B[1 + z][idx];
                }
            }
#pragma unroll
            for (int z = 0; z < 2; ++z) {
                B[3 + 2 * z][a] = lo[z];
                B[3 + 2 * z + 1][a] = hi[z];
            }
        }
    __syncthreads();
    if (active) {  // x: slots 3 + y + 2z -> child x + 2y + 4z, added to the children's locals with 2^-|a|
        double *__restrict__ dst = Lam + (int64_t)child0 * ldk;  // 8 consecutive children
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int a = lane + kWave * n;
            if (a >= k_child) continue;
            double lo[4] = {0.0, 0.0, 0.0, 0.0}, hi[4] = {0.0, 0.0, 0.0, 0.0};
            for (int b = ex[n]; b <= Q - dg[n] + ex[n]; ++b) {
                const int idx = mi_index(b, ey[n], ez[n]);
                const double wt = w[b - ex[n]][0], sg = ((b - ex[n]) & 1) ? -wt : wt;
#pragma unroll
                for (int yz = 0; yz < 4; ++yz) {
                    hi[yz] += wt * B[3 + yz][idx];
                    lo[yz] += sg * B[3 + yz][idx];
                }
            }
            const double sc = ldexp(1.0, -dg[n]);
#pragma unroll
            for (int yz = 0; yz < 4; ++yz) {
                dst[(int64_t)(2 * yz) * ldk + a] = fma(lo[yz], sc, old[n][2 * yz]);
                dst[(int64_t)(2 * yz + 1) * ldk + a] = fma(hi[yz], sc, old[n][2 * yz + 1]);
            }
        }
    }
}

// The last level's L2L fused with the evaluation of its children, all of them leaves of one level
// (fixed orders): u_c += a^3 sum_a kappa_a (Lambda_c^a + the parent's L2L contribution), with the
// parent's part through kLeafEval, so the children's locals are read but not written. One wave per
// kLeafEvalPar consecutive parents, one after the other; lane l takes child l / 8 and its coefficients
// l % 8 + 8 i, whose table entries it keeps in registers.
constexpr int kLeafEvalPar = 4;
template <int Q>
__global__ __launch_bounds__(256) void leaf_eval_kernel(int n_par, const int32_t *__restrict__ parents,
                                                        const double *__restrict__ Lam, int32_t ldk,
                                                        const int32_t *__restrict__ cell_leaf,
                                                        const double4 *__restrict__ geom, double *__restrict__ u)
{
    constexpr int K = MultiIndex<Q>::K, NI = (K + 7) / 8;
    const int lane = threadIdx.x % kWave, c = lane >> 3, j = lane & 7;
    const int p0 = (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kLeafEvalPar;
    if (p0 >= n_par) return;  // uniform per wave
    double ke[NI], kk[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int b = j + 8 * i;
        ke[i] = b < K ? kLeafEval<Q>.E[c][b] : 0.0;
        kk[i] = b < K ? kKappa<Q>.v[b] : 0.0;
    }
    const int p1 = min(p0 + kLeafEvalPar, n_par);
    for (int pi = p0; pi < p1; ++pi) {
        const int32_t child = parents[2 * pi + 1] + c;  // 8 consecutive children
        const double *__restrict__ lp = Lam + (int64_t)parents[2 * pi] * ldk;
        const double *__restrict__ lc = Lam + (int64_t)child * ldk;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int b = j + 8 * i;
            if (b < K) s = fma(kk[i], lc[b], fma(ke[i], lp[b], s));
        }
        s += __shfl_xor(s, 1, kWave);
        s += __shfl_xor(s, 2, kWave);
        s += __shfl_xor(s, 4, kWave);
        if (j == 0) {
            const int32_t leaf = cell_leaf[child];
            const double a = geom[leaf].w;
            u[leaf] = fma(s, a * a * a, u[leaf]);
        }
    }
}

// ---- M2L in the harmonic reduction ----------------------------------------------------------------
// With the scaled coefficients (M^b = (-1)^|b| m^b / (b! a^|b|), Lambda^a = lambda^a a! a^|a|) the
// interaction is Lambda^a = sum_{|a| + |b| <= Q} G_{a+b} M^b, G_g = a^|g| D^g G(x_w - x_w'). G is
// harmonic, so G_{g + 2e_z} = -G_{g + 2e_x} - G_{g + 2e_y} (all three of degree |g| + 2). Hence,
// exactly (the constraint |a| + |b| <= Q only involves degrees, which these maps keep):
//  * the moments fold onto b_z <= 1: Mr^b = sum_k (-1)^k sum_{i + j = k} C(k, i)
//    M^{b - 2i e_x - 2j e_y + 2k e_z}, and Lambda^a = sum_{b_z <= 1} G_{a+b} Mr^b;
//  * Lambda^a for a_z >= 2 follows from the a_z <= 1 ones: with k = floor(a_z / 2),
//    Lambda^a = (-1)^k sum_{i + j = k} C(k, i) Lambda^{a - 2k e_z + 2i e_x + 2j e_y}.
// So the pair loop runs over a_z <= 1 and b_z <= 1 only: sum_{n + m <= Q} (2n + 1)(2m + 1) FMAs per
// pair (532 at Q = 6, against C(Q + 6, 6) = 924 over all multi-indices), and a source row holds
// (Q + 1)^2 folded moments instead of K.
template <int Q>
struct RTables {
    static constexpr ReducedIndex<Q> ri{};
    static constexpr ExpandTable<Q> ex{};
};

// acc[a - A0] += G_{a+b} * Mr^b for the reduced a in [A0, A1) with |a| + |b| <= Q (straight-line
// code from the index tables); column b touches a < min(A1, (Q - |b| + 1)^2).
template <int Q, int A0, int B, class T, class GP, int... A>
__device__ __forceinline__ void m2l_column(T *acc, GP G, T mb, std::integer_sequence<int, A...>)
{
    constexpr auto &ri = RTables<Q>::ri;
    ((acc[A] = fma(G[ri.sum(A0 + A, B)], mb, acc[A])), ...);
}

template <int Q, int A0, int A1, int B, class T>
__device__ __forceinline__ void m2l_beta_reg(T *acc, const T *__restrict__ G, T mb)
{
    constexpr int n = nreduced(Q - RTables<Q>::ri.deg[B]);
    constexpr int hi = n < A1 ? n : A1;
    if constexpr (hi > A0) m2l_column<Q, A0, B>(acc, G, mb, std::make_integer_sequence<int, hi - A0>{});
}

// Block (a in [A0, A1)) x (b in [B0, B0 + NB)) with the lane's folded source moments in registers:
// m[b - B0] holds Mr^b.
template <int Q, int A0, int A1, int B0, class T, int... Bs>
__device__ __forceinline__ void m2l_block_reg(T *acc, const T *__restrict__ G, const T *m,
                                             std::integer_sequence<int, Bs...>)
{
    (m2l_beta_reg<Q, A0, A1, B0 + Bs>(acc, G, m[Bs]), ...);
}

// Lambda^a (full position FA) from the reduced accumulators of the block starting at A0.
template <int Q, int A0, int FA, class T, int... Ts>
__device__ __forceinline__ double expand_one(const T *acc, std::integer_sequence<int, Ts...>)
{
    constexpr auto &ex = RTables<Q>::ex;
    return (0.0 + ... + (ex.c[FA][Ts] * (double)acc[ex.src[FA][Ts] - A0]));
}

template <int Q, int A0, int FA0, bool kAdd, class T, int... Fs>
__device__ __forceinline__ void store_expanded(const T *acc, double scale, double *__restrict__ dst, int64_t stride,
                                               std::integer_sequence<int, Fs...>)
{
    constexpr auto &ex = RTables<Q>::ex;
    ((kAdd ? (void)(dst[Fs * stride] += scale * expand_one<Q, A0, FA0 + Fs>(
                        acc, std::make_integer_sequence<int, ex.n[FA0 + Fs]>{}))
           : (void)(dst[Fs * stride] = scale * expand_one<Q, A0, FA0 + Fs>(
                        acc, std::make_integer_sequence<int, ex.n[FA0 + Fs]>{}))),
     ...);
}

// Lane l takes lane l - 1's value; lane 0 keeps its own (DPP wave shift right by one lane; a double
// moves as its two 32-bit halves).
__device__ __forceinline__ int shift_up_b32(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ float shift_up(float v) { return __int_as_float(shift_up_b32(__float_as_int(v))); }
__device__ __forceinline__ double shift_up(double v)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = shift_up_b32((int)(uint32_t)b), hi = shift_up_b32((int)(b >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD b mod 8). XCD x runs
// the tasks [begin[x], begin[x + 1]), a spatially contiguous range, so that neighbouring targets
// share its L2; the ranges carry about equal work. Launch 8 * (longest range) workgroups.
struct XcdRanges {
    int32_t begin[kXcds + 1];
};
__device__ __forceinline__ int xcd_task(const XcdRanges &r)
{
    const int x = (int)(blockIdx.x % kXcds);
    const int t = r.begin[x] + (int)(blockIdx.x / kXcds);
    return t < r.begin[x + 1] ? t : -1;
}

// Interaction kernel with lane shifts. The plan lays a task's targets along rows (lane l + 1 one or
// two cells after lane l, except at the task's head lanes) and orders its slots so that
// consecutive offsets step by that many cells along the same axis: at a slot without the gather
// bit every lane's new source is the previous slot's source of the lane below, so the folded source
// moments stay in registers, move up one lane by a DPP shift, and only the head lanes read a row,
// instead of 64 lanes gathering 64 rows. Every slot names the real source of every lane (the zero
// row where there is no cell) and, in bit 31, whether the offset is in the lane's list; only those
// lanes accumulate. One launch covers the block a in [A0, A1), b in [B0, B1) of the reduced sums;
// [A0, A1) is a whole band of degrees, so the block expands its accumulators to every Lambda^a of
// those degrees. The launches of a full interaction phase tile the reduced triangle in blocks that
// fit 128 registers (four waves per SIMD, which covers the latency of the row reads at the start
// of each slot) or 256 (two waves); the block with B0 = 0 writes Lambda^a, the others add to it and
// are launched after it.
template <int Q, class T, int A0, int A1, int B0, int B1, int kWaves>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kWaves, kWaves))) void m2l_shift_kernel(
    XcdRanges ranges, const M2LTask *__restrict__ tasks, const int32_t *__restrict__ targets,
    const int32_t *__restrict__ slot_off, const uint32_t *__restrict__ slot_src, const T *__restrict__ G,
    const T *__restrict__ Mr, double *__restrict__ partial, double *__restrict__ Lam, int32_t ldr, int32_t ldk)
{
    constexpr int NA = A1 - A0, NB = B1 - B0;
    constexpr auto &ri = RTables<Q>::ri;
    constexpr int D0 = ri.deg[A0], D1 = ri.deg[A1 - 1];
    static_assert(A0 == D0 * D0 && A1 == (D1 + 1) * (D1 + 1), "the a range must be a band of whole degrees");
    constexpr int FA0 = D0 == 0 ? 0 : ncoef(D0 - 1), FA1 = ncoef(D1);
    const int ti = xcd_task(ranges);
    if (ti < 0) return;
    const M2LTask task = tasks[ti];
    const int lane = threadIdx.x;
    const bool head = ((task.heads >> lane) & 1ull) != 0ull;
    const int n = task.n_slots;
    const int64_t s0 = task.slot_begin;
    T acc[NA], m[NB];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = T(0);
    if (n > 0) {
        int32_t ow = slot_off[s0], ow1 = 0;
        uint32_t w = slot_src[s0 * kWave + lane], w1 = 0;
        if (n > 1) {
            ow1 = slot_off[s0 + 1];
            w1 = slot_src[(s0 + 1) * kWave + lane];
        }
        for (int j = 0; j < n; ++j) {
            int32_t ow2 = 0;  // the slot words are read two slots ahead
            uint32_t w2 = 0;
            if (j + 2 < n) {
                ow2 = slot_off[s0 + j + 2];
                w2 = slot_src[(s0 + j + 2) * kWave + lane];
            }
            const T *__restrict__ Ms = Mr + (int64_t)(w & 0x7FFFFFFFu) * ldr + B0;
            if (ow < 0 || j == 0) {  // gather the sources of all lanes
#pragma unroll
                for (int b = 0; b < NB; ++b) m[b] = Ms[b];
            } else {  // shift by one lane; the head lanes then read their new source
#pragma unroll
                for (int b = 0; b < NB; ++b) m[b] = shift_up(m[b]);
                if (head) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) m[b] = Ms[b];
                }
            }
            if (w >> 31)
                m2l_block_reg<Q, A0, A1, B0>(acc, G + (int64_t)(ow & 0x7FFFFFFF) * ldk, m,
                                             std::make_integer_sequence<int, NB>{});
            ow = ow1, w = w1, ow1 = ow2, w1 = w2;
        }
    }
    // keep the FP64 conversions below the loop (folded into the loop's exit they would hold all NA
    // results in FP64 at once, twice the registers)
#pragma unroll
    for (int a = 0; a < NA; ++a) asm volatile("" : "+v"(acc[a]));
    const int32_t t = targets[(int64_t)ti * kWave + lane];
    if (t < 0) return;
    const double inv_a = ldexp(1.0, task.level);
    if (task.out < 0)
        store_expanded<Q, A0, FA0, (B0 > 0)>(acc, inv_a, Lam + (int64_t)t * ldk + FA0, 1,
                                             std::make_integer_sequence<int, FA1 - FA0>{});
    else  // [piece][a][lane]: coalesced
        store_expanded<Q, A0, FA0, (B0 > 0)>(acc, inv_a, partial + ((int64_t)task.out * ldk + FA0) * kWave + lane,
                                             kWave, std::make_integer_sequence<int, FA1 - FA0>{});
}

// Split tasks: Lambda_t = sum of the pieces' partial local coefficients, in piece order. Block
// (split, g) handles coefficients 4g .. 4g + 3 of the split's 64 targets, one thread per (a, lane);
// a task of level l has ncoef(q_l) coefficients.
__global__ __launch_bounds__(256) void m2l_combine_kernel(const M2LSplit *__restrict__ splits,
                                                          const M2LTask *__restrict__ tasks,
                                                          const int32_t *__restrict__ targets,
                                                          const double *__restrict__ partial,
                                                          double *__restrict__ Lam, const LevelOrders lo)
{
    const M2LSplit sp = splits[blockIdx.x];
    const int lane = threadIdx.x & (kWave - 1);
    const int a = 4 * (int)blockIdx.y + (int)(threadIdx.x / kWave);
    const int32_t t = targets[(int64_t)sp.task * kWave + lane];
    if (t < 0 || a >= lo.k[tasks[sp.task].level]) return;
    const double *__restrict__ src = partial + ((int64_t)sp.first * lo.ldk + a) * kWave + lane;
    double s = 0.0;
    for (int k = 0; k < sp.count; ++k) s += src[(int64_t)k * lo.ldk * kWave];
    Lam[(int64_t)t * lo.ldk + a] = s;
}

// ---- interaction phase on the matrix cores (BCV_MIXED_SPLIT16, q = 6) ------------------------------
// For one slot (one offset o_k shared by the task's 64 targets) the reduced interaction is a matrix
// product
//     Lr[a][t] += sum_b T_k[a][b] Mr[b][src(t)],   T_k[a][b] = 4 pi G_{a+b}(o_k) where |a| + |b| <= 6,
// over the 49 reduced multi-indices a, b (degree-major: the (d + 1)^2 of degree <= d come first). It
// runs as v_mfma_f32_16x16x32_f16: the 64 targets form four column sets of 16 (target t = 4n + T is
// column n of set T), b is cut into two K-chunks (b < 32 and 32 <= b < 64, zero beyond 48) and a into
// row blocks of 16. The degree truncation leaves four nonzero tiles (row block, chunk) = (0, 0), (0, 1),
// (1, 0), (2, 0); row a = 48 (degree 6) meets b = 0 only and runs on the vector units.
// Precision: every FP32 operand x is split into hi = fp16(x) and lo = fp16(x - hi), and the products
// hi*hi, hi*lo and lo*hi accumulate in FP32 (the lo*lo term, about 2^-22 relative, is dropped).
// Lane layout of the instruction: A[i][k] in lane i + 16 (k / 8), element k % 8; B[k][n] in lane
// n + 16 (k / 8), element k % 8; D[i][n] in lane n + 16 (i / 4), element i % 4.
// Source rows: a cell's folded moments times 2^(3 level) / S (S the power of two at or above max |f|,
// so every value is at most a few units), as FP16 hi[64] then lo[64] (kSplitRowHalves). Lane
// (n, g = lane / 16) of set T holds the g-th 8 values of both chunks of target 4n + T's source, hi and
// lo: four 16-byte words.
// Shifts: at a shifting slot target t takes target t - 1's previous source (the lane-shift kernel's
// relation). With t = 4n + T that is set T - 1 -> set T for T >= 1, the same lanes (a renaming of
// register sets), and set 3 -> set 0 one column up (DPP row_shr:1 inside each 16-lane row); column 0
// of set 0 is target 0, always a head lane, which reads its row. The renaming rotates four register
// sets and is unrolled over four slots: at slot j logical set T is buffer (T - j) mod 4.
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));

constexpr int kSplitTiles = 4;
constexpr int kTileBlock[kSplitTiles] = {0, 0, 1, 2};   // row block of each tile
constexpr int kTileChunk[kSplitTiles] = {0, 1, 0, 0};   // K-chunk of each tile
constexpr int kTileGroups[kSplitTiles] = {4, 3, 2, 1};  // k-groups of 8 that hold nonzero entries

struct SrcPart {  // this lane's 8 values of both chunks, hi and lo
    u4_t h0, h1, l0, l1;
};

__device__ __forceinline__ uint32_t row_shr1(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x111, 0xf, 0xf, false);
}
__device__ __forceinline__ u4_t row_shr1(u4_t v)
{
    return u4_t{row_shr1(v.x), row_shr1(v.y), row_shr1(v.z), row_shr1(v.w)};
}
__device__ __forceinline__ SrcPart row_shr1(const SrcPart &s)
{
    return SrcPart{row_shr1(s.h0), row_shr1(s.h1), row_shr1(s.l0), row_shr1(s.l1)};
}
__device__ __forceinline__ SrcPart load_src(const u4_t *__restrict__ rows, uint32_t row, int g)
{
    const u4_t *r = rows + (size_t)row * (kSplitRowHalves / 8);
    return SrcPart{r[g], r[4 + g], r[8 + g], r[12 + g]};
}
__device__ __forceinline__ h8_t as_h8(u4_t v) { return __builtin_bit_cast(h8_t, v); }
__device__ __forceinline__ f4_t mfma3(u4_t ah, u4_t al, u4_t bh, u4_t bl, f4_t c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(ah), as_h8(bh), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(ah), as_h8(bl), c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(al), as_h8(bh), c, 0, 0, 0);
}

// Partial maxima of |f|: block b writes the maximum over its grid-stride share (kFscaleParts blocks).
__global__ __launch_bounds__(256) void fmax_partial_kernel(int64_t n, const double *__restrict__ f,
                                                           float *__restrict__ part)
{
    __shared__ float sm[256];
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = fmaxf(m, (float)fabs(f[i]));
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

struct LevelStarts {
    int32_t s[kMaxLevel + 2];
    int32_t L;
};

// FP16 hi/lo rows from the FP32 folded rows: row c of level l gets Mr * 2^(3 l) / S, S = the power of two
// at or above max |f| (from the partial maxima; 1 for f = 0), which block 0 also stores after them.
// One thread per (row, j < 64); entries j >= ldr are zero.
__global__ __launch_bounds__(256) void split_rows_kernel(int64_t n_rows, const float *__restrict__ rows32,
                                                         int32_t ldr, uint16_t *__restrict__ rows16,
                                                         float *__restrict__ fscale, const LevelStarts ls)
{
    __shared__ float sm[kFscaleParts];
    sm[threadIdx.x] = fscale[threadIdx.x];
    __syncthreads();
    for (int h = kFscaleParts / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + h]);
        __syncthreads();
    }
    int e = 0;
    (void)frexpf(sm[0], &e);  // sm[0] = m 2^e, 1/2 <= m < 1
    const float S = sm[0] > 0.0f ? ldexpf(1.0f, e) : 1.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0) fscale[kFscaleParts] = S;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t row = idx >> 6;
    const int j = (int)(idx & 63);
    if (row >= n_rows) return;
    int lev = 0;
    while (lev < ls.L && row >= ls.s[lev + 1]) ++lev;
    const float v = j < ldr ? rows32[row * ldr + j] * ldexpf(1.0f / S, 3 * lev) : 0.0f;
    const _Float16 hi = (_Float16)v;
    const _Float16 lo = (_Float16)(v - (float)hi);
    rows16[row * kSplitRowHalves + j] = __builtin_bit_cast(uint16_t, hi);
    rows16[row * kSplitRowHalves + 64 + j] = __builtin_bit_cast(uint16_t, lo);
}

template <int Q>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2, 2))) void m2l_mfma_kernel(
    XcdRanges ranges, const M2LTask *__restrict__ tasks, const int32_t *__restrict__ targets,
    const int32_t *__restrict__ slot_off, const uint32_t *__restrict__ slot_src, const uint64_t *__restrict__ slot_mask,
    const u4_t *__restrict__ Atab, const float *__restrict__ G48, const u4_t *__restrict__ rows,
    const float *__restrict__ fscale, double *__restrict__ partial, double *__restrict__ Lam, int32_t ldk)
{
    static_assert(Q == 6, "the tile set is that of q = 6");
    constexpr int R = nreduced(Q), FA1 = ncoef(Q);
    __shared__ float tr[R][kWave + 1];
    const int ti = xcd_task(ranges);
    if (ti < 0) return;
    const M2LTask task = tasks[ti];
    const int lane = threadIdx.x, n = lane & 15, g = lane >> 4;
    const int32_t my_target = targets[(int64_t)ti * kWave + lane];
    const uint64_t idle = __ballot(my_target < 0);                          // targets without a cell
    const uint32_t heads4 = (uint32_t)((task.heads >> (4 * n)) & 0xFull);   // bit T: target 4n + T is a head
    const int nsl = task.n_slots;
    const int64_t s0 = task.slot_begin;
    f4_t acc[3][4];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int T = 0; T < 4; ++T) acc[b][T] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
    float acc48[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    SrcPart buf[4];
    const u4_t zero4 = u4_t{0u, 0u, 0u, 0u};
#pragma unroll
    for (int T = 0; T < 4; ++T) buf[T] = SrcPart{zero4, zero4, zero4, zero4};

    // The slot loop runs in groups of four (the rotation period); slots past the end of the list
    // are idle (zero operands, nothing read), so that every group has the same straight-line code.
    // A operands: a lane's k-groups beyond kTileGroups hold zeros for every offset, so those
    // registers are cleared once and never loaded. The slot words (offset, mask, the four source
    // words of the lane's targets) are read one slot ahead.
    u4_t ah[kSplitTiles], al[kSplitTiles];
#pragma unroll
    for (int tl = 0; tl < kSplitTiles; ++tl) ah[tl] = al[tl] = zero4;
    struct SlotWords {
        int32_t ow;
        uint64_t mk;
        u4_t w;
    };
    auto load_words = [&](int j) {
        SlotWords sw{0, 0ull, zero4};
        if (j < nsl) {
            const int64_t sl = s0 + j;
            sw.ow = slot_off[sl];
            sw.mk = slot_mask[sl];
            if (sw.ow < 0 || heads4) sw.w = *reinterpret_cast<const u4_t *>(slot_src + sl * kWave + 4 * n);
        }
        return sw;
    };
    auto body = [&](int j, auto rot_c, const SlotWords &sw) {
        constexpr int ROT = decltype(rot_c)::value;  // logical set T is buf[(T + ROT) & 3]
        const bool live = j < nsl;
        const int off = sw.ow & 0x7FFFFFFF;
#pragma unroll
        for (int tl = 0; tl < kSplitTiles; ++tl)
            if (live && g < kTileGroups[tl]) {
                const u4_t *p = Atab + ((int64_t)(off * kSplitTiles + tl) * 2) * kWave + lane;
                ah[tl] = p[0];
                al[tl] = p[kWave];
            }
        const float g48 = live ? G48[off] : 0.0f;
        const bool gather = live && sw.ow < 0;  // the plan sets the gather bit on every piece's first slot
        if (!gather) buf[ROT] = row_shr1(buf[ROT]);  // old set 3 -> new set 0, one column up
        const uint32_t need = gather ? 0xFu : (live ? heads4 : 0u);
#pragma unroll
        for (int T = 0; T < 4; ++T)
            if ((need >> T) & 1u) buf[(T + ROT) & 3] = load_src(rows, sw.w[T] & 0x7FFFFFFFu, g);
        // targets whose list lacks the offset take a zero column (a full slot keeps every column;
        // an idle slot none)
        const uint32_t mbits = live ? ((uint32_t)((sw.mk >> (4 * n)) & 0xFull) | ((sw.mk | idle) == ~0ull ? 0xFu : 0u))
                                    : 0u;
#pragma unroll
        for (int T = 0; T < 4; ++T) {
            const uint32_t keep = 0u - ((mbits >> T) & 1u);
            const SrcPart &v = buf[(T + ROT) & 3];
            const SrcPart x{v.h0 & keep, v.h1 & keep, v.l0 & keep, v.l1 & keep};
            acc[0][T] = mfma3(ah[0], al[0], x.h0, x.l0, acc[0][T]);
            acc[1][T] = mfma3(ah[2], al[2], x.h0, x.l0, acc[1][T]);
            acc[2][T] = mfma3(ah[3], al[3], x.h0, x.l0, acc[2][T]);
            acc[0][T] = mfma3(ah[1], al[1], x.h1, x.l1, acc[0][T]);
            const h8_t bh = as_h8(x.h0), bl = as_h8(x.l0);
            acc48[T] = fmaf(g48, (float)bh[0] + (float)bl[0], acc48[T]);
        }
    };
    SlotWords w0 = load_words(0), w1;
    for (int j = 0; j < nsl; j += 4) {
        w1 = load_words(j + 1);
        body(j, std::integral_constant<int, 0>{}, w0);
        w0 = load_words(j + 2);
        body(j + 1, std::integral_constant<int, 3>{}, w1);
        w1 = load_words(j + 3);
        body(j + 2, std::integral_constant<int, 2>{}, w0);
        w0 = load_words(j + 4);
        body(j + 3, std::integral_constant<int, 1>{}, w1);
    }
    // transpose through LDS: tr[a][t], then lane t expands its 49 reduced coefficients
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int T = 0; T < 4; ++T)
#pragma unroll
            for (int e = 0; e < 4; ++e) tr[16 * b + 4 * g + e][4 * n + T] = acc[b][T][e];
    if (g == 0)
#pragma unroll
        for (int T = 0; T < 4; ++T) tr[R - 1][4 * n + T] = acc48[T];
    __syncthreads();
    float lr[R];
#pragma unroll
    for (int a = 0; a < R; ++a) lr[a] = tr[a][lane];
    if (my_target < 0) return;
    // Lambda = a^-1 (S 2^(-3 level) / (4 pi)) lr with a = 2^-level
    const double scale = (double)fscale[kFscaleParts] * ldexp(kInv4Pi, -2 * task.level);
    if (task.out < 0)
        store_expanded<Q, 0, 0, false>(lr, scale, Lam + (int64_t)my_target * ldk, 1,
                                       std::make_integer_sequence<int, FA1>{});
    else
        store_expanded<Q, 0, 0, false>(lr, scale, partial + (int64_t)task.out * ldk * kWave + lane, kWave,
                                       std::make_integer_sequence<int, FA1>{});
}

// ---- near field + evaluation: one wave per work unit --------------------------------------------
// Row t of the near CSR holds the touching pairs in [row[t], split[t]) and the point-rule pairs in
// [split[t], row[t+1]); a unit covers a range of one row. Touching pairs cost one FMA; the
// point-rule loop fetches the next pair's source while it evaluates the current one. A unit that
// is its target's whole row writes u (adding the evaluation phase when Lam is given); the units
// of a longer row write partial sums that near_combine_kernel adds up.
// u_w += a^3 sum_a kappa_a Lambda^a over the leaf's n coefficients (its level's order; the kappa
// table is graded, so its first n entries are those of that order).
template <int Q>
__device__ __forceinline__ double eval_far(const double *__restrict__ lam, double a, int lane, int n)
{
    double s = 0.0;
    for (int k = lane; k < n; k += kWave) s = fma(kKappa<Q>.v[k], lam[k], s);
    return s * (a * a * a);
}

// Exact entry of a touching pair from its code (class + 1, + 8 if the source is the smaller cube) and
// the target's side: C_class a_small^5 / (4 pi), a_small = a_t / 2 for a smaller source (ratio 2).
__device__ __forceinline__ double touch_entry(uint32_t code, double a_t, const TouchValues &tv)
{
    const uint32_t cls = code >> 28;
    const double a = (cls & 8u) ? 0.5 * a_t : a_t;
    return tv.v[(cls & 7u) - 1] * (a * a) * (a * a) * a;
}

// sum over entries e in [e0, e1) of val[e] f[source(e)], this lane's share (the wave sums the lanes):
// entries e0 + lane + 64 k, four per lane per step.
template <class V>
__device__ __forceinline__ double assembled_dot(const uint32_t *__restrict__ col, const V *__restrict__ val,
                                                const double *__restrict__ f, int64_t e0, int64_t e1, int lane,
                                                double acc)
{
    int64_t e = e0 + lane;
    for (; e + 3 * kWave < e1; e += 4 * kWave) {
        uint32_t c[4];
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = col[e + k * kWave], v[k] = (double)val[e + k * kWave];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc = fma(v[k], f[c[k] & 0x0FFFFFFFu], acc);
    }
    for (; e < e1; e += kWave) acc = fma((double)val[e], f[col[e] & 0x0FFFFFFFu], acc);
    return acc;
}

// Units are dealt to the XCDs in contiguous target ranges (XcdRanges over units): workgroup b runs on
// XCD b mod 8 and its 4 waves take units begin[x] + 4 (b / 8) + wave.
template <int Q, bool kAssembled, bool kMixed>
__global__ __launch_bounds__(256) void near_eval_kernel(XcdRanges xr, const NearUnit *__restrict__ units,
                                                        const int64_t *__restrict__ split,
                                                        const uint32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const float *__restrict__ val32,
                                                        const double4 *__restrict__ geom,
                                                        const double *__restrict__ f,
                                                        const double *__restrict__ Lam,
                                                        const int32_t *__restrict__ leaf_cell, TouchValues tv,
                                                        int parts, double *__restrict__ partial,
                                                        double *__restrict__ u, const LevelOrders lo)
{
    constexpr int K = MultiIndex<Q>::K;
    const int lane = threadIdx.x & (kWave - 1);
    const int x = (int)(blockIdx.x % kXcds);
    const int64_t w = xr.begin[x] + (int64_t)(blockIdx.x / kXcds) * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= xr.begin[x + 1]) return;  // uniform per wave
    const NearUnit un = units[w];
    const int32_t t = un.target;
    const double4 gt = geom[t];
    double acc = 0.0;
    if (parts & BCV_PART_NEAR) {
        const int64_t e0 = un.begin, e1 = un.end;
        if (kAssembled && !kMixed) {
            acc = assembled_dot(col, val, f, e0, e1, lane, acc);
        } else if (kAssembled) {  // FP32 entries; the touching pairs exact, in FP64 (from the class
                                  // value, or per pair where the plan keeps FP64 entries: mapped meshes)
            const int64_t es = min(max(split[t], e0), e1);
            const double a_t = gt.w;
            for (int64_t e = e0 + lane; e < es; e += kWave) {
                const uint32_t code = col[e];
                acc = fma(val != nullptr ? val[e] : touch_entry(code, a_t, tv), f[code & 0x0FFFFFFFu], acc);
            }
            acc = assembled_dot(col, val32, f, es, e1, lane, acc);
        } else {
            const int64_t es = min(max(split[t], e0), e1);
            const double a_t = gt.w;
            for (int64_t e = e0 + lane; e < es; e += kWave) {  // touching pairs
                const uint32_t code = col[e];
                acc = fma(touch_entry(code, a_t, tv), f[code & 0x0FFFFFFFu], acc);
            }
            int64_t e = es + lane;
            double4 gs_next = make_double4(0.0, 0.0, 0.0, 1.0);
            double f_next = 0.0;
            if (e < e1) {
                const int32_t s = (int32_t)(col[e] & 0x0FFFFFFFu);
                gs_next = geom[s];
                f_next = f[s];
            }
            for (; e < e1; e += kWave) {
                const double4 gs = gs_next;
                const double fs = f_next;
                if (e + kWave < e1) {
                    const int32_t s = (int32_t)(col[e + kWave] & 0x0FFFFFFFu);
                    gs_next = geom[s];
                    f_next = f[s];
                }
                acc = fma(kMixed ? point_rule_f32(gt, gs) : point_rule(gt, gs), fs, acc);
            }
        }
    }
    if (un.out < 0 && (parts & BCV_PART_FAR) && Lam != nullptr)
        acc += eval_far<Q>(Lam + (int64_t)leaf_cell[t] * lo.ldk, gt.w, lane, lo.k[level_of_side(gt.w)]);
    acc = wave_sum(acc);
    if (lane == 0) {
        if (un.out < 0)
            u[t] = acc;
        else
            partial[un.out] = acc;
    }
}

// Rows cut into several units: u = sum of the partial sums in row order (+ evaluation phase).
template <int Q>
__global__ __launch_bounds__(256) void near_combine_kernel(int64_t n_splits, const NearSplit *__restrict__ splits,
                                                           const double *__restrict__ partial,
                                                           const double4 *__restrict__ geom,
                                                           const double *__restrict__ Lam,
                                                           const int32_t *__restrict__ leaf_cell,
                                                           double *__restrict__ u, const LevelOrders lo)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= n_splits) return;  // uniform per wave
    const NearSplit sp = splits[w];
    double v = 0.0;
    if (Lam != nullptr) {
        const double a = geom[sp.target].w;
        v = eval_far<Q>(Lam + (int64_t)leaf_cell[sp.target] * lo.ldk, a, lane, lo.k[level_of_side(a)]);
    }
    for (int k = lane; k < sp.count; k += kWave) v += partial[sp.first + k];  // fixed order per lane
    v = wave_sum(v);
    if (lane == 0) u[sp.target] = v;
}

// u[i] *= scale[i] (the side^5 factor of a domain that is not the unit cube).
__global__ __launch_bounds__(256) void scale_kernel(int64_t n, const double *__restrict__ scale, double *__restrict__ u)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] *= scale[i];
}

// ---- evaluation phase alone (near field computed concurrently): u += a^3 sum_a kappa_a Lambda^a --
// One wave per leaf.
template <int Q>
__global__ __launch_bounds__(256) void eval_add_kernel(int64_t n_leaves, const double4 *__restrict__ geom,
                                                       const double *__restrict__ Lam,
                                                       const int32_t *__restrict__ leaf_cell,
                                                       double *__restrict__ u, const LevelOrders lo)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t t = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (t >= n_leaves) return;
    const double a = geom[t].w;
    const double s = wave_sum(eval_far<Q>(Lam + (int64_t)leaf_cell[t] * lo.ldk, a, lane, lo.k[level_of_side(a)]));
    if (lane == 0) u[t] += s;
}

// The same for a list of leaves (those off the finest level, whose leaves leaf_eval_kernel
// evaluates): 8 lanes per leaf, lane j of a group takes coefficients j, j + 8, ...
template <int Q>
__global__ __launch_bounds__(256) void eval_list_kernel(int64_t n, const int32_t *__restrict__ list,
                                                        const double4 *__restrict__ geom,
                                                        const double *__restrict__ Lam,
                                                        const int32_t *__restrict__ leaf_cell,
                                                        double *__restrict__ u, const LevelOrders lo)
{
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int j = threadIdx.x & 7;
    const int32_t t = i < n ? list[i] : 0;
    double s = 0.0, a = 0.0;
    if (i < n) {
        a = geom[t].w;
        const int nk = lo.k[level_of_side(a)];
        const double *__restrict__ lam = Lam + (int64_t)leaf_cell[t] * lo.ldk;
        for (int k = j; k < nk; k += 8) s = fma(kKappa<Q>.v[k], lam[k], s);
    }
    s += __shfl_xor(s, 1, kWave);
    s += __shfl_xor(s, 2, kWave);
    s += __shfl_xor(s, 4, kWave);
    if (i < n && j == 0) u[t] = fma(s, a * a * a, u[t]);
}

// ---- BtV (Algorithm 3): boundary moments and the near field of boundary faces --------------------

// Moments of every leaf from its boundary faces (zero for leaves without one): one thread per
// (leaf, coefficient).
template <int Q, class TR>
__global__ void btv_p2m_kernel(int64_t n_leaves, const int32_t *__restrict__ leaf_cell,
                               const double4 *__restrict__ geom, const int32_t *__restrict__ leaf_faces,
                               const uint32_t *__restrict__ faces, const double *__restrict__ qf,
                               const double *__restrict__ gf, double *__restrict__ M, TR *__restrict__ Mr)
{
    constexpr int K = MultiIndex<Q>::K, R = nreduced(Q);
    const int64_t leaf = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;  // one wave per leaf
    const int lane = threadIdx.x % kWave;
    if (leaf >= n_leaves) return;
    const double a = geom[leaf].w;
    const int64_t c = leaf_cell[leaf];
    const int32_t f0 = leaf_faces[leaf], f1 = leaf_faces[leaf + 1];
    for (int b = lane; b < K; b += kWave) {
        double m = 0.0;
        for (int32_t f = f0; f < f1; ++f) {
            const int type = (int)(faces[f] >> 28);
            m += a * (a * qf[f] * kFaceKappa<Q>.phi[type][b] - gf[f] * kFaceKappa<Q>.psi[type][b]);
        }
        M[c * K + b] = m;
    }
    for (int b = lane; b < R; b += kWave) {
        double m = 0.0;
        for (int32_t f = f0; f < f1; ++f) {
            const int type = (int)(faces[f] >> 28);
            m += a * (a * qf[f] * kFoldedFaceKappa<Q>.phi[type][b] - gf[f] * kFoldedFaceKappa<Q>.psi[type][b]);
        }
        Mr[c * R + b] = (TR)m;
    }
}

__device__ __forceinline__ double pick3(const double v[3], int d) { return d == 0 ? v[0] : (d == 1 ? v[1] : v[2]); }
__device__ __forceinline__ double rsq(double x) { return rsqrt_pos(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Point rule of a cell (2x2x2 Gauss points) against a boundary face (2x2 Gauss points): the
// single-layer entry sv = sum w w' G and the double-layer entry dv = sum w w' n.(x - y)/(4 pi r^3).
// The 32 kernel evaluations run in R (double, or float in the mixed path with the per-axis
// differences formed in FP64 first, as in the volume point rule).
template <class R>
__device__ __forceinline__ void face_rule(const double4 gt, const double4 gf, int ax, int side, double &sv,
                                          double &dv)
{
    const double lt[3] = {gt.x, gt.y, gt.z}, lf[3] = {gf.x, gf.y, gf.z};
    const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
    const double plane = pick3(lf, ax) + side * gf.w;
    const R dn[2] = {(R)(pick3(lt, ax) + gt.w * kNode0 - plane), (R)(pick3(lt, ax) + gt.w * kNode1 - plane)};
    R p1[4], p2[4];
    {
        const double x0 = pick3(lt, o1) + gt.w * kNode0, x1 = pick3(lt, o1) + gt.w * kNode1;
        const double y0 = pick3(lf, o1) + gf.w * kNode0, y1 = pick3(lf, o1) + gf.w * kNode1;
        const R d[4] = {(R)(x0 - y0), (R)(x0 - y1), (R)(x1 - y0), (R)(x1 - y1)};
#pragma unroll
        for (int m = 0; m < 4; ++m) p1[m] = d[m] * d[m];
    }
    {
        const double x0 = pick3(lt, o2) + gt.w * kNode0, x1 = pick3(lt, o2) + gt.w * kNode1;
        const double y0 = pick3(lf, o2) + gf.w * kNode0, y1 = pick3(lf, o2) + gf.w * kNode1;
        const R d[4] = {(R)(x0 - y0), (R)(x0 - y1), (R)(x1 - y0), (R)(x1 - y1)};
#pragma unroll
        for (int m = 0; m < 4; ++m) p2[m] = d[m] * d[m];
    }
    R s = 0, k = 0;
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const R dn2 = dn[n] * dn[n];
        R kn = 0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const R x = dn2 + p1[a];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const R ir = rsq(x + p2[b]);
                s += ir;
                kn += ir * ir * ir;
            }
        }
        k += dn[n] * kn;
    }
    const double w = (gt.w * gt.w * gt.w * 0.125) * (gf.w * gf.w * 0.25) * kInv4Pi;
    sv = (double)s * w;
    dv = (side ? 1.0 : -1.0) * (double)k * w;
}

// u_w = sum over the near faces of V q - K g (touching pairs from the class table, scaled by a^4
// and a^3; the others by the point rule), plus the evaluation phase; one wave per work unit.
template <int Q, bool kMixed>
__global__ __launch_bounds__(256) void btv_near_kernel(int64_t n_units, const NearUnit *__restrict__ units,
                                                       const uint32_t *__restrict__ col,
                                                       const uint32_t *__restrict__ faces,
                                                       const double4 *__restrict__ geom,
                                                       const double *__restrict__ qf, const double *__restrict__ gf,
                                                       const double *__restrict__ touch,
                                                       const double *__restrict__ Lam,
                                                       const int32_t *__restrict__ leaf_cell,
                                                       double *__restrict__ partial, double *__restrict__ u)
{
    constexpr int K = MultiIndex<Q>::K;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= n_units) return;  // uniform per wave
    const NearUnit un = units[w];
    const int32_t t = un.target;
    const double4 gt = geom[t];
    double acc = 0.0;
    for (int64_t e = un.begin + lane; e < un.end; e += kWave) {
        const uint32_t code = col[e];
        const uint32_t f = code & 0x00FFFFFFu, cls = code >> 24;
        const double q = qf[f], g = gf[f];
        if (cls) {
            const double a = gt.w, a3 = a * a * a;
            acc += touch[cls - 1] * a3 * a * q - touch[kFaceClasses + cls - 1] * a3 * g;
        } else {
            const uint32_t fw = faces[f];
            const int type = (int)(fw >> 28);
            double sv, dv;
            face_rule<typename std::conditional<kMixed, float, double>::type>(gt, geom[fw & 0x0FFFFFFFu], type >> 1,
                                                                              type & 1, sv, dv);
            acc += sv * q - dv * g;
        }
    }
    if (un.out < 0 && Lam != nullptr) acc += eval_far<Q>(Lam + (int64_t)leaf_cell[t] * K, gt.w, lane, K);
    acc = wave_sum(acc);
    if (lane == 0) {
        if (un.out < 0)
            u[t] = acc;
        else
            partial[un.out] = acc;
    }
}

// ---- VtB (Algorithm 2): face integrals of the volume potential -------------------------------------

// Evaluation at a face of cell w (side a, face type): int_face sum_a lambda^a (y - x_w)^a dS
// = a^2 sum_a Lambda^a (-1)^|a| phi_type^a (the face table of the boundary moments without the
// moments' sign); this lane's share of the sum.
template <int Q>
__device__ __forceinline__ double eval_face(const double *__restrict__ lam, double a, int type, int lane)
{
    constexpr int K = MultiIndex<Q>::K;
    double s = 0.0;
    for (int k = lane; k < K; k += kWave) {
        const double phi = kFaceKappa<Q>.phi[type][k];
        s = fma((Tables<Q>::mi.deg[k] & 1) ? -phi : phi, lam[k], s);
    }
    return s * (a * a);
}

// u_f = sum over the near sources s of V_sf f_s (touching pairs from the class table, scaled by
// a^4; the others by the single-layer part of the face point rule), plus the evaluation at the face;
// one wave per work unit (targets are faces).
template <int Q, bool kMixed>
__global__ __launch_bounds__(256) void vtb_near_kernel(int64_t n_units, const NearUnit *__restrict__ units,
                                                       const uint32_t *__restrict__ col,
                                                       const uint32_t *__restrict__ faces,
                                                       const double4 *__restrict__ geom,
                                                       const double *__restrict__ f, const double *__restrict__ touch,
                                                       const double *__restrict__ Lam,
                                                       const int32_t *__restrict__ leaf_cell,
                                                       double *__restrict__ partial, double *__restrict__ u)
{
    constexpr int K = MultiIndex<Q>::K;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= n_units) return;  // uniform per wave
    const NearUnit un = units[w];
    const uint32_t fw = faces[un.target];
    const int32_t leaf = (int32_t)(fw & 0x0FFFFFFFu);
    const int type = (int)(fw >> 28);
    const double4 gf = geom[leaf];
    double acc = 0.0;
    for (int64_t e = un.begin + lane; e < un.end; e += kWave) {
        const uint32_t code = col[e];
        const int32_t s = (int32_t)(code & 0x00FFFFFFu);
        const uint32_t cls = code >> 24;
        if (cls) {
            const double a = gf.w;
            acc += touch[cls - 1] * (a * a) * (a * a) * f[s];
        } else {
            double sv, dv;
            face_rule<typename std::conditional<kMixed, float, double>::type>(geom[s], gf, type >> 1, type & 1, sv,
                                                                              dv);
            acc += sv * f[s];
        }
    }
    if (un.out < 0 && Lam != nullptr) acc += eval_face<Q>(Lam + (int64_t)leaf_cell[leaf] * K, gf.w, type, lane);
    acc = wave_sum(acc);
    if (lane == 0) {
        if (un.out < 0)
            u[un.target] = acc;
        else
            partial[un.out] = acc;
    }
}

// Face rows cut into several units: u_f = sum of the partial sums in row order (+ evaluation).
template <int Q>
__global__ __launch_bounds__(256) void vtb_combine_kernel(int64_t n_splits, const NearSplit *__restrict__ splits,
                                                          const double *__restrict__ partial,
                                                          const uint32_t *__restrict__ faces,
                                                          const double4 *__restrict__ geom,
                                                          const double *__restrict__ Lam,
                                                          const int32_t *__restrict__ leaf_cell,
                                                          double *__restrict__ u)
{
    constexpr int K = MultiIndex<Q>::K;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= n_splits) return;  // uniform per wave
    const NearSplit sp = splits[w];
    const uint32_t fw = faces[sp.target];
    const int32_t leaf = (int32_t)(fw & 0x0FFFFFFFu);
    double far = 0.0;
    if (Lam != nullptr)
        far = wave_sum(eval_face<Q>(Lam + (int64_t)leaf_cell[leaf] * K, geom[leaf].w, (int)(fw >> 28), lane));
    if (lane == 0) {
        double acc = 0.0;
        for (int k = 0; k < sp.count; ++k) acc += partial[sp.first + k];
        u[sp.target] = acc + far;
    }
}

// ---- plan-time assembly of the near-pair entries --------------------------------------------------
__global__ __launch_bounds__(256) void near_assemble_kernel(int64_t n_units, const NearUnit *__restrict__ units,
                                                            const uint32_t *__restrict__ col,
                                                            const double4 *__restrict__ geom, TouchValues tv,
                                                            double *__restrict__ val)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= n_units) return;
    const NearUnit un = units[w];
    const double4 gt = geom[un.target];
    for (int64_t e = un.begin + lane; e < un.end; e += kWave) val[e] = near_entry(col[e], gt, geom, tv);
}

// Level-dependent near-field rule (Sec. 4, near-field quadrature: fixed order on the finest level,
// raised on coarser levels): the listed entries are non-touching pairs (t, s) whose cells carry n_t
// and n_s Gauss points per axis; the entry is the n_t^3 x n_s^3-point tensor rule. One wave per
// entry, the point pairs spread over the lanes. gx, gw: node and weight tables on [0, 1], row n
// (16 wide) holding the n-point rule.
__global__ __launch_bounds__(256) void near_assemble_ordered_kernel(int64_t n, const int64_t *__restrict__ entry,
                                                                    const int32_t *__restrict__ target,
                                                                    const uint32_t *__restrict__ col,
                                                                    const double4 *__restrict__ geom,
                                                                    const int8_t *__restrict__ order,
                                                                    const double *__restrict__ gx,
                                                                    const double *__restrict__ gw,
                                                                    double *__restrict__ val)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= n) return;  // uniform per wave
    const int64_t e = entry[w];
    const int32_t t = target[w], s = (int32_t)(col[e] & 0x0FFFFFFFu);
    const double4 gt = geom[t], gs = geom[s];
    const int nt = order[t], ns = order[s];
    const int ps = ns * ns * ns, total = nt * nt * nt * ps;
    const double *xt = gx + 16 * nt, *wt = gw + 16 * nt, *xs = gx + 16 * ns, *ws = gw + 16 * ns;
    double acc = 0.0;
    for (int i = lane; i < total; i += kWave) {
        const int a = i / ps, b = i - a * ps;
        const int a1 = a % nt, a2 = (a / nt) % nt, a3 = a / (nt * nt);
        const int b1 = b % ns, b2 = (b / ns) % ns, b3 = b / (ns * ns);
        const double dx = (gt.x + gt.w * xt[a1]) - (gs.x + gs.w * xs[b1]);
        const double dy = (gt.y + gt.w * xt[a2]) - (gs.y + gs.w * xs[b2]);
        const double dz = (gt.z + gt.w * xt[a3]) - (gs.z + gs.w * xs[b3]);
        const double wgt = (wt[a1] * wt[a2] * wt[a3]) * (ws[b1] * ws[b2] * ws[b3]);
        acc += wgt / sqrt(dx * dx + dy * dy + dz * dz);
    }
    acc = wave_sum(acc);
    const double vt = gt.w * gt.w * gt.w, vs = gs.w * gs.w * gs.w;
    if (lane == 0) val[e] = acc * vt * vs * kInv4Pi;
}

// FP32 copy of the assembled entries (mixed precision).
__global__ __launch_bounds__(256) void narrow_kernel(int64_t n, const double *__restrict__ in, float *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

// ---- regular cube pairs (touching-integral self-similarity system) -------------------------------
constexpr int kMaxGauss = 16;
struct GaussRule {
    double x[kMaxGauss], w[kMaxGauss];
};

__global__ __launch_bounds__(256) void regular_cube_pairs_kernel(const int *__restrict__ deltas, int n_gauss,
                                                                 GaussRule rule, double *__restrict__ out)
{
    __shared__ double part[256];
    const int d0 = deltas[3 * blockIdx.x], d1 = deltas[3 * blockIdx.x + 1], d2 = deltas[3 * blockIdx.x + 2];
    const int n2 = n_gauss * n_gauss;
    const int64_t total = (int64_t)n2 * n2 * n2;
    double s = 0.0;
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int p0 = (int)(idx % n2), p1 = (int)((idx / n2) % n2), p2 = (int)(idx / ((int64_t)n2 * n2));
        // axis pair (g, h): x = node g of the first cube, y = d + node h of the second
        const double x0 = rule.x[p0 / n_gauss] - (d0 + rule.x[p0 % n_gauss]);
        const double x1 = rule.x[p1 / n_gauss] - (d1 + rule.x[p1 % n_gauss]);
        const double x2 = rule.x[p2 / n_gauss] - (d2 + rule.x[p2 % n_gauss]);
        const double w = rule.w[p0 / n_gauss] * rule.w[p0 % n_gauss] * rule.w[p1 / n_gauss] * rule.w[p1 % n_gauss] *
                         rule.w[p2 / n_gauss] * rule.w[p2 % n_gauss];
        s = fma(w, rsqrt(x0 * x0 + x1 * x1 + x2 * x2), s);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

TouchValues touch_values(const bcv_plan_s &p)
{
    TouchValues tv;
    for (int c = 0; c < kTouchClasses; ++c) tv.v[c] = p.touch_value[c];
    return tv;
}

void check_launch()
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(BCV_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
}

// Start and stop events of each phase of the current apply, if timing is on. A phase that does not
// run gets both events recorded back to back on the caller's stream (zero time).
struct PhaseMarks {
    const bcv_plan_s &p;
    int slot;
    bool done[BCV_N_PHASES] = {};
    explicit PhaseMarks(const bcv_plan_s &plan) : p(plan), slot(-1)
    {
        if (p.timing_used < p.timing_cap) slot = p.timing_used++;
    }
    hipEvent_t ev(int k, int which) const { return p.events[2 * (BCV_N_PHASES * slot + k) + which]; }
    void start(int k, hipStream_t st) const
    {
        if (slot >= 0) BCV_HIP(hipEventRecord(ev(k, 0), st));
    }
    void stop(int k, hipStream_t st)
    {
        if (slot >= 0) BCV_HIP(hipEventRecord(ev(k, 1), st));
        done[k] = true;
    }
    void finish(hipStream_t st)
    {
        for (int k = 0; k < BCV_N_PHASES; ++k)
            if (!done[k]) {
                start(k, st);
                stop(k, st);
            }
    }
};

// The largest expansion order of any level of the plan.
int max_order(const bcv_plan_s &p)
{
    int q = 0;
    for (int l = 0; l <= p.L; ++l) q = std::max(q, p.q_level[l]);
    return q;
}

LevelOrders level_orders(const bcv_plan_s &p)
{
    LevelOrders lo{};
    for (int l = 0; l <= kMaxLevel; ++l) {
        lo.k[l] = ncoef(p.q_level[l]);
        lo.r[l] = nreduced(p.q_level[l]);
    }
    lo.ldk = p.K;
    lo.ldr = p.R;
    return lo;
}

template <int Q>
void launch_near_q(const bcv_plan_s &p, const double *f, const double *lam, int parts, double *u, hipStream_t st)
{
    const LevelOrders lo = level_orders(p);
    XcdRanges xr;
    int32_t longest = 0;
    for (int x = 0; x <= kXcds; ++x) xr.begin[x] = p.near_xcd[x];
    for (int x = 0; x < kXcds; ++x) longest = std::max(longest, xr.begin[x + 1] - xr.begin[x]);
    const unsigned blocks = (unsigned)(kXcds * ((longest + 3) / 4));
    const auto *geom = reinterpret_cast<const double4 *>(p.d_leaf_geom);
    const bool mixed = p.precision != BCV_FP64;
    if (p.nearfield == BCV_NEAR_ASSEMBLED && mixed)
        near_eval_kernel<Q, true, true><<<blocks, 256, 0, st>>>(xr, p.d_units, p.d_split, p.d_col, p.d_val,
                                                                p.d_val32, geom, f, lam, p.d_leaf_cell,
                                                                touch_values(p), parts, p.d_partial, u, lo);
    else if (p.nearfield == BCV_NEAR_ASSEMBLED)
        near_eval_kernel<Q, true, false><<<blocks, 256, 0, st>>>(xr, p.d_units, p.d_split, p.d_col, p.d_val,
                                                                 nullptr, geom, f, lam, p.d_leaf_cell,
                                                                 touch_values(p), parts, p.d_partial, u, lo);
    else if (mixed)
        near_eval_kernel<Q, false, true><<<blocks, 256, 0, st>>>(xr, p.d_units, p.d_split, p.d_col, nullptr,
                                                                 nullptr, geom, f, lam, p.d_leaf_cell,
                                                                 touch_values(p), parts, p.d_partial, u, lo);
    else
        near_eval_kernel<Q, false, false><<<blocks, 256, 0, st>>>(xr, p.d_units, p.d_split, p.d_col, nullptr,
                                                                  nullptr, geom, f, lam, p.d_leaf_cell,
                                                                  touch_values(p), parts, p.d_partial, u, lo);
    check_launch();
    if (p.n_splits > 0) {
        near_combine_kernel<Q><<<(unsigned)((p.n_splits + 3) / 4), 256, 0, st>>>(
            p.n_splits, p.d_splits, p.d_partial, geom, (parts & BCV_PART_FAR) ? lam : nullptr, p.d_leaf_cell, u, lo);
        check_launch();
    }
}

// With level-dependent orders the evaluation reads each leaf's own number of coefficients from the
// largest-order tables.
template <int Q>
void launch_near(const bcv_plan_s &p, const double *f, const double *lam, int parts, double *u, hipStream_t st)
{
    if (p.q_schedule)
        launch_near_q<kMaxSchedQ>(p, f, lam, parts, u, st);
    else
        launch_near_q<Q>(p, f, lam, parts, u, st);
}
template <int Q, int A0, int A1, int B0, int B1, class T>
void launch_m2l_block(const bcv_plan_s &p, const XcdRanges &ranges, const T *G, const T *Mr, hipStream_t st, size_t lds = 0)
{
    // four waves per SIMD (128 registers) where the block fits, else two; eight (64 registers) for the
    // smallest blocks up to order 8 (the FP32 order-4 block: 17% faster than at four waves; above
    // order 8 their expansion epilogue spills at 64)
    constexpr int regs = (A1 - A0 + B1 - B0) * (int)(sizeof(T) / 4);
    m2l_shift_kernel<Q, T, A0, A1, B0, B1, (regs > 110 ? 2 : (regs <= 50 && Q <= 8 ? 8 : 4))><<<(unsigned)p.m2l_groups, kWave, lds, st>>>(
        ranges, p.d_tasks, p.d_task_targets, p.d_slot_off, p.d_slot_src, G, Mr, p.d_m2l_partial, p.d_Lam, p.R, p.K);
    check_launch();
}

// Interaction phase over all tasks: lane-shifting launches over blocks of the reduced (a, b)
// triangle, by degree bands (n(d) = (d + 1)^2 reduced multi-indices of degree <= d); the block that
// writes comes first.
template <int Q>
void launch_m2l(const bcv_plan_s &p, const double *G, const double *Mr, hipStream_t st, size_t lds = 0)
{
    constexpr int R = nreduced(Q);
    XcdRanges ranges;
    for (int x = 0; x <= kXcds; ++x) ranges.begin[x] = p.xcd_begin[x];
    if constexpr (Q == 4) {
        launch_m2l_block<Q, 0, R, 0, R>(p, ranges, G, Mr, st, lds);  // everything: 50 doubles
    } else if constexpr (Q == 6) {
        launch_m2l_block<Q, 0, R, 0, R>(p, ranges, G, Mr, st, lds);  // everything: 98 doubles (two waves)
    } else {
        static_assert(Q == 8, "orders 4, 6, 8");
        launch_m2l_block<Q, 0, R, 0, 36>(p, ranges, G, Mr, st, lds);  // all a, |b| <= 5 (two waves)
        launch_m2l_block<Q, 0, 9, 36, R>(p, ranges, G, Mr, st, lds);  // |a| <= 2, |b| >= 6
    }
}

template <int Q>
void launch_m2l(const bcv_plan_s &p, const float *G, const float *Mr, hipStream_t st, size_t lds = 0)
{
    constexpr int R = nreduced(Q);
    XcdRanges ranges;
    for (int x = 0; x <= kXcds; ++x) ranges.begin[x] = p.xcd_begin[x];
    if constexpr (Q <= 6) {
        launch_m2l_block<Q, 0, R, 0, R>(p, ranges, G, Mr, st, lds);  // everything: 2 (Q + 1)^2 floats
    } else {
        static_assert(Q == 8, "orders 4, 6, 8");
        launch_m2l_block<Q, 0, R, 0, 16>(p, ranges, G, Mr, st, lds);  // all a, |b| <= 3
        launch_m2l_block<Q, 0, 25, 16, R>(p, ranges, G, Mr, st, lds);  // |a| <= 4, |b| >= 4
    }
}

// Interaction phase on the matrix cores (BCV_MIXED_SPLIT16): FP16 hi/lo rows from the FP32 folded
// rows (which P2M and M2M wrote), then one launch over all tasks.
void launch_m2l_split16(const bcv_plan_s &p, hipStream_t st)
{
    LevelStarts ls{};
    for (int l = 0; l <= kMaxLevel + 1; ++l) ls.s[l] = p.lvl_start[l];
    ls.L = p.L;
    split_rows_kernel<<<(unsigned)((p.n_cells * 64 + 255) / 256), 256, 0, st>>>(p.n_cells, p.d_M32, p.R, p.d_M16,
                                                                                p.d_fscale, ls);
    check_launch();
    XcdRanges ranges;
    for (int x = 0; x <= kXcds; ++x) ranges.begin[x] = p.xcd_begin[x];
    m2l_mfma_kernel<6><<<(unsigned)p.m2l_groups, kWave, 0, st>>>(
        ranges, p.d_tasks, p.d_task_targets, p.d_slot_off, p.d_slot_src, p.d_slot_mask,
        reinterpret_cast<const u4_t *>(p.d_m2l_A), p.d_G48, reinterpret_cast<const u4_t *>(p.d_M16), p.d_fscale,
        p.d_m2l_partial, p.d_Lam, p.K);
    check_launch();
}

// Upward pass (M2M, l = L-1 .. 2; moments below level 2 are never used), interaction phase (M2L
// with the FP32 copy of the moments in the mixed path) and downward pass (L2L), shared by the VtV
// and BtV applies.
// ---- level-dependent orders: the per-level kernels are chosen at run time --------------------------
template <class F>
void with_order(int q, F &&f)
{
    switch (q) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    default: fail(BCV_ENOTSUP, "expansion order not compiled");
    }
}

// Interaction blocks for any order, generated: bands of source degrees from 0 upward, each with the
// target degrees it reaches (0 .. Q - d0); a band grows while its registers fit the budget (W words
// per value: 1 for float, 2 for double) and its target degrees are cut into bands where even one
// source degree would not fit. Every block's target range is a band of whole degrees; the blocks of
// the first source band write Lambda, the rest add.
struct BlockSpec {
    int a0, a1, b0, b1;
};
template <int Q, int W>
struct BlockPlanTable {
    // FP64 blocks may take nearly all 256 registers (two waves): fewer launches re-read fewer rows,
    // which measured faster than three four-wave blocks at orders 6 and 8; fewer spare registers at
    // high Q
    static constexpr int kBudget = W == 1 ? (Q >= 9 ? 88 : 100) : (Q >= 9 ? 176 : 234);
    BlockSpec b[32];
    int n;
    constexpr BlockPlanTable() : b{}, n(0)
    {
        int d0 = 0;
        while (d0 <= Q) {
            const int na = (Q - d0 + 1) * (Q - d0 + 1);
            int d1 = d0;
            while (d1 + 1 <= Q && (na + (d1 + 2) * (d1 + 2) - d0 * d0) * W <= kBudget) ++d1;
            const int nb = (d1 + 1) * (d1 + 1) - d0 * d0;
            if ((na + nb) * W <= kBudget) {
                b[n++] = BlockSpec{0, na, d0 * d0, (d1 + 1) * (d1 + 1)};
            } else {
                int e0 = 0;
                while (e0 <= Q - d0) {
                    int e1 = e0;
                    while (e1 + 1 <= Q - d0 && ((e1 + 2) * (e1 + 2) - e0 * e0 + nb) * W <= kBudget) ++e1;
                    b[n++] = BlockSpec{e0 * e0, (e1 + 1) * (e1 + 1), d0 * d0, (d1 + 1) * (d1 + 1)};
                    e0 = e1 + 1;
                }
            }
            d0 = d1 + 1;
        }
    }
};
template <int Q, int W>
constexpr BlockPlanTable<Q, W> kBlocks{};

template <int Q, class T, int I>
void launch_level_block(const bcv_plan_s &p, const XcdRanges &ranges, unsigned groups, const T *G, const T *Mr,
                        hipStream_t st)
{
    constexpr int W = (int)(sizeof(T) / 4);
    constexpr BlockSpec bs = kBlocks<Q, W>.b[I];
    constexpr int regs = (bs.a1 - bs.a0 + bs.b1 - bs.b0) * W;
    m2l_shift_kernel<Q, T, bs.a0, bs.a1, bs.b0, bs.b1, (regs > 110 ? 2 : (regs <= 50 && Q <= 8 ? 8 : 4))><<<groups, kWave, 0, st>>>(
        ranges, p.d_tasks, p.d_task_targets, p.d_slot_off, p.d_slot_src, G, Mr, p.d_m2l_partial, p.d_Lam, p.R, p.K);
    check_launch();
}

template <int Q, class T, int... I>
void launch_level_blocks(const bcv_plan_s &p, const XcdRanges &ranges, unsigned groups, const T *G, const T *Mr,
                         hipStream_t st, std::integer_sequence<int, I...>)
{
    (launch_level_block<Q, T, I>(p, ranges, groups, G, Mr, st), ...);
}

// The interaction tasks of one level at that level's order.
template <int Q, class T>
void launch_m2l_level(const bcv_plan_s &p, int lev, const T *G, const T *Mr, hipStream_t st)
{
    XcdRanges ranges;
    int32_t longest = 0;
    for (int x = 0; x <= kXcds; ++x) ranges.begin[x] = p.level_xcd[lev][x];
    for (int x = 0; x < kXcds; ++x) longest = std::max(longest, ranges.begin[x + 1] - ranges.begin[x]);
    if (longest == 0) return;
    launch_level_blocks<Q, T>(p, ranges, (unsigned)(kXcds * longest), G, Mr, st,
                              std::make_integer_sequence<int, kBlocks<Q, (int)(sizeof(T) / 4)>.n>{});
}

// P2M with the folded rows (FP32 in the mixed path).
// fused: the finest level's leaves write only their folded rows, and upward_pass computes their
// parents' moments from f (fixed orders only).
template <int Q>
void launch_p2m(const bcv_plan_s &p, const double *f, hipStream_t st, bool fused = false)
{
    const int skip = fused && !p.q_schedule ? p.L : -1;
    const auto *geom = reinterpret_cast<const double4 *>(p.d_leaf_geom);
    const unsigned blocks = (unsigned)((p.n_leaves + 255) / 256);  // 64 leaves per wave
    LevelOrders lo = level_orders(p);
    if (p.exact_moments)  // every leaf's moments to the largest order (its folded row keeps its own)
        for (int l = 0; l <= kMaxLevel; ++l) lo.k[l] = p.K;
    constexpr int QT = Q > kMaxSchedQ ? Q : kMaxSchedQ;  // tables large enough for every level's order
    if (p.precision != BCV_FP64) {
        if (p.q_schedule)
            p2m_kernel<QT, float><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, geom, f, p.d_M, p.d_M32, lo,
                                                          skip);
        else
            p2m_kernel<Q, float><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, geom, f, p.d_M, p.d_M32, lo,
                                                         skip);
    } else {
        if (p.q_schedule)
            p2m_kernel<QT, double><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, geom, f, p.d_M, p.d_Mr, lo,
                                                           skip);
        else
            p2m_kernel<Q, double><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, geom, f, p.d_M, p.d_Mr, lo,
                                                          skip);
    }
    check_launch();
}

// f_fused: the densities, when launch_p2m skipped the finest level's full moments (fixed orders).
template <int Q>
void upward_pass(const bcv_plan_s &p, hipStream_t st, const double *f_fused = nullptr)
{
    for (int lev = p.L - 1; lev >= 2; --lev) {
        const int n_par = p.parent_begin[lev + 1] - p.parent_begin[lev];
        if (n_par == 0) continue;
        if (f_fused != nullptr && !p.q_schedule && lev == p.L - 1) {  // every child is a level-L leaf
            const auto *geom = reinterpret_cast<const double4 *>(p.d_leaf_geom);
            const unsigned blocks = (unsigned)((n_par + 255) / 256);  // 64 parents per wave
            const int32_t *par = p.d_parents + 2 * p.parent_begin[lev];
            if (p.precision != BCV_FP64)
                m2m_leaves_kernel<Q, float><<<blocks, 256, 0, st>>>(n_par, par, p.d_cell_leaf, geom, f_fused, p.d_M,
                                                                    p.d_M32, p.K, p.R);
            else
                m2m_leaves_kernel<Q, double><<<blocks, 256, 0, st>>>(n_par, par, p.d_cell_leaf, geom, f_fused, p.d_M,
                                                                     p.d_Mr, p.K, p.R);
            check_launch();
            continue;
        }
        auto run = [&](auto qc) {
            constexpr int QP = decltype(qc)::value;  // the parents' order
            const unsigned blocks = (unsigned)((n_par + tree_waves<QP>() - 1) / tree_waves<QP>());
            if (p.precision != BCV_FP64)
                m2m_kernel<QP, float><<<blocks, kWave * tree_waves<QP>(), 0, st>>>(
                    n_par, p.d_parents + 2 * p.parent_begin[lev], p.d_M, p.d_M32, p.K, p.R);
            else
                m2m_kernel<QP, double><<<blocks, kWave * tree_waves<QP>(), 0, st>>>(
                    n_par, p.d_parents + 2 * p.parent_begin[lev], p.d_M, p.d_Mr, p.K, p.R);
            check_launch();
        };
        if (p.exact_moments)  // parents keep every degree of the largest order
            with_order(max_order(p), run);
        else if (p.q_schedule)
            with_order(p.q_level[lev], run);
        else
            run(std::integral_constant<int, Q>{});
    }
}

// matrix_cores: the VtV apply of a BCV_MIXED_SPLIT16 plan (which ran fmax_partial_kernel over f);
// the BtV and VtB applies of such a plan take the FP32 lane-shift kernels.
// lds: bytes of (unused) LDS each lane-shifting interaction block reserves, to cap how many share a CU.
template <int Q>
void interaction_phase(const bcv_plan_s &p, hipStream_t st, bool matrix_cores = false, size_t lds = 0)
{
    if (p.n_tasks == 0) return;
    // the folded moment rows were written with the moments (P2M, boundary P2M, M2M)
    const bool mixed = p.precision != BCV_FP64;
    if (matrix_cores && p.precision == BCV_MIXED_SPLIT16) {
        if constexpr (Q == 6)
            launch_m2l_split16(p, st);
        else
            fail(BCV_ENOTSUP, "BCV_MIXED_SPLIT16 supports q = 6 only");
    } else if (p.q_schedule) {
        for (int lev = p.L; lev >= 2; --lev)
            with_order(p.q_level[lev], [&](auto qc) {
                constexpr int QL = decltype(qc)::value;
                if (mixed)
                    launch_m2l_level<QL, float>(p, lev, p.d_G32, p.d_M32, st);
                else
                    launch_m2l_level<QL, double>(p, lev, p.d_G, p.d_Mr, st);
            });
    } else if (mixed) {
        launch_m2l<Q>(p, p.d_G32, p.d_M32, st, lds);
    } else {
        launch_m2l<Q>(p, p.d_G, p.d_Mr, st, lds);
    }
    if (p.n_m2l_splits > 0) {
        m2l_combine_kernel<<<dim3((unsigned)p.n_m2l_splits, (unsigned)((p.K + 3) / 4)), 256, 0, st>>>(
            p.d_m2l_splits, p.d_tasks, p.d_task_targets, p.d_m2l_partial, p.d_Lam, level_orders(p));
        check_launch();
    }
}

// skip_last: the last level's L2L is left to l2l_eval (fused with the evaluation of the finest leaves).
template <int Q>
void downward_pass(const bcv_plan_s &p, hipStream_t st, bool skip_last = false)
{
    for (int lev = 2; lev < (skip_last ? p.L - 1 : p.L); ++lev) {
        const int n_par = p.parent_begin[lev + 1] - p.parent_begin[lev];
        if (n_par == 0) continue;
        auto run = [&](auto qc) {
            constexpr int QP = decltype(qc)::value;  // the parents' order
            l2l_kernel<QP><<<(unsigned)((n_par + tree_waves<QP>() - 1) / tree_waves<QP>()), kWave * tree_waves<QP>(), 0,
                             st>>>(n_par, p.d_parents + 2 * p.parent_begin[lev], p.d_Lam, p.K,
                                   ncoef(p.q_level[lev + 1]));
            check_launch();
        };
        if (p.q_schedule)
            with_order(p.q_level[lev], run);
        else
            run(std::integral_constant<int, Q>{});
    }
}

// With the near field on the side stream, every interaction block reserves this much LDS (unused),
// so that at most 12 of them (3 waves per SIMD) share a CU and the near field's blocks find wave slots
// beside them instead of waiting for the interaction phase to drain (measured 1.6% to 2.5% faster
// per apply at h = 1/256 than without; 8, 10 and 14 per CU were slower).
constexpr size_t kM2lShareLds = 13 * 1024;

template <int Q>
void apply_q(const bcv_plan_s &p, const double *f, double *u, int parts, hipStream_t st)
{
    constexpr int K = MultiIndex<Q>::K;
    const auto *geom = reinterpret_cast<const double4 *>(p.d_leaf_geom);
    const bool far = (parts & BCV_PART_FAR) && !p.direct;
    const bool near = (parts & BCV_PART_NEAR) != 0;
    const bool fork = far && near && p.streams == 2;
    // fixed orders, and parents on level L - 1 (whose children are all leaves of level L)
    const bool fuse_last = fork && !p.q_schedule && p.L - 1 >= 2 && p.parent_begin[p.L] > p.parent_begin[p.L - 1];
    PhaseMarks marks(p);
    const bool split16 = far && p.precision == BCV_MIXED_SPLIT16;
    if (far) {
        marks.start(BCV_PHASE_P2M, st);
        if (split16) {  // the scale of the FP16 moment rows
            fmax_partial_kernel<<<kFscaleParts, 256, 0, st>>>(p.n_leaves, f, p.d_fscale);
            check_launch();
        }
        launch_p2m<Q>(p, f, st, true);
        marks.stop(BCV_PHASE_P2M, st);
        marks.start(BCV_PHASE_M2M, st);
        upward_pass<Q>(p, st, f);
        marks.stop(BCV_PHASE_M2M, st);
        if (fork) {
            // Near field on the side stream, concurrently with the interaction phase. It is forked
            // after the upward pass: the short, level-by-level moment kernels are on the critical
            // path and would otherwise share the CUs with it.
            BCV_HIP(hipEventRecord(p.ev_fork, st));
            BCV_HIP(hipStreamWaitEvent(p.side, p.ev_fork, 0));
            marks.start(BCV_PHASE_NEAR, p.side);
            launch_near<Q>(p, f, nullptr, BCV_PART_NEAR, u, p.side);
            marks.stop(BCV_PHASE_NEAR, p.side);
            BCV_HIP(hipEventRecord(p.ev_join, p.side));
        }
        marks.start(BCV_PHASE_M2L, st);
        interaction_phase<Q>(p, st, split16, fork ? kM2lShareLds : 0);
        marks.stop(BCV_PHASE_M2L, st);
        marks.start(BCV_PHASE_L2L, st);
        downward_pass<Q>(p, st, fork && fuse_last);
        marks.stop(BCV_PHASE_L2L, st);
    }
    if (fork) {
        BCV_HIP(hipStreamWaitEvent(st, p.ev_join, 0));
        marks.start(BCV_PHASE_EVAL, st);
        if (fuse_last) {  // the last level's L2L fused with the evaluation of its leaf children
            const int lev = p.L - 1;
            const int n_par = p.parent_begin[lev + 1] - p.parent_begin[lev];
            leaf_eval_kernel<Q><<<(unsigned)((n_par + 4 * kLeafEvalPar - 1) / (4 * kLeafEvalPar)), 256, 0, st>>>(
                n_par, p.d_parents + 2 * p.parent_begin[lev], p.d_Lam, p.K, p.d_cell_leaf, geom, u);
            check_launch();
        }
        if (p.q_schedule)
            eval_add_kernel<kMaxSchedQ><<<(unsigned)((p.n_leaves + 3) / 4), 256, 0, st>>>(
                p.n_leaves, geom, p.d_Lam, p.d_leaf_cell, u, level_orders(p));
        else if (fuse_last) {
            if (p.n_rest_leaves > 0)
                eval_list_kernel<Q><<<(unsigned)((p.n_rest_leaves + 31) / 32), 256, 0, st>>>(
                    p.n_rest_leaves, p.d_rest_leaves, geom, p.d_Lam, p.d_leaf_cell, u, level_orders(p));
        } else
            eval_add_kernel<Q><<<(unsigned)((p.n_leaves + 3) / 4), 256, 0, st>>>(p.n_leaves, geom, p.d_Lam,
                                                                              p.d_leaf_cell, u, level_orders(p));
        check_launch();
        marks.stop(BCV_PHASE_EVAL, st);
    } else {
        // near field and evaluation fused (either part may be absent)
        marks.start(BCV_PHASE_NEAR, st);
        launch_near<Q>(p, f, far ? p.d_Lam : nullptr, (near ? BCV_PART_NEAR : 0) | (far ? BCV_PART_FAR : 0), u, st);
        marks.stop(BCV_PHASE_NEAR, st);
    }
    if (p.d_uscale != nullptr) {  // domains of side s != 1: u = s^5 u(unit cube)
        scale_kernel<<<(unsigned)((p.n_leaves + 255) / 256), 256, 0, st>>>(p.n_leaves, p.d_uscale, u);
        check_launch();
    }
    marks.finish(st);
}

// VtV apply with degree-p leaf bases (opts.basis_degree = 1), on the caller's stream: the leaf moments
// from all basis coefficients with each leaf's rule, the unchanged passes and interaction phase, the
// near field from the plan's blocks, then the evaluation of every coefficient.
template <int Q>
void basis_apply_q(const bcv_plan_s &p, const double *f, double *u, int parts, hipStream_t st)
{
    const bool far = (parts & BCV_PART_FAR) && !p.direct;
    const bool near = (parts & BCV_PART_NEAR) != 0;
    PhaseMarks marks(p);
    if (far) {
        marks.start(BCV_PHASE_P2M, st);
        launch_basis_p2m(p, f, st);
        marks.stop(BCV_PHASE_P2M, st);
        marks.start(BCV_PHASE_M2M, st);
        upward_pass<Q>(p, st, f);  // fixed orders: level L - 1 from the degree-0 coefficients of its children
        marks.stop(BCV_PHASE_M2M, st);
        marks.start(BCV_PHASE_M2L, st);
        interaction_phase<Q>(p, st);
        marks.stop(BCV_PHASE_M2L, st);
        marks.start(BCV_PHASE_L2L, st);
        downward_pass<Q>(p, st);
        marks.stop(BCV_PHASE_L2L, st);
    }
    marks.start(BCV_PHASE_NEAR, st);
    if (near)
        launch_basis_near(p, f, u, st);
    else
        launch_basis_zero(p, u, st);
    marks.stop(BCV_PHASE_NEAR, st);
    if (far) {
        marks.start(BCV_PHASE_EVAL, st);
        launch_basis_eval(p, u, st);
        marks.stop(BCV_PHASE_EVAL, st);
    }
    marks.finish(st);
}

// The plan with one of its other interaction plans (BtV, VtB) in place of the VtV one (a shallow
// copy: the device buffers stay the plan's).
bcv_plan_s with_m2l(const bcv_plan_s &p, const M2LSet &ms)
{
    bcv_plan_s q = p;
    q.n_tasks = ms.n_tasks;
    q.d_tasks = ms.d_tasks;
    q.d_task_targets = ms.d_task_targets;
    q.d_slot_off = ms.d_slot_off;
    q.d_slot_src = ms.d_slot_src;
    q.n_m2l_splits = ms.n_m2l_splits;
    q.d_m2l_splits = ms.d_m2l_splits;
    q.d_m2l_partial = ms.d_m2l_partial;
    q.m2l_groups = ms.m2l_groups;
    for (int x = 0; x <= kXcds; ++x) q.xcd_begin[x] = ms.xcd_begin[x];
    return q;
}

// BtV apply (Algorithm 3), on the caller's stream: boundary moments, upward pass, interaction
// phase over the boundary sources I(w) ∩ B_l (the plan's BtV interaction plan), downward pass, then
// the near field of the boundary faces fused with the evaluation phase.
template <int Q>
void btv_q(const bcv_plan_s &p, const double *qf, const double *gf, double *u, hipStream_t st)
{
    constexpr int K = MultiIndex<Q>::K;
    const auto *geom = reinterpret_cast<const double4 *>(p.d_leaf_geom);
    const bool far = !p.direct;
    if (far) {
        const unsigned blocks = (unsigned)((p.n_leaves + 3) / 4);
        if (p.precision != BCV_FP64)
            btv_p2m_kernel<Q, float><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, geom, p.d_leaf_faces,
                                                             p.d_faces, qf, gf, p.d_M, p.d_M32);
        else
            btv_p2m_kernel<Q, double><<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, geom, p.d_leaf_faces,
                                                              p.d_faces, qf, gf, p.d_M, p.d_Mr);
        check_launch();
        upward_pass<Q>(p, st);
        interaction_phase<Q>(with_m2l(p, p.btv_m2l), st);
        downward_pass<Q>(p, st);
    }
    const double *lam = far ? p.d_Lam : nullptr;
    const unsigned blocks = (unsigned)((p.n_btv_units + 3) / 4);
    if (p.precision != BCV_FP64)
        btv_near_kernel<Q, true><<<blocks, 256, 0, st>>>(p.n_btv_units, p.d_btv_units, p.d_btv_col, p.d_faces, geom, qf,
                                                         gf, p.d_btv_touch, lam, p.d_leaf_cell, p.d_btv_partial, u);
    else
        btv_near_kernel<Q, false><<<blocks, 256, 0, st>>>(p.n_btv_units, p.d_btv_units, p.d_btv_col, p.d_faces, geom,
                                                          qf, gf, p.d_btv_touch, lam, p.d_leaf_cell, p.d_btv_partial,
                                                          u);
    check_launch();
    if (p.n_btv_splits > 0) {
        near_combine_kernel<Q><<<(unsigned)((p.n_btv_splits + 3) / 4), 256, 0, st>>>(
            p.n_btv_splits, p.d_btv_splits, p.d_btv_partial, geom, lam, p.d_leaf_cell, u, level_orders(p));
        check_launch();
    }
}

// VtB apply (Algorithm 2), on the caller's stream: moments of every leaf, upward pass, interaction
// phase for the boundary cells only (the plan's VtB interaction plan), downward pass (the boundary
// cells' coefficients, whose ancestors are boundary cells, are the ones used; the other cells'
// coefficients are not written by this apply's interaction phase and are never read), then the near
// field of the faces fused with the evaluation at the faces.
template <int Q>
void vtb_q(const bcv_plan_s &p, const double *f, double *uf, hipStream_t st)
{
    constexpr int K = MultiIndex<Q>::K;
    const auto *geom = reinterpret_cast<const double4 *>(p.d_leaf_geom);
    const bool far = !p.direct;
    if (far) {
        launch_p2m<Q>(p, f, st, true);
        upward_pass<Q>(p, st, f);
        interaction_phase<Q>(with_m2l(p, p.vtb_m2l), st);
        downward_pass<Q>(p, st);
    }
    const double *lam = far ? p.d_Lam : nullptr;
    const unsigned blocks = (unsigned)((p.n_vtb_units + 3) / 4);
    if (p.precision != BCV_FP64)
        vtb_near_kernel<Q, true><<<blocks, 256, 0, st>>>(p.n_vtb_units, p.d_vtb_units, p.d_vtb_col, p.d_faces, geom, f,
                                                         p.d_btv_touch, lam, p.d_leaf_cell, p.d_vtb_partial, uf);
    else
        vtb_near_kernel<Q, false><<<blocks, 256, 0, st>>>(p.n_vtb_units, p.d_vtb_units, p.d_vtb_col, p.d_faces, geom, f,
                                                          p.d_btv_touch, lam, p.d_leaf_cell, p.d_vtb_partial, uf);
    check_launch();
    if (p.n_vtb_splits > 0) {
        vtb_combine_kernel<Q><<<(unsigned)((p.n_vtb_splits + 3) / 4), 256, 0, st>>>(
            p.n_vtb_splits, p.d_vtb_splits, p.d_vtb_partial, p.d_faces, geom, lam, p.d_leaf_cell, uf);
        check_launch();
    }
}

}  // namespace

void launch_vtb(const bcv_plan_s &p, const double *f, double *uf, hipStream_t st)
{
    switch (p.q) {
    case 4: vtb_q<4>(p, f, uf, st); break;
    case 6: vtb_q<6>(p, f, uf, st); break;
    case 8: vtb_q<8>(p, f, uf, st); break;
    default: fail(BCV_ENOTSUP, "expansion order not compiled");
    }
}

void launch_btv(const bcv_plan_s &p, const double *qf, const double *gf, double *u, hipStream_t st)
{
    switch (p.q) {
    case 4: btv_q<4>(p, qf, gf, u, st); break;
    case 6: btv_q<6>(p, qf, gf, u, st); break;
    case 8: btv_q<8>(p, qf, gf, u, st); break;
    default: fail(BCV_ENOTSUP, "expansion order not compiled");
    }
}

// VtV apply on a mapped mesh (mapped.hip), on the caller's stream: the near field from the assembled
// entries (it writes u), then P2M, the upward pass, the interaction phase (lattice tasks for the cells
// of cube meshes, pair by pair for the ball cells), the downward pass and the evaluation, which adds
// to u.
template <int Q>
void mapped_apply_q(const bcv_plan_s &p, const double *f, double *u, int parts, hipStream_t st)
{
    const bool far = (parts & BCV_PART_FAR) && !p.direct;
    const bool near = (parts & BCV_PART_NEAR) != 0;
    PhaseMarks marks(p);
    // With a second stream: after P2M (bandwidth-bound) the near field runs there beside M2M
    // (latency-bound, level by level), and then the ball cells' pair kernel beside the cube cells'
    // lattice tasks (disjoint targets), so that each fills the other's tail; the main stream waits
    // for both before L2L.
    const bool two = far && p.streams == 2 && p.side != nullptr;
    auto near_part = [&](hipStream_t ns) {
        marks.start(BCV_PHASE_NEAR, ns);
        if (near)
            launch_near<Q>(p, f, nullptr, BCV_PART_NEAR, u, ns);
        else
            launch_mapped_zero(p, u, ns);
        marks.stop(BCV_PHASE_NEAR, ns);
    };
    if (!two) near_part(st);
    if (far) {
        const int phase_id[4] = {BCV_PHASE_P2M, BCV_PHASE_M2M, BCV_PHASE_M2L, BCV_PHASE_L2L};
        for (int ph = 0; ph < 4; ++ph) {
            if (ph == 1 && two) {
                BCV_HIP(hipEventRecord(p.ev_fork, st));
                BCV_HIP(hipStreamWaitEvent(p.side, p.ev_fork, 0));
                near_part(p.side);
            }
            marks.start(phase_id[ph], st);
            if (ph == 2 && two) {
                BCV_HIP(hipEventRecord(p.ev_fork2, st));
                BCV_HIP(hipStreamWaitEvent(p.side, p.ev_fork2, 0));
                launch_mapped_phase(p, f, ph, p.side);
                BCV_HIP(hipEventRecord(p.ev_join, p.side));
                interaction_phase<Q>(p, st);
                BCV_HIP(hipStreamWaitEvent(st, p.ev_join, 0));
            } else {
                if (ph == 2) interaction_phase<Q>(p, st);  // the cube meshes' cells: lattice tasks
                launch_mapped_phase(p, f, ph, st);
            }
            marks.stop(phase_id[ph], st);
        }
        marks.start(BCV_PHASE_EVAL, st);
        launch_mapped_eval(p, u, st);
        marks.stop(BCV_PHASE_EVAL, st);
    }
    if (p.d_uscale != nullptr) {  // domains of side s != 1: u = s^5 u(unit side)
        scale_kernel<<<(unsigned)((p.n_leaves + 255) / 256), 256, 0, st>>>(p.n_leaves, p.d_uscale, u);
        check_launch();
    }
    marks.finish(st);
}

void launch_apply(const bcv_plan_s &p, const double *f, double *u, int parts, hipStream_t st)
{
    if (p.mapped) {
        switch (p.q) {
        case 4: mapped_apply_q<4>(p, f, u, parts, st); break;
        case 6: mapped_apply_q<6>(p, f, u, parts, st); break;
        case 8: mapped_apply_q<8>(p, f, u, parts, st); break;
        default: fail(BCV_ENOTSUP, "expansion order not compiled");
        }
        return;
    }
    if (p.basis) {
        if (p.q_schedule) {  // the passes pick their kernels level by level
            basis_apply_q<4>(p, f, u, parts, st);
            return;
        }
        switch (p.q) {
        case 4: basis_apply_q<4>(p, f, u, parts, st); break;
        case 6: basis_apply_q<6>(p, f, u, parts, st); break;
        case 8: basis_apply_q<8>(p, f, u, parts, st); break;
        default: fail(BCV_ENOTSUP, "expansion order not compiled");
        }
        return;
    }
    if (p.q_schedule) {  // every phase picks its kernels by the level's order (the template order is unused)
        apply_q<4>(p, f, u, parts, st);
        return;
    }
    switch (p.q) {
    case 4: apply_q<4>(p, f, u, parts, st); break;
    case 6: apply_q<6>(p, f, u, parts, st); break;
    case 8: apply_q<8>(p, f, u, parts, st); break;
    default: fail(BCV_ENOTSUP, "expansion order not compiled");
    }
}

void launch_near_assemble(const bcv_plan_s &p, hipStream_t st)
{
    const unsigned blocks = (unsigned)((p.n_units + 3) / 4);
    near_assemble_kernel<<<blocks, 256, 0, st>>>(p.n_units, p.d_units, p.d_col,
                                                 reinterpret_cast<const double4 *>(p.d_leaf_geom), touch_values(p),
                                                 p.d_val);
    check_launch();
}

void launch_near_narrow(const bcv_plan_s &p, hipStream_t st)
{
    const unsigned blocks = (unsigned)std::min<int64_t>((p.n_near + 255) / 256, 65536);
    if (p.n_near > 0) narrow_kernel<<<blocks, 256, 0, st>>>(p.n_near, p.d_val, p.d_val32);
    check_launch();
}

void gauss_legendre01(int n, double *x, double *w);

namespace {
// A device buffer freed on scope exit (plan-time temporaries).
template <class T>
struct TempBuffer {
    T *d = nullptr;
    explicit TempBuffer(const std::vector<T> &v)
    {
        if (v.empty()) return;
        if (hipMalloc(&d, v.size() * sizeof(T)) != hipSuccess) fail(BCV_ENOMEM, "hipMalloc failed (plan temporary)");
        const hipError_t e = hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            d = nullptr;
            BCV_HIP(e);
        }
    }
    ~TempBuffer() { (void)hipFree(d); }
    TempBuffer(const TempBuffer &) = delete;
    TempBuffer &operator=(const TempBuffer &) = delete;
};
}  // namespace

void launch_near_assemble_ordered(const bcv_plan_s &p, const std::vector<int64_t> &entry,
                                  const std::vector<int32_t> &target, const std::vector<int8_t> &order)
{
    BCV_REQUIRE(entry.size() == target.size() && (int64_t)order.size() == p.n_leaves, BCV_ESTATE,
                "internal: ordered near entries");
    if (entry.empty()) return;
    for (int8_t o : order) BCV_REQUIRE(o >= 1 && o <= kMaxGauss, BCV_ESTATE, "internal: Gauss order out of range");
    std::vector<double> gx(16 * (kMaxGauss + 1), 0.0), gw(16 * (kMaxGauss + 1), 0.0);
    for (int n = 1; n <= kMaxGauss; ++n) gauss_legendre01(n, &gx[16 * n], &gw[16 * n]);
    const TempBuffer<int64_t> d_entry(entry);
    const TempBuffer<int32_t> d_target(target);
    const TempBuffer<int8_t> d_order(order);
    const TempBuffer<double> d_gx(gx), d_gw(gw);
    const int64_t n = (int64_t)entry.size();
    near_assemble_ordered_kernel<<<(unsigned)((n + 3) / 4), 256, 0, nullptr>>>(
        n, d_entry.d, d_target.d, p.d_col, reinterpret_cast<const double4 *>(p.d_leaf_geom), d_order.d, d_gx.d,
        d_gw.d, p.d_val);
    check_launch();
    BCV_HIP(hipDeviceSynchronize());  // before the temporaries are freed
}

void split16_tables(int K, const std::vector<double> &G, int n_off, std::vector<uint16_t> &A, std::vector<float> &G48)
{
    constexpr int Q = 6, R = nreduced(Q);
    constexpr ReducedIndex<Q> ri{};
    if (K < ncoef(Q) || (int64_t)G.size() < (int64_t)n_off * K) fail(BCV_ESTATE, "internal: derivative tables too small");
    A.assign((size_t)n_off * kSplitTiles * 2 * kWave * 8, 0);
    G48.assign((size_t)std::max(n_off, 1), 0.0f);
    const double four_pi = 4.0 * M_PI;
    for (int o = 0; o < n_off; ++o) {
        const double *Go = &G[(size_t)o * K];
        for (int tl = 0; tl < kSplitTiles; ++tl)
            for (int lane = 0; lane < kWave; ++lane)
                for (int jj = 0; jj < 8; ++jj) {
                    const int a = 16 * kTileBlock[tl] + (lane & 15);
                    const int b = 32 * kTileChunk[tl] + 8 * (lane >> 4) + jj;
                    const double v = (a < R && b < R && ri.deg[a] + ri.deg[b] <= Q) ? four_pi * Go[ri.sum(a, b)] : 0.0;
                    if (v != 0.0 && (lane >> 4) >= kTileGroups[tl])
                        fail(BCV_ESTATE, "internal: a nonzero interaction entry outside the loaded k-groups");
                    const _Float16 hi = (_Float16)v;
                    const _Float16 lo = (_Float16)(v - (double)hi);
                    const size_t at = (((size_t)o * kSplitTiles + tl) * 2) * kWave * 8 + (size_t)lane * 8 + jj;
                    A[at] = __builtin_bit_cast(uint16_t, hi);
                    A[at + (size_t)kWave * 8] = __builtin_bit_cast(uint16_t, lo);
                }
        G48[o] = (float)(four_pi * Go[ri.sum(R - 1, 0)]);
    }
}

void regular_cube_pairs(const int *deltas, int n, int n_gauss, double *out)
{
    BCV_REQUIRE(n_gauss >= 1 && n_gauss <= kMaxGauss, BCV_EINVAL, "bad Gauss order");
    GaussRule rule{};
    gauss_legendre01(n_gauss, rule.x, rule.w);
    int *d_deltas = nullptr;
    double *d_out = nullptr;
    BCV_HIP(hipMalloc(&d_deltas, sizeof(int) * 3 * n));
    BCV_HIP(hipMalloc(&d_out, sizeof(double) * n));
    BCV_HIP(hipMemcpy(d_deltas, deltas, sizeof(int) * 3 * n, hipMemcpyHostToDevice));
    regular_cube_pairs_kernel<<<n, 256>>>(d_deltas, n_gauss, rule, d_out);
    const hipError_t e = hipGetLastError();
    hipError_t e2 = hipMemcpy(out, d_out, sizeof(double) * n, hipMemcpyDeviceToHost);
    (void)hipFree(d_deltas);
    (void)hipFree(d_out);
    BCV_HIP(e);
    BCV_HIP(e2);
}

}  // namespace bcv
