// Degree-p leaf bases for the VtV apply (Sec. 1.2: the finite element space with polynomials of
// degree p_w on each leaf; Sec. 4, approximation errors: p_l = L - l on the leaves of level l).
//
// Leaf w (level l, side a, centre c) carries phi^alpha_w(x) = prod_i P_{alpha_i}(2 (x_i - c_i)/a),
// |alpha| <= p_w = L - l (Legendre, orthogonal on w, phi^0 the indicator) and the tensor
// Gauss-Legendre rule of n_w = p_w + 2 points per axis. With xi = (x - c)/a in [-1/2, 1/2]^3:
//   near entries  A[(t,alpha),(s,beta)] = the exact touching block (singular_basis.cpp) times
//                 a_small^5 / (4 pi), or sum_g sum_h W_g W_h phi^alpha(x_g) phi^beta(y_h) / (4 pi |x_g - y_h|);
//   moments       M^b = a^3 sum_alpha f_alpha prod_i t_p[b_i][alpha_i],
//                 t_p[b][k] = (-1)^b / b! sum_g w_g xi_g^b P_k(2 xi_g)
//                 (the library's scaled moments M^b = (-1)^|b| m^b / (b! a^|b|), m^b = int (y - c)^b f);
//   evaluation    u_alpha += a^3 sum_b Lambda^b prod_i e_p[alpha_i][b_i],
//                 e_p[k][b] = sum_g w_g P_k(2 xi_g) xi_g^b / b!
// (w_g the per-axis weights, summing to 1). Degree 0 reduces to the indicator basis: t_0 = e_0 = kappa.
//
// Coefficient layout (f and u): entries 0 .. n_leaves - 1 are the alpha = 0 coefficients in leaf
// order, then every leaf's higher coefficients alpha = 1 .. ncoef(p_w) - 1 follow, leaf by leaf.
// The near field is stored as blocks at plan time: the near row of target t has row_len(t) =
// sum over its sources of ncoef(p_s) columns (source coefficients), shared by its ncoef(p_t) rows.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.hpp"
#include "multiindex.hpp"

namespace bcv {

void gauss_legendre01(int n, double *x, double *w);

namespace {

constexpr int kWave = 64;
constexpr double kInv4Pi = 0.079577471545947667884;
constexpr int kMaxRule = kMaxBasisDegree + 2;  // Gauss points per axis
constexpr int kBlockChunk = 8;                 // source functions per register pass of the block kernel

__device__ __forceinline__ int level_of(double a)
{
    return 1023 - (int)((__double_as_longlong(a) >> 52) & 0x7FF);
}

// position of the coefficient alpha of leaf w (alpha given by its graded position r)
__device__ __forceinline__ int64_t dof_of(int64_t w, int r, int64_t n_leaves, const int64_t *hi_off)
{
    return r == 0 ? w : n_leaves + hi_off[w] + (r - 1);
}

template <int Q>
__constant__ constexpr MultiIndex<Q> kMi{};
template <int Q>
__constant__ constexpr FoldTable<Q> kFoldB{};
__constant__ constexpr MultiIndex<kMaxBasisDegree> kMiB{};

// One wave per near pair: the block of (target t, source s) into its place in t's block row.
__global__ __launch_bounds__(256) void basis_block_kernel(int64_t n_pairs, const int32_t *__restrict__ pair_t,
                                                          const int32_t *__restrict__ pair_pos,
                                                          const uint32_t *__restrict__ col,
                                                          const double4 *__restrict__ geom, int L,
                                                          const int64_t *__restrict__ bcb,
                                                          const int64_t *__restrict__ bvb,
                                                          const BasisTables *__restrict__ tab,
                                                          const double *__restrict__ touch_equal,
                                                          const double *__restrict__ touch_sb, int nbP,
                                                          double *__restrict__ bval)
{
    __shared__ double vls[4][kWave][kBlockChunk];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t e = (int64_t)blockIdx.x * 4 + wv;
    if (e >= n_pairs) return;
    const int32_t t = pair_t[e];
    const uint32_t cw = col[e];
    const int32_t s = (int32_t)(cw & 0x0FFFFFFFu);
    const bool touching = (cw >> 28) != 0;
    const double4 gt = geom[t], gs = geom[s];
    const int pt = L - level_of(gt.w), ps = L - level_of(gs.w);
    const int nt = ncoef(pt), ns = ncoef(ps);
    const int64_t rl = bcb[t + 1] - bcb[t];
    double *out = bval + bvb[t] + pair_pos[e];  // entry (alpha, beta) at out[alpha rl + beta]
    if (touching) {
        const double as = fmin(gt.w, gs.w);
        const double sc = as * as * as * as * as * kInv4Pi;
        int o[3];
        o[0] = (int)rint((gs.x - gt.x) / as);
        o[1] = (int)rint((gs.y - gt.y) / as);
        o[2] = (int)rint((gs.z - gt.z) / as);
        const double *blk;
        bool transpose = false;
        if (gt.w == gs.w) {
            blk = touch_equal + (int64_t)((o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)) * nbP * nbP;
        } else if (gt.w < gs.w) {  // target is the unit cube, source the side-2 cube at b = o
            blk = touch_sb + (int64_t)((o[0] + 2) + 4 * (o[1] + 2) + 16 * (o[2] + 2)) * nbP * nbP;
        } else {  // target side 2, source unit cube at o: b = -o, transposed
            blk = touch_sb + (int64_t)((2 - o[0]) + 4 * (2 - o[1]) + 16 * (2 - o[2])) * nbP * nbP;
            transpose = true;
        }
        for (int k = lane; k < nt * ns; k += kWave) {
            const int a = k / ns, b = k - a * ns;
            out[(int64_t)a * rl + b] = sc * (transpose ? blk[b * nbP + a] : blk[a * nbP + b]);
        }
        return;
    }
    // Outer side A: the one with more functions (its points go over the lanes); inner side B.
    const bool swap = ns > nt;
    const double4 ga = swap ? gs : gt, gb = swap ? gt : gs;
    const int pa = swap ? ps : pt, pb = swap ? pt : ps;
    const int na = pa + 2, nb = pb + 2;
    const int nfa = swap ? ns : nt, nfb = swap ? nt : ns;
    const int PA = na * na * na, PB = nb * nb * nb;
    const double wa3 = ga.w * ga.w * ga.w, wb3 = gb.w * gb.w * gb.w;
    for (int g0 = 0; g0 < PA; g0 += kWave) {
        const int g = g0 + lane;
        const bool act = g < PA;
        const int gx = g % na, gy = (g / na) % na, gz = g / (na * na);
        const double x0 = ga.x + ga.w * tab->x[na][act ? gx : 0];
        const double x1 = ga.y + ga.w * tab->x[na][act ? gy : 0];
        const double x2 = ga.z + ga.w * tab->x[na][act ? gz : 0];
        for (int b0 = 0; b0 < nfb; b0 += kBlockChunk) {
            const int nc = min(kBlockChunk, nfb - b0);
            double v[kBlockChunk];
#pragma unroll
            for (int c = 0; c < kBlockChunk; ++c) v[c] = 0.0;
            if (act)
                for (int h = 0; h < PB; ++h) {
                    const int hx = h % nb, hy = (h / nb) % nb, hz = h / (nb * nb);
                    const double d0 = x0 - (gb.x + gb.w * tab->x[nb][hx]);
                    const double d1 = x1 - (gb.y + gb.w * tab->x[nb][hy]);
                    const double d2 = x2 - (gb.z + gb.w * tab->x[nb][hz]);
                    const double k =
                        wb3 * tab->w[nb][hx] * tab->w[nb][hy] * tab->w[nb][hz] / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
#pragma unroll
                    for (int c = 0; c < kBlockChunk; ++c)
                        if (c < nc) {
                            const int bi = b0 + c;
                            v[c] = fma(k,
                                       tab->leg[nb][kMiB.e[bi][0]][hx] * tab->leg[nb][kMiB.e[bi][1]][hy] *
                                           tab->leg[nb][kMiB.e[bi][2]][hz],
                                       v[c]);
                        }
                }
#pragma unroll
            for (int c = 0; c < kBlockChunk; ++c) vls[wv][lane][c] = v[c];
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            for (int k = lane; k < nfa * nc; k += kWave) {
                const int a = k / nc, c = k - a * nc;
                double acc = 0.0;
                const int gend = min(kWave, PA - g0);
                for (int gg = 0; gg < gend; ++gg) {
                    const int G = g0 + gg;
                    const int qx = G % na, qy = (G / na) % na, qz = G / (na * na);
                    const double wphi = wa3 * tab->w[na][qx] * tab->w[na][qy] * tab->w[na][qz] *
                                        tab->leg[na][kMiB.e[a][0]][qx] * tab->leg[na][kMiB.e[a][1]][qy] *
                                        tab->leg[na][kMiB.e[a][2]][qz];
                    acc = fma(wphi, vls[wv][gg][c], acc);
                }
                acc *= kInv4Pi;
                const int bi = b0 + c;
                double *dst = swap ? out + (int64_t)bi * rl + a : out + (int64_t)a * rl + bi;
                *dst = g0 == 0 ? acc : *dst + acc;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Near field: one wave per work unit (kBasisRows rows of a target over a column range): the block
// entries times the source coefficients, summed over the unit's columns; writes u (whole rows) or the
// unit's partial sums.
__global__ __launch_bounds__(256) void basis_near_kernel(int64_t n_work, const BasisUnit *__restrict__ work,
                                                         const int64_t *__restrict__ bcb,
                                                         const int64_t *__restrict__ bvb,
                                                         const int32_t *__restrict__ bcol,
                                                         const double *__restrict__ bval,
                                                         const double4 *__restrict__ geom, int L, int64_t n_leaves,
                                                         const int64_t *__restrict__ hi_off,
                                                         const double *__restrict__ f, double *__restrict__ partial,
                                                         double *__restrict__ u)
{
    const int64_t wi = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    if (wi >= n_work) return;
    const BasisUnit wk = work[wi];
    const int nt = ncoef(L - level_of(geom[wk.t].w));
    const int nr = min(kBasisRows, nt - wk.a0);
    const int64_t cb = bcb[wk.t] + wk.j0, rl = bcb[wk.t + 1] - bcb[wk.t];
    const double *v = bval + bvb[wk.t] + (int64_t)wk.a0 * rl + wk.j0;
    double acc[kBasisRows];
#pragma unroll
    for (int c = 0; c < kBasisRows; ++c) acc[c] = 0.0;
    for (int j = lane; j < wk.len; j += kWave) {
        const double fj = f[bcol[cb + j]];
#pragma unroll
        for (int c = 0; c < kBasisRows; ++c)
            if (c < nr) acc[c] = fma(v[(int64_t)c * rl + j], fj, acc[c]);
    }
#pragma unroll
    for (int c = 0; c < kBasisRows; ++c) {
        double x = acc[c];
        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
        acc[c] = x;
    }
    if (lane < nr) {
        double x = 0.0;
#pragma unroll
        for (int c = 0; c < kBasisRows; ++c)
            if (c == lane) x = acc[c];
        if (wk.out < 0)
            u[dof_of(wk.t, wk.a0 + lane, n_leaves, hi_off)] = x;
        else
            partial[wk.out + lane] = x;
    }
}

// Rows cut into several units: their partial sums added in column order (one thread per row).
__global__ void basis_combine_kernel(int64_t n_splits, const BasisSplit *__restrict__ splits,
                                     const double *__restrict__ partial, const double4 *__restrict__ geom, int L,
                                     int64_t n_leaves, const int64_t *__restrict__ hi_off, double *__restrict__ u)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_splits * kBasisRows) return;
    const BasisSplit sp = splits[i / kBasisRows];
    const int c = (int)(i % kBasisRows);
    const int nt = ncoef(L - level_of(geom[sp.t].w));
    if (sp.a0 + c >= nt) return;
    double x = 0.0;
    for (int k = 0; k < sp.count; ++k) x += partial[sp.first + k * kBasisRows + c];
    u[dof_of(sp.t, sp.a0 + c, n_leaves, hi_off)] = x;
}

// Moments of every leaf (one thread per (leaf, j < ldr)): the full coefficients j, j + ldr, ... < ncoef(q_l)
// (not for the degree-0 leaves of level L when skip_finest, whose parents take their moments from
// the densities, see m2m_leaves_kernel) and the folded coefficient j < (q_l + 1)^2. The multi-index
// and fold tables of order 10 serve every order: both orders are graded, so those of order q are
// their prefixes.
__global__ __launch_bounds__(256) void basis_p2m_kernel(int64_t n_leaves, const int32_t *__restrict__ leaf_cell,
                                                        const double4 *__restrict__ geom, int L,
                                                        const int64_t *__restrict__ hi_off,
                                                        const BasisTables *__restrict__ tab, const BasisOrders bo,
                                                        int skip_finest, const double *__restrict__ f,
                                                        double *__restrict__ M, double *__restrict__ Mr)
{
    constexpr int QT = kMaxBasisQ;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = idx / bo.ldr;
    const int j = (int)(idx - w * bo.ldr);
    if (w >= n_leaves) return;
    const double a = geom[w].w;
    const int lev = level_of(a);
    const int p = L - lev;
    const int nf = ncoef(p);
    const double a3 = a * a * a;
    auto moment = [&](int b) {
        double s = 0.0;
        for (int r = 0; r < nf; ++r)
            s = fma(tab->t[p][kMi<QT>.e[b][0]][kMiB.e[r][0]] * tab->t[p][kMi<QT>.e[b][1]][kMiB.e[r][1]] *
                        tab->t[p][kMi<QT>.e[b][2]][kMiB.e[r][2]],
                    f[dof_of(w, r, n_leaves, hi_off)], s);
        return s * a3;
    };
    const int64_t c = leaf_cell[w];
    if (p > 0 || !skip_finest)
        for (int b = j; b < bo.k[lev]; b += bo.ldr) M[c * bo.ldk + b] = moment(b);
    if (j < bo.r[lev]) {
        double s = 0.0;
        for (int k = 0; k < kFoldB<QT>.n[j]; ++k) s = fma(kFoldB<QT>.c[j][k], moment(kFoldB<QT>.src[j][k]), s);
        Mr[c * bo.ldr + j] = s;
    }
}

// Evaluation of every coefficient (one thread each): u[(w, alpha)] += a^3 sum_{b < ncoef(q_l)} e(alpha, b) Lambda_w^b.
__global__ __launch_bounds__(256) void basis_eval_kernel(int64_t n_dofs, int64_t n_leaves,
                                                         const int32_t *__restrict__ leaf_cell,
                                                         const double4 *__restrict__ geom, int L,
                                                         const int64_t *__restrict__ hi_off,
                                                         const int32_t *__restrict__ dof_leaf,
                                                         const BasisTables *__restrict__ tab, const BasisOrders bo,
                                                         const double *__restrict__ Lam, double *__restrict__ u)
{
    constexpr int QT = kMaxBasisQ;
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n_dofs) return;
    const int64_t w = d < n_leaves ? d : dof_leaf[d - n_leaves];
    const int r = d < n_leaves ? 0 : (int)(d - n_leaves - hi_off[w]) + 1;
    const double a = geom[w].w;
    const int lev = level_of(a);
    const int p = L - lev;
    const double *lam = Lam + (int64_t)leaf_cell[w] * bo.ldk;
    const int r0 = kMiB.e[r][0], r1 = kMiB.e[r][1], r2 = kMiB.e[r][2];
    double s = 0.0;
    for (int b = 0; b < bo.k[lev]; ++b)
        s = fma(tab->e[p][r0][kMi<QT>.e[b][0]] * tab->e[p][r1][kMi<QT>.e[b][1]] * tab->e[p][r2][kMi<QT>.e[b][2]],
                lam[b], s);
    u[d] += s * a * a * a;
}

__global__ void fill_zero_kernel(int64_t n, double *__restrict__ u)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        u[i] = 0.0;
}

void check()
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(BCV_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
}

}  // namespace

BasisTables basis_tables()
{
    BasisTables tb{};
    for (int n = 1; n <= kMaxRule; ++n) {
        double x[kMaxRule], w[kMaxRule];
        gauss_legendre01(n, x, w);
        for (int k = 0; k < n; ++k) {
            tb.x[n][k] = x[k];
            tb.w[n][k] = w[k];
            double p0 = 1.0, p1 = 2.0 * x[k] - 1.0;  // P_a(2 x - 1), three-term recurrence
            const double tt = p1;
            tb.leg[n][0][k] = 1.0;
            if (kMaxBasisDegree >= 1) tb.leg[n][1][k] = p1;
            for (int a = 1; a < kMaxBasisDegree; ++a) {
                const double p2 = ((2 * a + 1) * tt * p1 - a * p0) / (a + 1);
                p0 = p1;
                p1 = p2;
                tb.leg[n][a + 1][k] = p2;
            }
        }
    }
    for (int p = 0; p <= kMaxBasisDegree; ++p) {
        const int n = p + 2;
        for (int b = 0; b <= kMaxBasisQ; ++b) {
            double fact = 1.0;
            for (int i = 2; i <= b; ++i) fact *= i;
            for (int k = 0; k <= kMaxBasisDegree; ++k) {
                double s = 0.0;
                for (int g = 0; g < n; ++g) s += tb.w[n][g] * std::pow(tb.x[n][g] - 0.5, b) * tb.leg[n][k][g];
                tb.t[p][b][k] = ((b & 1) ? -s : s) / fact;
                tb.e[p][k][b] = s / fact;
            }
        }
    }
    return tb;
}

void launch_basis_assemble(const bcv_plan_s &p, const std::vector<int32_t> &pair_t, const std::vector<int32_t> &pair_pos,
                           const BasisTouchTable &touch)
{
    const int64_t n = (int64_t)pair_t.size();
    if (n == 0) return;
    int32_t *d_t = nullptr, *d_pos = nullptr;
    double *d_eq = nullptr, *d_sb = nullptr;
    BCV_HIP(hipMalloc(&d_t, sizeof(int32_t) * n));
    BCV_HIP(hipMalloc(&d_pos, sizeof(int32_t) * n));
    BCV_HIP(hipMalloc(&d_eq, sizeof(double) * touch.equal.size()));
    BCV_HIP(hipMalloc(&d_sb, sizeof(double) * touch.small_big.size()));
    BCV_HIP(hipMemcpy(d_t, pair_t.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    BCV_HIP(hipMemcpy(d_pos, pair_pos.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    BCV_HIP(hipMemcpy(d_eq, touch.equal.data(), sizeof(double) * touch.equal.size(), hipMemcpyHostToDevice));
    BCV_HIP(hipMemcpy(d_sb, touch.small_big.data(), sizeof(double) * touch.small_big.size(), hipMemcpyHostToDevice));
    const int64_t per_launch = int64_t(1) << 24;  // pairs per launch: 2^22 blocks of 256 work-items
    for (int64_t b = 0; b < n; b += per_launch) {
        const int64_t m = std::min(per_launch, n - b);
        basis_block_kernel<<<(unsigned)((m + 3) / 4), 256>>>(m, d_t + b, d_pos + b, p.d_col + b,
                                                            reinterpret_cast<const double4 *>(p.d_leaf_geom), p.L,
                                                            p.d_bcb, p.d_bvb, p.d_btab, d_eq, d_sb, touch.nb,
                                                            p.d_bval);
        check();
    }
    const hipError_t e = hipDeviceSynchronize();
    (void)hipFree(d_t);
    (void)hipFree(d_pos);
    (void)hipFree(d_eq);
    (void)hipFree(d_sb);
    BCV_HIP(e);
}

void launch_basis_near(const bcv_plan_s &p, const double *f, double *u, hipStream_t st)
{
    const auto *geom = reinterpret_cast<const double4 *>(p.d_leaf_geom);
    if (p.n_bwork > 0) {
        basis_near_kernel<<<(unsigned)((p.n_bwork + 3) / 4), 256, 0, st>>>(p.n_bwork, p.d_bwork, p.d_bcb, p.d_bvb,
                                                                        p.d_bcol, p.d_bval, geom, p.L, p.n_leaves,
                                                                        p.d_hi_off, f, p.d_bpartial, u);
        check();
    }
    if (p.n_bsplits > 0) {
        basis_combine_kernel<<<(unsigned)((p.n_bsplits * kBasisRows + 255) / 256), 256, 0, st>>>(
            p.n_bsplits, p.d_bsplits, p.d_bpartial, geom, p.L, p.n_leaves, p.d_hi_off, u);
        check();
    }
}

void launch_basis_zero(const bcv_plan_s &p, double *u, hipStream_t st)
{
    fill_zero_kernel<<<(unsigned)std::min<int64_t>((p.n_dofs + 255) / 256, 4096), 256, 0, st>>>(p.n_dofs, u);
    check();
}

namespace {
BasisOrders basis_orders(const bcv_plan_s &p)
{
    BasisOrders bo{};
    for (int l = 0; l <= kMaxLevel; ++l) {
        bo.k[l] = ncoef(p.q_level[l]);
        bo.r[l] = nreduced(p.q_level[l]);
    }
    bo.ldk = p.K;
    bo.ldr = p.R;
    return bo;
}
}  // namespace

void launch_basis_p2m(const bcv_plan_s &p, const double *f, hipStream_t st)
{
    const auto *geom = reinterpret_cast<const double4 *>(p.d_leaf_geom);
    const unsigned blocks = (unsigned)((p.n_leaves * p.R + 255) / 256);
    // with level-dependent orders the upward pass reads the level-L leaves' moments too
    basis_p2m_kernel<<<blocks, 256, 0, st>>>(p.n_leaves, p.d_leaf_cell, geom, p.L, p.d_hi_off, p.d_btab,
                                             basis_orders(p), p.q_schedule ? 0 : 1, f, p.d_M, p.d_Mr);
    check();
}

void launch_basis_eval(const bcv_plan_s &p, double *u, hipStream_t st)
{
    const auto *geom = reinterpret_cast<const double4 *>(p.d_leaf_geom);
    const unsigned blocks = (unsigned)((p.n_dofs + 255) / 256);
    basis_eval_kernel<<<blocks, 256, 0, st>>>(p.n_dofs, p.n_leaves, p.d_leaf_cell, geom, p.L, p.d_hi_off, p.d_dof_leaf,
                                              p.d_btab, basis_orders(p), p.d_Lam, u);
    check();
}

}  // namespace bcv
