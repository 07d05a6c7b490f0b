// Launchers of the device kernels (kernels.hip, singular.hip).
#pragma once
#include <vector>

#include "internal.hpp"

namespace bcv {

// Algorithm 1 on `stream`: moments, upward pass, interaction phase, downward pass, and the
// near field fused with the evaluation phase. parts: BCV_PART_NEAR | BCV_PART_FAR.
void launch_apply(const bcv_plan_s &p, const double *f, double *u, int parts, hipStream_t stream);
// mapped meshes (mapped.hip): phase 0 P2M, 1 M2M, 2 interaction, 3 L2L; evaluation adds to u
void launch_mapped_phase(const bcv_plan_s &p, const double *f, int phase, hipStream_t stream);
void launch_mapped_eval(const bcv_plan_s &p, double *u, hipStream_t stream);
void launch_mapped_zero(const bcv_plan_s &p, double *u, hipStream_t stream);
void launch_mapped_assemble(const bcv_plan_s &p, const std::vector<int64_t> &touch_entry,
                            const std::vector<int64_t> &work_entry, const std::vector<int32_t> &work_target,
                            const std::vector<int64_t> &work_mirror, const int rule_orders[5],
                            std::vector<double> &cache);
// BtV apply (Algorithm 3): u = <1_w, V[q] - K[g]> from face data qf, gf (device, n_faces each).
void launch_btv(const bcv_plan_s &p, const double *qf, const double *gf, double *u, hipStream_t stream);
// VtB apply (Algorithm 2): uf = <1_f, N f> on every boundary face from leaf densities f.
void launch_vtb(const bcv_plan_s &p, const double *f, double *uf, hipStream_t stream);

// Matrix-core interaction phase (BCV_MIXED_SPLIT16, q = 6): a folded moment row holds
// kSplitRowHalves FP16 values (hi[64], lo[64]); the maxima of |f| are reduced in kFscaleParts parts.
constexpr int kSplitRowHalves = 128;
constexpr int kFscaleParts = 256;
// The A operands of every offset (FP16 bits, in the lane layout of the kernel) and the one entry per
// offset that runs on the vector units, from the FP64 derivative tables G (n_off x K).
void split16_tables(int K, const std::vector<double> &G, int n_off, std::vector<uint16_t> &A, std::vector<float> &G48);

// Stores every near-pair Galerkin entry of the plan in p.d_val (plan time).
void launch_near_assemble(const bcv_plan_s &p, hipStream_t stream);
// p.d_val32 = FP32 copy of p.d_val (plan time, mixed precision).
void launch_near_narrow(const bcv_plan_s &p, hipStream_t stream);
// Overwrites the near entries d_val[entry[k]] (row target[k]; non-touching pairs) with the tensor
// Gauss rule of order[t] points per axis on the target and order[s] on the source (plan time, on
// the null stream; synchronizes). order: one per leaf, 1..16.
void launch_near_assemble_ordered(const bcv_plan_s &p, const std::vector<int64_t> &entry,
                                  const std::vector<int32_t> &target, const std::vector<int8_t> &order);

// Degree-p leaf bases (basis.hip). Plan time: every near pair's block (pair k: target pair_t[k],
// source in p.d_col[k], block at column pair_pos[k] of the target's block row), on the null stream
// (synchronizes). Apply: the near field (overwrites u), a zero fill of u, the leaf moments (full and
// folded rows) and the evaluation of every coefficient (adds to u).
void launch_basis_assemble(const bcv_plan_s &p, const std::vector<int32_t> &pair_t,
                           const std::vector<int32_t> &pair_pos, const BasisTouchTable &touch);
void launch_basis_near(const bcv_plan_s &p, const double *f, double *u, hipStream_t stream);
void launch_basis_zero(const bcv_plan_s &p, double *u, hipStream_t stream);
void launch_basis_p2m(const bcv_plan_s &p, const double *f, hipStream_t stream);
void launch_basis_eval(const bcv_plan_s &p, double *u, hipStream_t stream);

// int_{[0,1]^3} int_{delta+[0,1]^3} 1/|x-y| dy dx for n non-touching integer offsets (host arrays:
// deltas 3 per offset, out n), by an n_gauss-point Gauss-Legendre rule in each of the six variables,
// on the current device.
void regular_cube_pairs(const int *deltas, int n, int n_gauss, double *out);

}  // namespace bcv
