// Internal object layouts behind the opaque bcv_tree / bcv_plan handles.
#pragma once
#include <cstdint>
#include <vector>

#include "common.hpp"

struct bcv_tree_s {
    static constexpr uint32_t kMagic = 0x42435654u;  // "BCVT"
    uint32_t magic = kMagic;
    int L = 0;
    // Cells of all levels, numbered level by level and in Morton order within a level. The
    // children of a marked cell are 8 consecutive cells of the next level (x fastest).
    std::vector<int32_t> lvl_start;  // L + 2 entries
    std::vector<int32_t> ijk;        // 3 per cell
    std::vector<int8_t> level;
    std::vector<uint8_t> refined;    // marked (has children)
    std::vector<int32_t> parent;     // -1 for the root
    std::vector<int32_t> first_child;
    std::vector<int32_t> leaf_of_cell;  // leaf number or -1 (marked cell)
    std::vector<int32_t> leaf_cell;     // cell of each leaf, leaf order

    // Forest of meshes (a single mesh is the forest of one): mesh m occupies [4m, 4m + 1) x [0, 1)^2
    // and has finest level mesh_L[m].
    int n_meshes = 1;
    std::vector<int> mesh_L;
    // Physical domain of each mesh: the cube with lower corner mesh_lo[3m..3m+2] and side mesh_side[m]
    // (the unit cube unless the description says otherwise).
    std::vector<double> mesh_lo, mesh_side;
    // Geometry of each mesh: BCV_GEOM_BOX (the cube itself) or BCV_GEOM_BALL (the cube's octree pushed
    // through the cube-to-ball map onto the inscribed ball).
    std::vector<int8_t> mesh_geom;
    // Touching near entries of ball leaves by the singular rule, per value of the plan's direct flag,
    // in the order of the planner's list: computed by the first plan of the tree, reused by later
    // ones (the near lists depend on the tree and the direct flag only).
    mutable std::vector<double> mapped_touch_cache[2];

    int64_t n_cells() const { return (int64_t)level.size(); }
    int64_t n_leaves() const { return (int64_t)leaf_cell.size(); }
};

namespace bcv {

// Device-side description of one 64-lane interaction (M2L) task: 64 targets of one level that
// share their child position, laid out along rows, and a list of slots, each an interaction offset
// shared by the lanes together with one source row per lane and whether the offset is in that
// lane's own list.
struct M2LTask {
    int32_t slot_begin;  // first slot
    int32_t n_slots;
    int32_t level;  // level of the 64 targets (cell side 2^-level); targets at 64 * task index
    int32_t out;    // -1: write the local coefficients; else the piece's partial block (see M2LSplit)
    uint64_t heads; // lanes that read their own source at a shifting slot (lane 0 and row starts)
};

// A 64-target task whose slot list was cut into `count` pieces (tasks with out = first ...
// first + count - 1, all holding the same targets): their partial local coefficients are summed
// in piece order. `task` is the first piece.
struct M2LSplit {
    int32_t task, first, count, pad;
};

// Tasks are dealt to the 8 XCDs in contiguous ranges of about equal work.
constexpr int kXcds = 8;
// Deepest supported level, and the largest expansion order of any level (q_schedule).
constexpr int kMaxLevel = 9;
constexpr int kMaxSchedQ = 10;

// One wave's share of the near field: entries [begin, end) of the near row of `target`. Rows
// longer than a unit (the coarse leaves, whose extended neighbour lists reach thousands of fine
// leaves) are cut into several units, so that no wave holds the GPU much longer than the others.
struct NearUnit {
    int64_t begin, end;
    int32_t target;
    int32_t out;  // -1: the unit is the whole row and writes u[target]; else its partial-sum index
};

// A target whose row is cut into units: their partial sums are [first, first + count), in row order.
struct NearSplit {
    int32_t target, first, count, pad;
};

// Touching-pair classes in the order of bcv_touching_integrals().
constexpr int kTouchClasses = 7;

// Degree-p leaf bases (bcv_plan_opts.basis_degree): Legendre tensor polynomials of total degree
// <= p on each leaf, p <= kMaxBasisDegree, n_basis(p) = ncoef(p) per leaf.
constexpr int kMaxBasisDegree = 8;

// Exact touching blocks with Legendre weights at degree P (singular_basis.cpp), unit scale (the
// smaller side 1), without 1/(4 pi); every block is nb x nb, [alpha][beta] in the graded order, and
// its leading ncoef(p_t) x ncoef(p_s) corner is the block of degrees (p_t, p_s).
struct BasisTouchTable {
    int P = 0, nb = 0;
    // equal sides: source = target + o, o in {-1,0,1}^3, block index (o0+1) + 3 (o1+1) + 9 (o2+1)
    std::vector<double> equal;
    // target of side 1 at the origin, source of side 2 with lower corner b in {-2..1}^3 (not both
    // -1/0 on every axis), block index (b0+2) + 4 (b1+2) + 16 (b2+2); the pair with the larger
    // target is the transpose (b = minus the small cube's offset)
    std::vector<double> small_big;
};
const BasisTouchTable &basis_touch_table(int P);

// Near-field work of the leaf bases: up to kBasisRows rows (coefficients a0 .. of target t) over
// the columns [j0, j0 + len) of t's block row; out = -1 writes u, else the unit's kBasisRows partial
// sums go to partial[out .. out + kBasisRows).
constexpr int kBasisRows = 8;
struct BasisUnit {
    int64_t j0;
    int32_t t, a0, len, out;
};
// A (target, first row) whose columns are cut into `count` units with partial sums at
// [first, first + count) (in kBasisRows blocks), added in column order.
struct BasisSplit {
    int32_t t, a0, first, count;
};

// Gauss rules and the per-degree moment and evaluation factors of the leaf bases (basis.hip).
constexpr int kMaxBasisQ = kMaxSchedQ;  // expansion orders up to 10 (level-dependent orders)
struct BasisTables {
    double x[kMaxBasisDegree + 3][kMaxBasisDegree + 2];  // [n][k]: n-point Gauss-Legendre nodes on [0, 1]
    double w[kMaxBasisDegree + 3][kMaxBasisDegree + 2];  // and weights (summing to 1)
    double leg[kMaxBasisDegree + 3][kMaxBasisDegree + 1][kMaxBasisDegree + 2];  // [n][a][k] = P_a(2 x_k - 1)
    double t[kMaxBasisDegree + 1][kMaxBasisQ + 1][kMaxBasisDegree + 1];   // [p][b][a]: moments
    double e[kMaxBasisDegree + 1][kMaxBasisDegree + 1][kMaxBasisQ + 1];   // [p][a][b]: evaluation
};
BasisTables basis_tables();
// Expansion sizes per level for the basis kernels: ncoef(q_l) and (q_l + 1)^2, and the row strides.
struct BasisOrders {
    int32_t k[kMaxLevel + 1], r[kMaxLevel + 1];
    int32_t ldk, ldr;
};

// Boundary faces (BtV): a face is (leaf, axis, side), the leaf's face normal to `axis` at its low
// (side 0) or high (side 1) end. A touching (cell, face) pair of equal size is the cube [0,1]^3 and
// the face of the cube at integer offset o in {-1, 0, 1}^3 (units of the cell side); its class
// numbers (axis, o, side) (162 numbers, of which the 108 where the two meet are used).
constexpr int kFaceClasses = 162;
inline int face_class(const int o[3], int ax, int side)
{
    return (((ax * 3 + o[0] + 1) * 3 + o[1] + 1) * 3 + o[2] + 1) * 2 + side;
}

}  // namespace bcv

// Surrogate network (surrogate.cpp): FP32 parameters, gradient and Adam moments on `device`.
struct bcv_mlp_s {
    static constexpr uint32_t kMagic = 0x42435650u ^ 0x00FF00FFu;
    uint32_t magic = kMagic;
    int device = 0;
    int d_in = 0, width = 0;
    int trained = 0;
    int n_gauss_lo = 0, n_gauss_hi = 0;
    double scale = 0.0;  // RMS of the relative residual (J_hi - J_lo) / J_lo over the training pairs
    double kappa = 1.0;  // calibrated factor of the error estimate
    float *d_params = nullptr, *d_grad = nullptr, *d_m = nullptr, *d_v = nullptr;
};

namespace bcv {
constexpr int kMlpIn = 6, kMlpOut = 2;
// Orders of the singular rule for touching mapped cells (lambda, mu, z, s, r; see mapped.hip): within
// about 1.3e-6 relative of the same rule at orders (8, 12, 8, 8, 8) on ball cells of side 1/16 away
// from the cube's edges (1e-4 on cells along an edge, 1e-3 at a corner, where det D Phi tends to 0),
// at 1.8M kernel evaluations per leaf of a uniform region.
constexpr int kMappedRule[5] = {5, 7, 5, 3, 4};
// The singular rule on explicit pairs (4 doubles per cube: lower corner in the reference cube [0,1]^3
// and side; host arrays), results into out (host).
void mapped_rule_values(int64_t n, const double *geom_t, const double *geom_s, const int orders[5], double *out);
int64_t mlp_n_params(const bcv_mlp_s &net);
bcv_mlp_s *mlp_create(int width, uint64_t seed, int device);
void mlp_destroy(bcv_mlp_s *net);
void mlp_get_params(const bcv_mlp_s &net, float *host);
void mlp_set_params(bcv_mlp_s &net, const float *host);
void mlp_forward_host(const bcv_mlp_s &net, int64_t n, const float *X, float *Y);
void mlp_forward_noalloc(const bcv_mlp_s &net, int64_t n, const float *X, float *Y, hipStream_t st);
double mlp_loss_grad_host(const bcv_mlp_s &net, int64_t n, const float *X, const float *r, float *grad);
void mlp_train(bcv_mlp_s &net, const bcv_mlp_train_opts &o, bcv_mlp_train_report *rep);
void surrogate_eval(const bcv_mlp_s &net, int64_t n, const bcv_touch_pair *pairs, double tol, double *value,
                    double *est_err, int32_t *fallback, int64_t *n_fallback);
void touch_pair_quadrature(int device, int64_t n, const bcv_touch_pair *pairs, int n_gauss, double *out);
// Single- and double-layer integrals of the touching (cell, face) classes of side 1 (boundary.cpp).
void boundary_touching_integrals(double V[kFaceClasses], double K[kFaceClasses]);
// Boundary faces of a single-mesh tree: (leaf, axis, side) triples in leaf order, then axis, side.
std::vector<int32_t> tree_faces(const bcv_tree_s &t);
void mlp_save(const bcv_mlp_s &net, const char *path);
bcv_mlp_s *mlp_load(const char *path, int device);
}  // namespace bcv

// An interaction plan other than the VtV one (opts.boundary): the BtV plan, whose lists hold the
// boundary sources only (I(w) ∩ B_l, Algorithm 3), and the VtB plan, whose targets are the boundary
// cells only (Algorithm 2 needs their local coefficients alone). Same layout as the plan's own
// M2L fields; the apply swaps them in.
struct M2LSet {
    int64_t n_tasks = 0, n_pairs = 0, n_m2l_splits = 0, m2l_groups = 0;
    bcv::M2LTask *d_tasks = nullptr;
    int32_t *d_task_targets = nullptr;
    int32_t *d_slot_off = nullptr;
    uint32_t *d_slot_src = nullptr;
    bcv::M2LSplit *d_m2l_splits = nullptr;
    double *d_m2l_partial = nullptr;
    int32_t xcd_begin[bcv::kXcds + 1] = {};
};

struct bcv_plan_s {
    static constexpr uint32_t kMagic = 0x42435650u;  // "BCVP"
    uint32_t magic = kMagic;
    int device = 0;
    int L = 0, q = 0, K = 0;
    int direct = 0, nearfield = 0, precision = 0;
    int near_order = 0;            // 1: level-dependent Gauss rule on the non-touching near pairs
    // Expansion orders per level: q_level[l] = q (fixed) or q + L - l (q_schedule = 1). K is the row
    // stride of the moment and local arrays, ncoef(max order); R = (max order + 1)^2 that of the
    // folded rows.
    int q_schedule = 0;
    int exact_moments = 0;  // q_schedule: every cell's moments to the largest order (M2M untruncated)
    int q_level[bcv::kMaxLevel + 1] = {};
    int R = 0;
    int64_t n_near_ordered = 0;    // near entries that took it
    int64_t n_leaves = 0, n_cells = 0, n_near = 0, n_touch = 0, n_m2l = 0, n_m2l_lanes = 0, n_offsets = 0,
            n_m2l_read_lanes = 0;
    int64_t device_bytes = 0;
    double touch_value[bcv::kTouchClasses];  // touching integrals / (4 pi), smaller side 1
    double *d_uscale = nullptr;  // per leaf: side^5 of its mesh, when some mesh is not the unit cube (else NULL)
    int surrogate_classes = 0;               // classes whose value came from the surrogate

    // Second stream for the near field (streams == 2) and its fork/join events.
    int streams = 1;
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_fork2 = nullptr;  // the second fork of a mapped apply (its interaction phase)

    // Phase timing: a start and a stop event per phase per recorded apply, see bcv_plan_enable_timing.
    std::vector<hipEvent_t> events;
    int timing_cap = 0;
    mutable int timing_used = 0;

    // Host copies needed to launch level-by-level passes.
    std::vector<int32_t> parent_begin;  // per level l: range of marked cells of level l in d_parents
    int64_t n_tasks = 0;
    int64_t n_units = 0, n_splits = 0;
    int32_t near_xcd[bcv::kXcds + 1] = {};     // near-field units of each XCD (contiguous target ranges)
    int64_t n_m2l_splits = 0, m2l_groups = 0;  // split tasks; workgroups of the interaction kernel
    int32_t xcd_begin[bcv::kXcds + 1] = {};     // task range of each XCD
    // q_schedule: the tasks of level l are [level_xcd[l][0], level_xcd[l][kXcds]), cut into XCD
    // ranges like xcd_begin, and launched level by level
    int32_t level_xcd[bcv::kMaxLevel + 1][bcv::kXcds + 1] = {};
    int32_t lvl_start[bcv::kMaxLevel + 2] = {};  // first cell of each level (cells are numbered level by level)

    // Device buffers (owned).
    double *d_leaf_geom = nullptr;  // 4 per leaf: lower corner x, y, z and side
    int32_t *d_leaf_cell = nullptr;
    int32_t *d_cell_leaf = nullptr;  // per cell: its leaf number, -1 for a marked cell (far-field plans)
    int32_t *d_rest_leaves = nullptr;  // the leaves above the finest level, in leaf order
    int64_t n_rest_leaves = 0;
    int64_t *d_split = nullptr;     // per near row: first point-rule entry (touching entries come first)
    uint32_t *d_col = nullptr;      // source leaf | code << 28: code = touch class + 1 (0: not touching),
                                    // + 8 where the source is the smaller cube of a touching pair
    double *d_val = nullptr;        // assembled near entries (nearfield == ASSEMBLED, FP64 plans)
    float *d_val32 = nullptr;       // the same in FP32 (nearfield == ASSEMBLED, mixed plans)
    bcv::NearUnit *d_units = nullptr;   // near-field work units, longest first
    bcv::NearSplit *d_splits = nullptr; // targets whose row spans several units
    double *d_partial = nullptr;        // one partial near sum per unit of a split row
    double *d_M = nullptr;          // moments, (n_cells + 1) x K; the last row stays zero
    double *d_Lam = nullptr;        // local coefficients, n_cells x K
    double *d_G = nullptr;          // derivative tables, n_offsets x K
    float *d_M32 = nullptr;         // BCV_MIXED_F32: folded moments in FP32, (n_cells + 1) x (q + 1)^2
    double *d_Mr = nullptr;         // BCV_FP64: folded moments, (n_cells + 1) x (q + 1)^2
    float *d_G32 = nullptr;         // BCV_MIXED_F32: FP32 derivative tables
    int32_t *d_parents = nullptr;   // (marked cell, first child) pairs, grouped by level
    bcv::M2LTask *d_tasks = nullptr;
    int32_t *d_task_targets = nullptr;  // 64 per task, -1 = idle lane
    int32_t *d_slot_off = nullptr;      // offset id per slot | (the slot gathers) << 31
    uint32_t *d_slot_src = nullptr;     // 64 per slot: source row (n_cells: none) | (in the lane's list) << 31
    uint64_t *d_slot_mask = nullptr;    // BCV_MIXED_SPLIT16: per slot, bit t = the offset is in target t's list
    uint32_t *d_m2l_A = nullptr;        // BCV_MIXED_SPLIT16: per offset, the matrix-core A operands (see kernels.hip)
    float *d_G48 = nullptr;             // BCV_MIXED_SPLIT16: per offset, the one entry handled off the matrix cores
    uint16_t *d_M16 = nullptr;          // BCV_MIXED_SPLIT16: folded moments as FP16 hi/lo rows, (n_cells + 1) x 128
    float *d_fscale = nullptr;          // BCV_MIXED_SPLIT16: partial maxima of |f| (256) and the scale (1)
    bcv::M2LSplit *d_m2l_splits = nullptr;
    double *d_m2l_partial = nullptr;    // 64 x K per piece of a split task

    // Degree-p leaf bases (opts.basis_degree = 1): leaf w has ncoef(L - level) coefficients; entries
    // 0 .. n_leaves - 1 of f and u are the degree-0 ones, the others follow leaf by leaf.
    int basis = 0;
    int basis_P = 0;                  // largest leaf degree
    int64_t n_dofs = 0;               // length of f and u
    int64_t n_bvals = 0, n_bcols = 0, n_bwork = 0, n_bsplits = 0;
    int64_t *d_hi_off = nullptr;      // per leaf: first higher coefficient minus n_leaves
    int32_t *d_dof_leaf = nullptr;    // per higher coefficient: its leaf
    int64_t *d_bcb = nullptr;         // n_leaves + 1: near row of target t is columns [bcb[t], bcb[t+1])
    int64_t *d_bvb = nullptr;         // per target leaf: first block entry (row alpha at + alpha row_len)
    int32_t *d_bcol = nullptr;        // near-row columns: source coefficient positions
    double *d_bval = nullptr;         // near-field blocks
    bcv::BasisUnit *d_bwork = nullptr;    // apply work units, longest first
    bcv::BasisSplit *d_bsplits = nullptr; // rows cut into several units
    double *d_bpartial = nullptr;         // kBasisRows partial sums per unit of a cut row
    bcv::BasisTables *d_btab = nullptr;

    // Mapped meshes (some mesh of the tree is BCV_GEOM_BALL): every cell's expansion centre is the
    // image of its reference centre, every leaf has its own moment row, the interaction phase works
    // pair by pair, and the near field is assembled (mapped.hip).
    int mapped = 0;
    double *d_leaf_pts = nullptr;   // 8 per leaf: mapped Gauss point x, y, z and weight
    double *d_centre = nullptr;     // 4 per cell: expansion centre x, y, z and side a (reference frame)
    double *d_kap = nullptr;        // per leaf: kappa^b = sum_g w_g ((x_g - x_w)/a)^b / b!, K entries
    double *d_kapr = nullptr;       // per leaf: the folded rows of (-1)^|b| kappa^b, R entries
    uint8_t *d_leaf_mapped = nullptr;  // per leaf: 1 if its mesh is a ball
    int64_t n_ilist = 0;            // interaction-list pairs of the ball cells (levels >= 2), CSR by target
    int64_t n_ilist_targets = 0;
    int32_t *d_ilist_tgt = nullptr;   // the target cells
    int64_t *d_ilist_off = nullptr;
    int32_t *d_ilist_src = nullptr;
    int64_t n_mapped_touch = 0;     // touching near entries of ball leaves (singular rule)
    int64_t n_mapped_pairs = 0;     // of which computed (a pair and its mirror once)

    // BtV (Algorithm 3), built when the plan options ask for it.
    int boundary = 0;
    M2LSet btv_m2l, vtb_m2l;  // their interaction plans (far-field plans only)
    int64_t n_faces = 0, n_btv_near = 0, n_btv_touch = 0, n_btv_units = 0, n_btv_splits = 0;
    uint32_t *d_faces = nullptr;        // per boundary face: leaf | (2 axis + side) << 28
    int32_t *d_leaf_faces = nullptr;    // n_leaves + 1: the faces of leaf t are [d_leaf_faces[t], d_leaf_faces[t + 1])
    uint32_t *d_btv_col = nullptr;      // near entries: face | (touching class + 1) << 24 (0: point rule)
    bcv::NearUnit *d_btv_units = nullptr;
    bcv::NearSplit *d_btv_splits = nullptr;
    double *d_btv_partial = nullptr;
    double *d_btv_touch = nullptr;      // 2 x kFaceClasses: V, then K, of touching pairs of side 1
    // VtB (Algorithm 2): near rows of the boundary faces, sources from the near row of the face's cell
    int64_t n_vtb_near = 0, n_vtb_units = 0, n_vtb_splits = 0;
    uint32_t *d_vtb_col = nullptr;      // source leaf | (touching class + 1) << 24 (0: point rule)
    bcv::NearUnit *d_vtb_units = nullptr;  // targets are faces
    bcv::NearSplit *d_vtb_splits = nullptr;
    double *d_vtb_partial = nullptr;
};

// A captured apply (graph.cpp).
struct bcv_graph_s {
    static constexpr uint32_t kMagic = 0x42434752u;  // "BCGR"
    uint32_t magic = kMagic;
    int device = 0;
    const bcv_plan_s *plan = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace bcv {
bcv_graph_s *graph_create(const bcv_plan_s &p, const double *f, double *u);
void graph_launch(const bcv_graph_s &g, hipStream_t st);
void graph_destroy(bcv_graph_s *g);
double autotune(const bcv_tree_s &t, const bcv_plan_opts &base, int device, int n_applies, bcv_plan_opts &best);
}  // namespace bcv
