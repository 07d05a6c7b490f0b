/*
 * bcv.h -- C ABI of the boundary-concentrated FMM for Galerkin volume potentials on MI355X (gfx950).
 *
 * The library evaluates the volume-to-volume (VtV) potential of Mohyaddin & Tausch,
 * "A fast method for evaluating volume potentials in the Galerkin boundary element method":
 * given a density f that is constant on each leaf of a boundary-concentrated (BC) mesh of
 * Omega = [0,1]^3, it returns the Galerkin coefficients
 *
 *     u_w = < 1_w , N f >_{L2(Omega)},   N f(x) = int_Omega G(x,y) f(y) dy,   G = 1/(4 pi |x-y|)
 *
 * for every leaf w (Sec. 1: volume potential and its L2 projection with degree-0 elements;
 * Sec. 3: Algorithm 1). The mesh is a cube octree refined towards the boundary (Sec. 2 with
 * cube cells); the far field uses Cartesian Taylor expansions of order q (Sec. 3, translation
 * operators); the near field uses exact integrals for touching cell pairs and the 2x2x2 Gauss
 * rule on both cells otherwise.
 *
 * Conventions shared by every entry point:
 *   - Every call returns a bcv_status. No C++ exception crosses this interface. On failure the
 *     thread-local message returned by bcv_last_error() describes the cause.
 *   - The library owns trees and plans (opaque handles, created here, freed by *_destroy).
 *     The caller owns every pointer it passes.
 *   - Device pointers are HIP device addresses on the plan's device; host pointers are ordinary
 *     process memory. Each argument says which it is.
 *   - Leaf order: leaves are numbered by the Morton key of their lower corner at level-L
 *     resolution (bit b of i, j, k at bits 3b, 3b+1, 3b+2). bcv_tree_leaves() exposes
 *     (level, i, j, k) per leaf in this order; densities and potentials use it.
 *   - A plan may be used from any host thread. Calls that run on one plan and overlap in time
 *     (two streams, or two threads) race on the plan's workspace: serialise them.
 */
#ifndef BCV_H
#define BCV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bcv_tree_s *bcv_tree;
typedef struct bcv_plan_s *bcv_plan;
typedef struct bcv_mlp_s *bcv_mlp;
typedef struct bcv_graph_s *bcv_graph;

typedef enum {
    BCV_OK = 0,
    BCV_EINVAL = 1,  /* an argument is out of range or a required pointer is NULL */
    BCV_ENOMEM = 2,  /* host or device allocation failed */
    BCV_EDEVICE = 3, /* a HIP call failed; bcv_last_error() carries the HIP message */
    BCV_ENOTSUP = 4, /* valid request that the library does not implement */
    BCV_ESTATE = 5   /* a handle is not a live object of the expected kind */
} bcv_status;

/* Mesh description (Sec. 2, Boundary Concentrated Mesh, with cube cells).
 * Level 0 is the domain cube; level-l cells are cubes of side s 2^-l (s the side of the domain). For
 * l < L a cell is marked (refined) by the marking rule; every level-L cell is a leaf. */
enum {
    BCV_GEOM_BOX = 0, /* the axis-aligned cube [lo, hi] (all of lo and hi zero: the unit cube [0,1]^3) */
    BCV_GEOM_BALL = 1 /* the ball inscribed in the cube [lo, hi]: the cube's BC octree pushed through the
                         analytic cube-to-sphere map (volume form of the mapping reviewed by Zucker and
                         Higashi, JCGT 7(2), 2018; with u = 2 xi - 1, y_i = u_i sqrt(1 - u_j^2/2 - u_k^2/2
                         + u_j^2 u_k^2/3)). Cells are curved; the near and interaction lists are those
                         of the reference octree, expansion centres the images of the reference centres,
                         non-touching entries the mapped 2x2x2 rule (weights (a^3/8) det D Phi), touching
                         entries a singular rule in the relative coordinate (Sec. 1.2 entries on curved
                         cells). Plans need BCV_NEAR_ASSEMBLED, q = 4, 6 or 8, BCV_FP64 or BCV_MIXED_F32,
                         and no boundary, basis, surrogate, level-dependent order or near_order options
                         (BCV_ENOTSUP otherwise); a forest may mix cubes and balls */
};
enum {
    BCV_MARK_FACE = 0,     /* marked iff the cell has a face on the boundary (M_l = B_l) */
    BCV_MARK_NEIGHBOR = 1  /* marked iff a neighbour (eq. def:neighbors, eta0 = 1/2) has a face on the
                              boundary: the marking rule of Sec. 2. With cube cells this refines
                              every cell within three cells of the boundary (all of levels 0-3), and
                              near-field pairs differ by at most two levels (up to L - 1 with
                              BCV_MARK_FACE) */
};
typedef struct {
    int geometry;     /* BCV_GEOM_BOX or BCV_GEOM_BALL */
    double lo[3];     /* lower corner of the domain cube */
    double hi[3];     /* upper corner; hi - lo must be the same positive side s on all three axes */
    int L;            /* finest level, 2 <= L <= 9 (boundary leaves have side h = s 2^-L) */
    int marking;      /* BCV_MARK_FACE or BCV_MARK_NEIGHBOR */
} bcv_mesh_desc;
/* Every operator scales exactly with the side: on the cube of side s the VtV entries are s^5 times
 * those of the unit cube (u = <1_w, N f>: volumes s^3 twice, the kernel 1/s), the VtB ones s^4, the
 * BtV single-layer ones s^4 and the double-layer ones s^3; a translation changes nothing. The library
 * computes on the unit cube and applies these factors. */

enum { BCV_NEAR_QUADRATURE = 0, BCV_NEAR_ASSEMBLED = 1 };
/* Arithmetic of the apply.
 * BCV_FP64: every phase in FP64.
 * BCV_MIXED_F32: the interaction phase (M2L) reads FP32 copies of the (folded) moments and the
 *   derivative tables and accumulates in FP32; the non-touching near-field pairs evaluate their 64
 *   kernel values in FP32 (per-axis differences formed in FP64), or, assembled, are stored in FP32;
 *   the touching (singular) pairs, the moments, the upward and downward passes, the evaluation and
 *   the final accumulation of u stay in FP64. */
/* BCV_MIXED_SPLIT16: as BCV_MIXED_F32, but the VtV apply's interaction phase runs on the matrix
 *   cores (MFMA): every FP32 operand is split into two FP16 numbers (hi + lo), the three products
 *   hi*hi + hi*lo + lo*hi are accumulated in FP32 (about 22 significant bits per operand). The folded
 *   moments are scaled by the cell volume and by the power of two at or above max |f| before the split.
 *   Fixed q = 6 only (q_schedule = 0); BtV and VtB applies of such a plan run their interaction
 *   phase as BCV_MIXED_F32 does. */
enum { BCV_FP64 = 0, BCV_MIXED_F32 = 1, BCV_MIXED_SPLIT16 = 2 };

/* Plan options. */
typedef struct {
    double eta0;   /* separation parameter of the neighbour test (eq. def:neighbors); must be 0.5 */
    int q;         /* expansion order, |alpha| + |beta| <= q (Sec. 3): 0..10. Orders 4, 6 and 8 have
                      their own interaction kernels; 0-3, 5, 7, 9 and 10 run the level-by-level
                      kernels of q_schedule with the same order on every level (single-mesh trees,
                      no opts.boundary) */
    int precision; /* BCV_FP64, BCV_MIXED_F32 or BCV_MIXED_SPLIT16 */
    int direct;    /* 1: every leaf pair is treated as near (no far field; small meshes only) */
    int nearfield; /* BCV_NEAR_QUADRATURE: the apply evaluates every near-pair entry on the fly;
                      BCV_NEAR_ASSEMBLED: the plan stores every near-pair entry once (computed in
                      FP64; stored in FP32 by BCV_MIXED_F32 plans, whose apply takes the touching
                      pairs' exact values in FP64 instead) and the apply multiplies by them */
    int streams;   /* 1: every phase runs on the caller's stream, in Algorithm 1's order;
                      2: after the upward pass, the near field is forked to a plan-owned second
                      stream (default priority), runs concurrently with the interaction phase
                      and the downward pass, and is joined back to the caller's stream before
                      the evaluation phase. Plans with cube-to-ball meshes fork twice instead:
                      the near field after P2M (beside M2M), then the ball cells' interaction
                      pairs beside the cube cells' interaction tasks, both joined before L2L */
    bcv_mlp surrogate;     /* NULL: the touching-pair integrals come from bcv_touching_integrals.
                              Else each of the six face/edge/vertex classes takes the trained
                              surrogate's value where its error estimate is <= surrogate_tol
                              (relative) and keeps the exact table value where it is not; the
                              self class keeps the exact value. The plan copies the values: the
                              network may be destroyed afterwards. */
    double surrogate_tol;  /* e.g. 1e-7; 0 forces the fallback for every class */
    int near_unit;         /* work-unit size of the near field: rows longer than this many entries are
                              cut into pieces of about equal length (0 = 2048; else 64..65536) */
    int m2l_max_slots;     /* longest slot list of one interaction task; longer lists are cut into
                              pieces whose partial sums are added in a fixed order (0 = 320, or 256
                              with q_schedule = 1 or under 2^20 slots in all; else 16..65536) */
    int q_schedule;        /* 0: the expansion order q on every level. 1: level-dependent orders
                              q_l = q + L - l (Sec. 4, the FMM error with level-dependent orders;
                              q is the finest level's): a level-l cell carries moments and local
                              coefficients of degree <= q_l, M2M maps a child's degree <= q_{l+1}
                              moments to the parent's degree <= q_l ones, the interaction phase at
                              level l truncates at |alpha| + |beta| <= q_l, and L2L keeps the
                              child's degrees <= q_{l+1}. Requires q + L - 2 <= 10 and a single-mesh
                              tree, and is not combined with opts.boundary */
    int near_order;        /* Gauss rule of the non-touching near-field pairs (Sec. 4, near-field
                              quadrature: fixed order on the finest level, raised on coarser ones).
                              0: 2x2x2 points on each cell. 1: a level-l leaf takes n_l = 2 + L - l
                              points per axis, and a pair takes n_l^3 points on each of its two
                              cells (the entry stays symmetric). 1 requires BCV_NEAR_ASSEMBLED (the
                              plan computes the entries once, in FP64); far pairs are unchanged */
    int boundary;          /* 1: also build the BtV structures (boundary faces, their near lists
                              and touching integrals) so that bcv_btv_apply can run; single-mesh
                              trees only. 0: VtV only */
    int basis_degree;      /* leaf bases (Sec. 1.2, the space S_h with degree-p_w polynomials on each
                              leaf). 0: degree 0, the indicator of each leaf (one unknown per leaf).
                              1: p_w = L - l on a leaf of level l (Sec. 4, approximation errors: this
                              choice with degree 0 on the finest level gives the O(h) best
                              approximation), basis phi^alpha_w(x) = prod_i P_{alpha_i}(2 (x_i - c_i)/a)
                              (Legendre, centre c and side a of w), |alpha| <= p_w, ncoef(p_w) =
                              (p_w+1)(p_w+2)(p_w+3)/6 unknowns per leaf; f holds the coefficients of the
                              density in this basis and u receives u_(w,alpha) = <phi^alpha_w, N f>.
                              Every leaf then carries the tensor Gauss rule of p_w + 2 points per
                              axis for its non-touching pairs, moments and evaluation; touching pairs
                              are exact (bcv_touching_basis_block). Layout of f and u: entries
                              0 .. n_leaves-1 are the alpha = 0 coefficients in leaf order, followed
                              by the alpha = 1 .. ncoef(p_w)-1 coefficients of every leaf with
                              p_w > 0, leaf by leaf (alpha in the graded order of
                              bcv_touching_basis_block); n_dofs in bcv_plan_info. The near field is
                              assembled at plan time (opts.nearfield is ignored). Combines with any
                              q and with q_schedule (the paper's experiments take p_l = L - l with
                              q_l = 4 + L - l, Sec. 5). Requires BCV_FP64, a single mesh of side 1, no
                              surrogate, no opts.boundary, and L - (coarsest leaf level) <= 8 */
    int exact_moments;     /* with q_schedule = 1 only (Algorithm 1's upward pass, the other reading of
                              its M2M with level-dependent orders). 0: as q_schedule describes (a
                              parent's top-degree moments receive only its children's lower-degree
                              terms). 1: every cell carries moments of degree <= the largest order
                              q + L - 2 (leaf moments to that degree, M2M untruncated), so a cell's
                              moments are those of all of its leaves; the interaction phase at level
                              l still uses the degrees <= q_l. Requires q_schedule = 1 and
                              basis_degree = 0 */
} bcv_plan_opts;

/* Sizes of a plan (all counts, no pointers). */
typedef struct {
    int64_t n_leaves;     /* unknowns */
    int64_t n_cells;      /* all cells of all levels */
    int64_t n_near;       /* ordered near (target leaf, source leaf) pairs */
    int64_t n_touch;      /* of which the closed cubes touch (exact singular entries) */
    int64_t n_m2l;        /* ordered interaction-list pairs (cells), all levels */
    int64_t n_m2l_lanes;  /* lane-pairs the interaction kernel executes (>= n_m2l; padding) */
    int64_t n_offsets;    /* distinct integer interaction offsets (derivative tables) */
    int64_t n_m2l_read_lanes; /* of n_m2l_lanes, those whose source moments the lane-shifting
                               * interaction kernels (FP32; FP64 up to q = 6) read from memory;
                               * the rest arrive by a lane shift */
    int64_t n_faces;      /* boundary faces (plans built with opts.boundary; else 0) */
    int64_t n_btv_near;   /* BtV near (leaf, face) pairs */
    int64_t n_btv_touch;  /* of which the closed cell and face meet (exact integrals) */
    int64_t n_vtb_near;   /* VtB near (face, source leaf) pairs */
    int64_t n_near_ordered; /* near entries that took the level-dependent rule (opts.near_order 1) */
    int64_t device_bytes; /* device memory held by the plan */
    int32_t K;            /* expansion coefficients per cell, (q+1)(q+2)(q+3)/6 */
    int32_t L;
    int32_t surrogate_classes; /* touching classes whose value came from the surrogate (0..6) */
    int32_t pad;
    int64_t n_dofs;       /* length of f and u: n_leaves, or with opts.basis_degree = 1 the number of
                             basis coefficients of all leaves */
    int64_t n_basis_vals; /* near-field block entries held by a plan with opts.basis_degree = 1 */
    int64_t n_basis_cols; /* their distinct columns: per target leaf, the coefficients of its near
                             sources (shared by the target's rows) */
    int64_t n_btv_m2l;    /* interaction-list pairs of the BtV apply: boundary sources only (0
                             without opts.boundary or for a direct plan) */
    int64_t n_vtb_m2l;    /* interaction-list pairs of the VtB apply: boundary targets only */
    int64_t n_mapped_touch_pairs; /* touching pairs of ball leaves (a pair and its mirror counted once) */
} bcv_plan_info;

/* Build the BC octree of Sec. 2 on the host. desc and out must be non-NULL.
 * Errors: BCV_EINVAL (L outside 2..9, marking not 0 or 1, a box that is not a cube of positive side),
 * BCV_ENOMEM. */
bcv_status bcv_build_bc_tree(const bcv_mesh_desc *desc, bcv_tree *out);

/* A forest of n_meshes BC meshes for a batched apply: one tree, one plan and one apply (and one
 * captured graph) evaluate all meshes at once. descs[m] describes mesh m (same rules as
 * bcv_build_bc_tree, 1 <= n_meshes <= 4096). Mesh m occupies [4m, 4m + 1) x [0, 1)^2 in units of a
 * level-0 cube, so leaves (level, i, j, k) of mesh m have i in [4m 2^level, (4m + 1) 2^level);
 * meshes never interact. Leaf order: the Morton order of the whole forest (bcv_tree_leaf_mesh
 * tells the mesh of each leaf). Errors: BCV_EINVAL, BCV_ENOMEM. */
bcv_status bcv_build_bc_forest(int n_meshes, const bcv_mesh_desc *descs, bcv_tree *out);

/* Mesh of every leaf (host, n_leaves int32). */
bcv_status bcv_tree_leaf_mesh(bcv_tree tree, int32_t *mesh_of_leaf);

/* Number of leaves (host integer). */
bcv_status bcv_tree_num_leaves(bcv_tree tree, int64_t *n);

/* Per leaf, in leaf order (host arrays, each may be NULL):
 *   level_ijk: n_leaves x 4 int32, (level, i, j, k) in units of the level's cell side (forests: the
 *              index space of bcv_build_bc_forest);
 *   gauss_xyz: n_leaves x 8 x 3 doubles, the 2x2x2 Gauss-Legendre points of the leaf in physical
 *              coordinates (x fastest: point g has offsets 1/2 -+ 1/(2 sqrt 3) of the side, bit 0 of g
 *              along x, bit 1 along y, bit 2 along z), the points of the point rule, the moments and
 *              the evaluation (Sec. 3 with this reading of the integrals);
 *   gauss_w:   n_leaves x 8 doubles, their weights |w|/8.
 * On a BCV_GEOM_BALL mesh the points are the images of the reference cube's points under the map and
 * the weights (s 2^-l)^3 / 8 times det D Phi there (s the side of the mesh's cube).
 * Errors: BCV_EINVAL (tree NULL), BCV_ESTATE. */
bcv_status bcv_tree_leaves(bcv_tree tree, int32_t *level_ijk, double *gauss_xyz, double *gauss_w);

void bcv_tree_destroy(bcv_tree tree);

/* Build the interaction plan of Sec. 3 for `tree` on HIP device `device`: neighbour lists
 * (eq. def:neighbors), interaction lists, extended neighbour lists N* with marked sources
 * expanded to their leaves (Lemma 1, eq. spaceDecomp:OmOm), touching classes, derivative
 * tables, and all device workspace. Allocates device memory; the apply never does.
 * The plan copies what it needs: the tree may be destroyed afterwards.
 * Errors: BCV_EINVAL (NULL pointers, eta0 != 0.5, q not supported, unknown precision),
 * BCV_ENOTSUP, BCV_ENOMEM, BCV_EDEVICE, BCV_ESTATE (bad tree handle). */
bcv_status bcv_plan_interactions(bcv_tree tree, const bcv_plan_opts *opts, int device, bcv_plan *out);

bcv_status bcv_plan_get_info(bcv_plan plan, bcv_plan_info *info);

void bcv_plan_destroy(bcv_plan plan);

/* VtV apply, Algorithm 1: u = near field + far field for density f.
 *   f_dev: device, n_leaves doubles in leaf order (the density value on each leaf);
 *   u_dev: device, n_leaves doubles in leaf order, OVERWRITTEN with u_w = <1_w, N f>.
 *   hip_stream: a hipStream_t on the plan's device (NULL = the null stream).
 * Stream-ordered and asynchronous: returns after enqueueing; allocates nothing.
 * f_dev and u_dev must not overlap. Errors: BCV_EINVAL (NULL pointers), BCV_ESTATE, BCV_EDEVICE. */
bcv_status bcv_vtv_apply(bcv_plan plan, const double *f_dev, double *u_dev, void *hip_stream);

/* Applies of several plans, one after another on one stream (Algorithm 1 for each mesh):
 *   plans: host array of n plan handles, all on the same device;
 *   f_dev, u_dev: host arrays of n device pointers; plan i reads f_dev[i] and overwrites u_dev[i]
 *   (n_leaves of plan i doubles each, leaf order), as bcv_vtv_apply does.
 * Stream-ordered, asynchronous, allocates nothing. Many small meshes run faster as one forest
 * (bcv_build_bc_forest: one plan, one apply, optionally one graph). 1 <= n <= 4096.
 * Errors: BCV_EINVAL (NULL arrays or pointers, n out of range, plans on different devices),
 * BCV_ESTATE, BCV_EDEVICE. */
bcv_status bcv_vtv_apply_batched(const bcv_plan *plans, int n, const double *const *f_dev, double *const *u_dev,
                                 void *hip_stream);

/* The same apply restricted to parts of Algorithm 1, for testing and timing:
 * parts = BCV_PART_NEAR (near field only), BCV_PART_FAR (moments through evaluation only),
 * or both. u_dev is overwritten with the sum of the selected parts. */
enum { BCV_PART_NEAR = 1, BCV_PART_FAR = 2 };
bcv_status bcv_vtv_apply_parts(bcv_plan plan, const double *f_dev, double *u_dev, void *hip_stream, int parts);

/* Per-phase device timing of applies, with HIP events recorded around each phase of Algorithm 1
 * on the stream it runs on: moments (P2M), upward pass (M2M), interaction phase (M2L), downward
 * pass (L2L), near field (NEAR; with streams = 1 it also contains the evaluation phase) and
 * evaluation (EVAL; streams = 2 only).
 * bcv_plan_enable_timing creates 2 * BCV_N_PHASES * max_applies events (host call, may allocate) and resets
 * the record; each following apply records its phase boundaries until max_applies applies have
 * been recorded (later applies are not timed). max_applies = 0 disables timing and frees the
 * events. bcv_plan_phase_times waits for the recorded events and returns, per phase, the total
 * milliseconds over the recorded applies (ms: host, BCV_N_PHASES doubles) and the number of
 * recorded applies (n_applies: host). Errors: BCV_EINVAL, BCV_ESTATE, BCV_EDEVICE. */
enum {
    BCV_PHASE_P2M = 0,
    BCV_PHASE_M2M = 1,
    BCV_PHASE_M2L = 2,
    BCV_PHASE_L2L = 3,
    BCV_PHASE_NEAR = 4,
    BCV_PHASE_EVAL = 5,
    BCV_N_PHASES = 6
};
bcv_status bcv_plan_enable_timing(bcv_plan plan, int max_applies);
bcv_status bcv_plan_phase_times(bcv_plan plan, double *ms, int64_t *n_applies);

/* The full apply (bcv_vtv_apply with both parts) captured once into an instantiated HIP graph:
 * every kernel of every phase, and the second stream's fork and join, become one graph launch.
 * Each launch reads f_dev and overwrites u_dev at the addresses given here (device, n_leaves
 * doubles each, owned by the caller, kept alive while the graph is used). The graph uses the
 * plan's workspace: launches must not overlap with each other or with applies of the same plan,
 * and the plan must outlive the graph. Phase timing must be off while capturing.
 * Errors: BCV_EINVAL, BCV_ESTATE (timing enabled, bad handle), BCV_EDEVICE. */
bcv_status bcv_vtv_graph_create(bcv_plan plan, const double *f_dev, double *u_dev, bcv_graph *out);
bcv_status bcv_graph_launch(bcv_graph graph, void *hip_stream);
void bcv_graph_destroy(bcv_graph graph);

/* Autotuner of the plan's work decomposition: for the tree and base options, builds plans with
 * candidate near_unit (256, 512, 1024, 2048) and then m2l_max_slots (128, 256, 320, 512, 1024) values,
 * times n_applies applies of each (HIP events, after two warm-up applies, density 1) on `device`,
 * and returns the options of the fastest plan in *best and its milliseconds per apply in *best_ms
 * (host). Allocates and frees plans and buffers. Errors: as bcv_plan_interactions. */
bcv_status bcv_autotune(bcv_tree tree, const bcv_plan_opts *base, int device, int n_applies, bcv_plan_opts *best,
                        double *best_ms);

/* Boundary faces of a single-mesh tree (BtV data lives on them): the faces of level-L leaves in
 * the planes x, y, z = 0 or 1 of the unit cube (every cell meeting the boundary has a face on it
 * and is refined down to level L). Face f is (leaf, axis, side): the leaf's face normal to `axis`
 * at its low (side 0) or high (side 1) end, outward normal (2 side - 1) e_axis. Order: by leaf,
 * then axis, then side. leaf_axis_side: host, n_faces x 3 int32.
 * Errors: BCV_EINVAL (NULL), BCV_ENOTSUP (a forest of several meshes). */
bcv_status bcv_tree_num_faces(bcv_tree tree, int64_t *n_faces);
bcv_status bcv_tree_faces(bcv_tree tree, int32_t *leaf_axis_side);

/* Boundary-to-volume apply, Algorithm 3 (BC-FMM for the BtV calculation), degree p = 0:
 *   u_w = <1_w, V[q] - K[g]>_{L2(w)} for every leaf w,
 *   V[q](x) = int_Gamma G(x - y) q(y) dS_y,  K[g](x) = int_Gamma dG(x - y)/dn_y g(y) dS_y,
 * G = 1/(4 pi |x - y|), Gamma the boundary of the unit cube, n its outward normal, q and g
 * constant on each boundary face (Sec. 1: for harmonic u, q = du/dn and g = u give u in the cube
 * by Green's representation formula).
 *   q_face_dev, g_face_dev: device, n_faces doubles each, in bcv_tree_faces order;
 *   u_dev: device, n_leaves doubles in leaf order, OVERWRITTEN.
 * Near pairs (the face's cell has an ancestor at the leaf's level among the leaf's neighbours)
 * use the exact integrals of bcv_boundary_touching_integrals where the closed cell and face meet
 * and the 2x2x2 x 2x2 point rule otherwise (FP32 kernel evaluations in BCV_MIXED_F32); the rest
 * goes through boundary moments (2x2 point rule per face), the upward pass, the interaction phase,
 * the downward pass and the evaluation phase of the plan. The plan must have been built with
 * opts.boundary = 1. Stream-ordered on hip_stream only (streams = 2 plays no part), asynchronous,
 * allocates nothing. Overwrites the plan's moment and local-coefficient workspace: do not run it
 * concurrently with another apply of the same plan.
 * Errors: BCV_EINVAL (NULL pointers), BCV_ESTATE (plan without boundary structures), BCV_EDEVICE. */
bcv_status bcv_btv_apply(bcv_plan plan, const double *q_face_dev, const double *g_face_dev, double *u_dev,
                         void *hip_stream);

/* Volume-to-boundary apply, Algorithm 2 (BC-FMM for the VtB calculation), degree p = 0 on the
 * faces: u_f = <1_f, N f_h>_{L2(f)} = int_f int_Omega G(x - y) f_h(y) dy dS_x for every boundary
 * face f, with f_h piecewise constant on the leaves.
 *   f_dev: device, n_leaves doubles in leaf order;
 *   u_face_dev: device, n_faces doubles in bcv_tree_faces order, OVERWRITTEN.
 * The near sources of a face are the near sources N*(w) of its level-L cell w (Algorithm 1's near
 * list); their entries are the single-layer entries of bcv_btv_apply (G is symmetric: the
 * discrete VtB operator is the transpose of the single-layer part of the discrete BtV operator).
 * The far field: moments of every leaf, upward pass, interaction phase, downward pass, and the local
 * expansion of w integrated over the face by the 2x2 point rule. Requires opts.boundary = 1 and at
 * most 2^24 leaves. Stream-ordered on hip_stream, asynchronous, allocates nothing; overwrites the
 * plan's moment and local-coefficient workspace (no concurrent applies of one plan).
 * Errors: BCV_EINVAL (NULL pointers), BCV_ESTATE (plan without boundary structures), BCV_EDEVICE. */
bcv_status bcv_vtb_apply(bcv_plan plan, const double *f_dev, double *u_face_dev, void *hip_stream);

/* The exact single- and double-layer integrals of touching (cell, boundary face) pairs of side 1:
 * V[c] = int_cube int_face G dS dx and K[c] = int_cube int_face dG/dn_y dS dx for the unit cube
 * [0,1]^3 and the face normal to `axis` at the low (side 0) or high (side 1) end of the unit cube
 * at integer offset o in {-1, 0, 1}^3, class c = (((axis 3 + o0 + 1) 3 + o1 + 1) 3 + o2 + 1) 2 + side
 * (162 classes; 0 where cell and face do not meet). Computed on the host once per process from the
 * self-similarity of the pair (halving the cube and the face) with regular pairs integrated by a
 * 5-D Gauss rule. V, K: host, 162 doubles each. Errors: BCV_EINVAL (NULL). */
bcv_status bcv_boundary_touching_integrals(double *V, double *K);

/* The seven exact touching-pair integrals int_A int_B 1/|x-y| the library uses for the singular
 * near-field entries (smaller side 1; order: self, face, edge, vertex, then face, edge, vertex
 * with the larger side 2). Computed on `device` once per process from the self-similarity of
 * the cube (splitting both cubes into halves) with regular pairs integrated by a 6-D Gauss rule.
 * out: host, 7 doubles. Errors: BCV_EINVAL, BCV_EDEVICE. */
bcv_status bcv_touching_integrals(int device, double *out);

/* Exact touching block of the degree-p leaf bases (Sec. 1.2, the finite element space with
 * polynomials on each leaf; bcv_plan_opts.basis_degree): int_t int_s phi^alpha_t(x) phi^beta_s(y)
 * / |x - y| dy dx for two touching cubes t, s of sides side_t, side_s in {1, 2} (units of the smaller
 * side: (1, 1), (1, 2) or (2, 1)), with s's lower corner at `offset` (3 ints, same units) from t's,
 * phi^alpha_w(x) = prod_i P_{alpha_i}(2 (x_i - c_i)/a) (Legendre, centre c and side a of w), all
 * |alpha| <= p_t, |beta| <= p_s in the graded order of the coefficients (total degree, then alpha_x
 * descending, then alpha_y descending). Scale: entries of cubes with smaller side a are the values
 * times a^5 (and 1/(4 pi) for the kernel G). Computed on the host, once per process and degree,
 * from the self-similarity of the cube (halving both cubes, the weights re-expanded on the halves)
 * with regular pairs integrated by a 6-D Gauss rule; no device is used. out: host,
 * ncoef(p_t) x ncoef(p_s) doubles, row-major, ncoef(p) = (p+1)(p+2)(p+3)/6. Errors: BCV_EINVAL
 * (NULL, degrees outside 0..8, sides or offset of cubes that do not touch or that overlap). */
bcv_status bcv_touching_basis_block(int p_t, int p_s, int side_t, int side_s, const int *offset, double *out);

/* ---- Touching-pair surrogate -------------------------------------------------------------
 * A small network (features -> width -> width -> 2, SiLU, FP32, trained on the GPU by the library's
 * own forward, backward and Adam kernels) that corrects a low-order quadrature of the Galerkin
 * integral of 1/|x-y| over two touching cubes to the accuracy of the high-order quadrature, which
 * stays the fallback and the reference of its error estimate (Sec. 3: singular near-field entries by singularity-removing
 * transforms and tensor Gauss rules).
 *
 * Canonical touching pair: A = [0,1]^3 is the smaller cube; B is a cube of side rho in [1, 2]
 * touching A's +x face (FACE), the +x,+y edge (EDGE) or the +x,+y,+z vertex (VERTEX). B's lower
 * corner is (1, off[0], off[1]) for FACE, (1, 1, off[0]) for EDGE and (1, 1, 1) for VERTEX, with
 * every used off[k] in (-rho, 1). Any touching pair of axis-aligned cubes with side ratio in [1, 2]
 * maps onto this form by a rigid motion and a scaling by the smaller side a; its Galerkin entry is
 * J * a^5 / (4 pi) with J the canonical integral. */
enum { BCV_CONTACT_FACE = 1, BCV_CONTACT_EDGE = 2, BCV_CONTACT_VERTEX = 3 };
typedef struct {
    int32_t contact; /* BCV_CONTACT_* */
    int32_t pad;
    double rho;      /* side of B / side of A, in [1, 2] */
    double off[2];   /* free coordinates of B's lower corner; unused entries are ignored */
} bcv_touch_pair;

typedef struct {
    int64_t n_train, n_valid; /* training pairs and held-out pairs (random canonical pairs) */
    int32_t epochs, batch;    /* passes over the training pairs; minibatch size */
    double lr;                /* peak Adam step (cosine decay to 0) */
    uint64_t seed;            /* pairs, shuffling */
    int32_t n_gauss_lo;       /* Gauss order of the corrected quadrature (e.g. 4) */
    int32_t n_gauss_hi;       /* Gauss order of the reference quadrature (e.g. 16, at most 16) */
    double tol;               /* acceptance tolerance used for the held-out report */
} bcv_mlp_train_opts;

/* The n_valid held-out pairs are split in two: the first half calibrates the error estimate, the
 * second half (valid_reported pairs, never used for training or calibration) gives the figures
 * below; with n_valid = 1 the one pair serves both. */
typedef struct {
    double residual_scale;             /* RMS of (J_hi - J_lo) / J_lo over the training pairs */
    double kappa;                      /* factor of the error estimate, calibrated on the first half
                                          of the held-out pairs: 1.5 x max (true error / raw estimate) */
    double valid_max_rel_err_lo;       /* reported pairs: max |J_lo - J_hi| / |J_hi| (without the network) */
    double valid_max_rel_err;          /* reported pairs: max relative error of the corrected value */
    double valid_rms_rel_err;
    double valid_max_rel_err_accepted; /* reported pairs: max relative error among accepted pairs */
    int64_t valid_accepted;            /* reported pairs whose error estimate is <= tol */
    int64_t valid_reported;            /* size of the reported half */
} bcv_mlp_train_report;

/* J for n pairs of axis-aligned boxes by the high-order quadrature: geom holds 12 doubles per pair
 * (A lower corner, A upper corner, B lower corner, B upper corner), n_gauss points (1..16) per
 * direction on every cell of the graded decomposition; out[n]. Host arrays; runs on `device`. A pair
 * whose decomposition exceeds the kernel's lists gets NaN. Errors: BCV_EINVAL, BCV_ENOMEM, BCV_EDEVICE. */
bcv_status bcv_box_pair_integrals(int device, int64_t n, const double *geom, int n_gauss, double *out);
/* The same for canonical touching pairs (host arrays). Errors: BCV_EINVAL (not a touching pair). */
bcv_status bcv_touch_pair_quadrature(int device, int64_t n, const bcv_touch_pair *pairs, int n_gauss, double *out);

/* A network of the given width (2..1024) with seeded uniform(+-1/sqrt(fan-in)) weights on `device`. */
bcv_status bcv_mlp_create(int width, uint64_t seed, int device, bcv_mlp *out);
void bcv_mlp_destroy(bcv_mlp mlp);
/* Parameters as one FP32 vector, in this order: W1 [6 x width] (row-major, input-major), b1 [width],
 * W2 [width x width], b2 [width], W3 [width x 2], b3 [2]. Host arrays of bcv_mlp_num_params floats. */
bcv_status bcv_mlp_num_params(bcv_mlp mlp, int64_t *n);
bcv_status bcv_mlp_get_params(bcv_mlp mlp, float *params);
bcv_status bcv_mlp_set_params(bcv_mlp mlp, const float *params);
/* Y [n x 2] = network(X [n x 6]) with the GPU kernels (host arrays). */
bcv_status bcv_mlp_forward(bcv_mlp mlp, int64_t n, const float *X, float *Y);
/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): bcv_mlp_forward on device arrays, allocating nothing.
 *   X_dev: device, n x 6 floats (row-major features); Y_dev: device, n x 2 floats, OVERWRITTEN;
 *   both owned by the caller, on the network's device; hip_stream: a hipStream_t there (NULL = null
 *   stream). Stream-ordered and asynchronous; the same kernels, in the same order, as
 *   bcv_mlp_forward, so the outputs are identical.
 * The hidden activations live in a fixed workspace the library holds in a static device array
 * (12 MiB per GPU it runs on, kept until the process ends): n x width must not exceed 2^20
 * (n <= 8192 at width 128), else BCV_EINVAL. Every call on one GPU shares that GPU's workspace
 * (the first call on a device looks its address up): calls that overlap in time on one GPU race
 * and give wrong results; serialise them (one stream, or events). n = 0 does nothing.
 * Errors: BCV_EINVAL (NULL pointers with n > 0, n too large), BCV_ESTATE (bad handle), BCV_EDEVICE. */
bcv_status bcv_mlp_forward_noalloc(bcv_mlp mlp, int64_t n, const float *X_dev, float *Y_dev, void *hip_stream);
/* Training loss of the batch (X [n x 6], targets r [n]) and its gradient with respect to every
 * parameter (host arrays; grad has bcv_mlp_num_params floats), with the GPU kernels:
 *   loss = mean (y0 - r)^2 + 0.1 mean (y1 - log(|y0 - r| + 1e-5))^2, the second term with y0 fixed. */
bcv_status bcv_mlp_loss_grad(bcv_mlp mlp, int64_t n, const float *X, const float *r, double *loss, float *grad);
/* Generates the pairs, computes J at both Gauss orders on the GPU, and trains with Adam. */
bcv_status bcv_mlp_train(bcv_mlp mlp, const bcv_mlp_train_opts *opts, bcv_mlp_train_report *report);
/* value[i] = the corrected J of pair i where its error estimate est_err[i] <= tol (relative; the raw
 * estimate of the network's second output times the calibrated factor kappa), else the
 * high-order quadrature (fallback[i] = 1); n_fallback counts the fallbacks. Host arrays.
 * Errors: BCV_ESTATE (untrained network), BCV_EINVAL. */
bcv_status bcv_surrogate_eval(bcv_mlp mlp, int64_t n, const bcv_touch_pair *pairs, double tol, double *value,
                              double *est_err, int32_t *fallback, int64_t *n_fallback);
/* Flat file: header (magic, version, inputs, width, both Gauss orders, residual scale, kappa) then the
 * FP32 parameters. */
/* Entries of n touching pairs of cube-to-ball mapped cells by the planner's singular rule (the
 * touching entries of BCV_GEOM_BALL plans, Sec. 1.2 entries on curved cells): cube t of pair i is
 * geom_t[4i..4i+3] (lower corner in the reference cube [0,1]^3, side 2^-l, l <= 12, a cube of the
 * octree), its partner geom_s[4i..4i+3] (equal cubes, or of equal side or ratio 2 with closed cubes
 * touching from outside); value[i] = int int G J J over the two curved cells of the unit-diameter ball.
 * Host arrays; synchronous. Errors: BCV_EINVAL (NULL arrays, cubes not of the octree or not
 * touching), BCV_EDEVICE. */
bcv_status bcv_mapped_pair_entries(int device, int64_t n, const double *geom_t, const double *geom_s, double *value);
bcv_status bcv_mlp_save(bcv_mlp mlp, const char *path);
bcv_status bcv_mlp_load(const char *path, int device, bcv_mlp *out);

/* Thread-local description of the last failure on this thread (valid until the next call). */
const char *bcv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BCV_H */
