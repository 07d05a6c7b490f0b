// extern "C" entry points of bcv.h: argument checks, handle checks, and translation of C++
// exceptions into bcv_status plus a thread-local message.
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "ballmap.hpp"
#include "internal.hpp"
#include "multiindex.hpp"
#include "kernels.hpp"
#include "quadrature.hpp"

namespace bcv {
bcv_tree_s *build_tree(int L, int marking);
bcv_tree_s *build_forest(int n, const int *Ls, const int *markings, const double *lo, const double *side,
                         const int *geoms);
bcv_plan_s *build_plan(const bcv_tree_s &t, const bcv_plan_opts &opts, int device);
void destroy_plan(bcv_plan_s *p);
void touching_integrals(int device, double out[kTouchClasses]);
void set_timing(bcv_plan_s *p, int max_applies);
void phase_times(const bcv_plan_s *p, double *ms, int64_t *n);
}  // namespace bcv

namespace {

thread_local std::string g_error;

template <class F>
bcv_status guard(F &&f)
{
    try {
        f();
        g_error.clear();
        return BCV_OK;
    } catch (const bcv::Error &e) {
        g_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_error = "host allocation failed";
        return BCV_ENOMEM;
    } catch (const std::exception &e) {
        g_error = std::string("internal error: ") + e.what();
        return BCV_ESTATE;
    } catch (...) {
        g_error = "internal error";
        return BCV_ESTATE;
    }
}

void check_tree(bcv_tree t)
{
    BCV_REQUIRE(t != nullptr, BCV_EINVAL, "tree handle is NULL");
    BCV_REQUIRE(t->magic == bcv_tree_s::kMagic, BCV_ESTATE, "not a live bcv_tree");
}

void check_mlp(bcv_mlp m)
{
    BCV_REQUIRE(m != nullptr, BCV_EINVAL, "network handle is NULL");
    BCV_REQUIRE(m->magic == bcv_mlp_s::kMagic, BCV_ESTATE, "not a live bcv_mlp");
}

void check_device(int device)
{
    int n_dev = 0;
    BCV_HIP(hipGetDeviceCount(&n_dev));
    BCV_REQUIRE(device >= 0 && device < n_dev, BCV_EINVAL, "no such HIP device");
}

// A mesh description: level, marking rule and a cube domain; writes the cube's lower corner and side.
void check_mesh_desc(const bcv_mesh_desc &d, double lo[3], double *side)
{
    BCV_REQUIRE(d.L >= 2 && d.L <= 9, BCV_EINVAL, "L must be in 2..9");
    BCV_REQUIRE(d.marking == 0 || d.marking == 1, BCV_EINVAL, "marking must be 0 or 1");
    BCV_REQUIRE(d.geometry == BCV_GEOM_BOX || d.geometry == BCV_GEOM_BALL, BCV_EINVAL,
                "geometry must be BCV_GEOM_BOX or BCV_GEOM_BALL");
    bool unit = true;
    for (int ax = 0; ax < 3; ++ax) unit = unit && d.lo[ax] == 0.0 && d.hi[ax] == 0.0;
    if (unit) {
        lo[0] = lo[1] = lo[2] = 0.0;
        *side = 1.0;
        return;
    }
    const double s = d.hi[0] - d.lo[0];
    BCV_REQUIRE(std::isfinite(s) && s > 0.0, BCV_EINVAL, "the box must have a positive side");
    for (int ax = 0; ax < 3; ++ax) {
        BCV_REQUIRE(std::isfinite(d.lo[ax]) && std::isfinite(d.hi[ax]), BCV_EINVAL, "the box must be finite");
        BCV_REQUIRE(std::fabs((d.hi[ax] - d.lo[ax]) - s) <= 1e-12 * s, BCV_EINVAL,
                    "the box must be a cube (the same side on every axis)");
        lo[ax] = d.lo[ax];
    }
    *side = s;
}

void check_plan_opts(const bcv_plan_opts &o, int device)
{
    BCV_REQUIRE(o.eta0 == 0.5, BCV_EINVAL, "eta0 must be 0.5");
    BCV_REQUIRE(o.q >= 0 && o.q <= 10, BCV_EINVAL, "q must be in 0..10");
    BCV_REQUIRE(o.precision == BCV_FP64 || o.precision == BCV_MIXED_F32 || o.precision == BCV_MIXED_SPLIT16,
                BCV_EINVAL, "precision must be BCV_FP64, BCV_MIXED_F32 or BCV_MIXED_SPLIT16");
    BCV_REQUIRE(o.direct == 0 || o.direct == 1, BCV_EINVAL, "direct must be 0 or 1");
    BCV_REQUIRE(o.nearfield == BCV_NEAR_QUADRATURE || o.nearfield == BCV_NEAR_ASSEMBLED, BCV_EINVAL,
                "unknown nearfield mode");
    BCV_REQUIRE(o.streams == 1 || o.streams == 2, BCV_EINVAL, "streams must be 1 or 2");
    BCV_REQUIRE(o.near_unit == 0 || (o.near_unit >= 64 && o.near_unit <= 65536), BCV_EINVAL,
                "near_unit must be 0 or 64..65536");
    BCV_REQUIRE(o.m2l_max_slots == 0 || (o.m2l_max_slots >= 16 && o.m2l_max_slots <= 65536),
                BCV_EINVAL, "m2l_max_slots must be 0 or 16..65536");
    BCV_REQUIRE(o.boundary == 0 || o.boundary == 1, BCV_EINVAL, "boundary must be 0 or 1");
    BCV_REQUIRE(o.near_order == 0 || o.near_order == 1, BCV_EINVAL, "near_order must be 0 or 1");
    BCV_REQUIRE(o.q_schedule == 0 || o.q_schedule == 1, BCV_EINVAL, "q_schedule must be 0 or 1");
    BCV_REQUIRE(o.exact_moments == 0 || o.exact_moments == 1, BCV_EINVAL, "exact_moments must be 0 or 1");
    BCV_REQUIRE(o.exact_moments == 0 || (o.q_schedule == 1 && o.basis_degree == 0), BCV_ENOTSUP,
                "exact_moments requires q_schedule = 1 and basis_degree = 0");
    BCV_REQUIRE(o.q_schedule == 0 || o.boundary == 0, BCV_ENOTSUP,
                "level-dependent orders are not combined with the boundary (BtV/VtB) structures");
    BCV_REQUIRE(o.q == 4 || o.q == 6 || o.q == 8 || o.boundary == 0, BCV_ENOTSUP,
                "the boundary (BtV/VtB) structures need q = 4, 6 or 8");
    BCV_REQUIRE(o.near_order == 0 || o.nearfield == BCV_NEAR_ASSEMBLED, BCV_EINVAL,
                "near_order 1 needs the assembled near field (BCV_NEAR_ASSEMBLED)");
    BCV_REQUIRE(o.basis_degree == 0 || o.basis_degree == 1, BCV_EINVAL, "basis_degree must be 0 or 1");
    BCV_REQUIRE(o.basis_degree == 0 || (o.precision == BCV_FP64 && !o.boundary && !o.surrogate), BCV_ENOTSUP,
                "degree-p leaf bases need BCV_FP64, no boundary structures and no surrogate");
    if (o.surrogate) {
        check_mlp(o.surrogate);
        BCV_REQUIRE(o.surrogate_tol >= 0.0, BCV_EINVAL, "negative surrogate tolerance");
        BCV_REQUIRE(o.surrogate->device == device, BCV_EINVAL, "the surrogate lives on another device");
    }
    int n_dev = 0;
    BCV_HIP(hipGetDeviceCount(&n_dev));
    BCV_REQUIRE(device >= 0 && device < n_dev, BCV_EINVAL, "no such HIP device");
}

void check_plan(bcv_plan p)
{
    BCV_REQUIRE(p != nullptr, BCV_EINVAL, "plan handle is NULL");
    BCV_REQUIRE(p->magic == bcv_plan_s::kMagic, BCV_ESTATE, "not a live bcv_plan");
}

// Runs f with the plan's device current and restores the caller's device afterwards.
template <class F>
void on_device(int device, F &&f)
{
    int old = 0;
    BCV_HIP(hipGetDevice(&old));
    BCV_HIP(hipSetDevice(device));
    try {
        f();
    } catch (...) {
        (void)hipSetDevice(old);
        throw;
    }
    BCV_HIP(hipSetDevice(old));
}

}  // namespace

extern "C" {

bcv_status bcv_build_bc_forest(int n_meshes, const bcv_mesh_desc *descs, bcv_tree *out)
{
    return guard([&] {
        BCV_REQUIRE(descs != nullptr && out != nullptr, BCV_EINVAL, "NULL argument");
        *out = nullptr;
        BCV_REQUIRE(n_meshes >= 1 && n_meshes <= 4096, BCV_EINVAL, "n_meshes must be in 1..4096");
        std::vector<int> Ls(n_meshes), marks(n_meshes), geoms(n_meshes);
        std::vector<double> lo(3 * (size_t)n_meshes), side(n_meshes);
        for (int m = 0; m < n_meshes; ++m) {
            check_mesh_desc(descs[m], &lo[3 * (size_t)m], &side[m]);
            Ls[m] = descs[m].L;
            marks[m] = descs[m].marking;
            geoms[m] = descs[m].geometry;
        }
        *out = bcv::build_forest(n_meshes, Ls.data(), marks.data(), lo.data(), side.data(), geoms.data());
    });
}

bcv_status bcv_tree_leaf_mesh(bcv_tree tree, int32_t *mesh_of_leaf)
{
    return guard([&] {
        check_tree(tree);
        BCV_REQUIRE(mesh_of_leaf != nullptr, BCV_EINVAL, "NULL argument");
        for (int64_t l = 0; l < tree->n_leaves(); ++l) {
            const int32_t c = tree->leaf_cell[l];
            mesh_of_leaf[l] = (tree->ijk[3 * c] >> tree->level[c]) / 4;
        }
    });
}

bcv_status bcv_build_bc_tree(const bcv_mesh_desc *desc, bcv_tree *out)
{
    return guard([&] {
        BCV_REQUIRE(desc != nullptr && out != nullptr, BCV_EINVAL, "NULL argument");
        *out = nullptr;
        double lo[3], side = 1.0;
        check_mesh_desc(*desc, lo, &side);
        const int L = desc->L, marking = desc->marking, geom = desc->geometry;
        *out = bcv::build_forest(1, &L, &marking, lo, &side, &geom);
    });
}

bcv_status bcv_tree_num_leaves(bcv_tree tree, int64_t *n)
{
    return guard([&] {
        check_tree(tree);
        BCV_REQUIRE(n != nullptr, BCV_EINVAL, "NULL argument");
        *n = tree->n_leaves();
    });
}

bcv_status bcv_tree_leaves(bcv_tree tree, int32_t *level_ijk, double *gauss_xyz, double *gauss_w)
{
    return guard([&] {
        check_tree(tree);
        const double node[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
        for (int64_t l = 0; l < tree->n_leaves(); ++l) {
            const int32_t c = tree->leaf_cell[l];
            const int lev = tree->level[c];
            if (level_ijk) {
                level_ijk[4 * l] = lev;
                for (int ax = 0; ax < 3; ++ax) level_ijk[4 * l + 1 + ax] = tree->ijk[3 * c + ax];
            }
            if (!gauss_xyz && !gauss_w) continue;
            const int m = (tree->ijk[3 * c] >> lev) / 4;  // mesh m occupies [4m, 4m + 1) in level-0 units
            const double s = tree->mesh_side[m], a = std::ldexp(s, -lev);
            const int64_t local[3] = {tree->ijk[3 * c] - ((int64_t)4 * m << lev), tree->ijk[3 * c + 1],
                                      tree->ijk[3 * c + 2]};
            const double ar = std::ldexp(1.0, -lev);  // side in the mesh's reference cube
            for (int g = 0; g < 8; ++g) {
                double x[3], p[3], jac = 1.0;
                for (int ax = 0; ax < 3; ++ax) x[ax] = ar * ((double)local[ax] + node[(g >> ax) & 1]);
                if (tree->mesh_geom[m] == BCV_GEOM_BALL)
                    bcv::ball_map(x, p, &jac);
                else
                    p[0] = x[0], p[1] = x[1], p[2] = x[2];
                if (gauss_xyz)
                    for (int ax = 0; ax < 3; ++ax) gauss_xyz[(8 * l + g) * 3 + ax] = tree->mesh_lo[3 * m + ax] + s * p[ax];
                if (gauss_w) gauss_w[8 * l + g] = a * a * a * 0.125 * jac;
            }
        }
    });
}

bcv_status bcv_vtv_apply_batched(const bcv_plan *plans, int n, const double *const *f_dev, double *const *u_dev,
                                 void *hip_stream)
{
    return guard([&] {
        BCV_REQUIRE(plans != nullptr && f_dev != nullptr && u_dev != nullptr, BCV_EINVAL, "NULL argument");
        BCV_REQUIRE(n >= 1 && n <= 4096, BCV_EINVAL, "n must be in 1..4096");
        for (int i = 0; i < n; ++i) {
            check_plan(plans[i]);
            BCV_REQUIRE(f_dev[i] != nullptr && u_dev[i] != nullptr, BCV_EINVAL, "NULL density or potential pointer");
            BCV_REQUIRE(plans[i]->device == plans[0]->device, BCV_EINVAL, "the plans live on different devices");
        }
        on_device(plans[0]->device, [&] {
            for (int i = 0; i < n; ++i)
                bcv::launch_apply(*plans[i], f_dev[i], u_dev[i], BCV_PART_NEAR | BCV_PART_FAR, (hipStream_t)hip_stream);
        });
    });
}

void bcv_tree_destroy(bcv_tree tree)
{
    if (tree && tree->magic == bcv_tree_s::kMagic) {
        tree->magic = 0;
        delete tree;
    }
}

bcv_status bcv_plan_interactions(bcv_tree tree, const bcv_plan_opts *opts, int device, bcv_plan *out)
{
    return guard([&] {
        check_tree(tree);
        BCV_REQUIRE(opts != nullptr && out != nullptr, BCV_EINVAL, "NULL argument");
        *out = nullptr;
        check_plan_opts(*opts, device);
        on_device(device, [&] { *out = bcv::build_plan(*tree, *opts, device); });
    });
}

bcv_status bcv_plan_get_info(bcv_plan plan, bcv_plan_info *info)
{
    return guard([&] {
        check_plan(plan);
        BCV_REQUIRE(info != nullptr, BCV_EINVAL, "NULL argument");
        info->n_leaves = plan->n_leaves;
        info->n_cells = plan->n_cells;
        info->n_near = plan->n_near;
        info->n_touch = plan->n_touch;
        info->n_m2l = plan->n_m2l;
        info->n_m2l_lanes = plan->n_m2l_lanes;
        info->n_offsets = plan->n_offsets;
        info->n_m2l_read_lanes = plan->n_m2l_read_lanes;
        info->n_faces = plan->n_faces;
        info->n_btv_near = plan->n_btv_near;
        info->n_btv_touch = plan->n_btv_touch;
        info->n_vtb_near = plan->n_vtb_near;
        info->n_near_ordered = plan->n_near_ordered;
        info->device_bytes = plan->device_bytes;
        info->K = plan->K;
        info->L = plan->L;
        info->surrogate_classes = plan->surrogate_classes;
        info->pad = 0;
        info->n_dofs = plan->basis ? plan->n_dofs : plan->n_leaves;
        info->n_basis_vals = plan->n_bvals;
        info->n_basis_cols = plan->n_bcols;
        info->n_btv_m2l = plan->btv_m2l.n_pairs;
        info->n_vtb_m2l = plan->vtb_m2l.n_pairs;
        info->n_mapped_touch_pairs = plan->n_mapped_pairs;
    });
}

void bcv_plan_destroy(bcv_plan plan)
{
    if (plan && plan->magic == bcv_plan_s::kMagic) bcv::destroy_plan(plan);
}

bcv_status bcv_vtv_apply_parts(bcv_plan plan, const double *f_dev, double *u_dev, void *hip_stream, int parts)
{
    return guard([&] {
        check_plan(plan);
        BCV_REQUIRE(f_dev != nullptr && u_dev != nullptr, BCV_EINVAL, "NULL density or potential pointer");
        BCV_REQUIRE(parts >= 1 && parts <= 3, BCV_EINVAL, "parts must be a non-empty subset of NEAR|FAR");
        on_device(plan->device, [&] { bcv::launch_apply(*plan, f_dev, u_dev, parts, (hipStream_t)hip_stream); });
    });
}

bcv_status bcv_vtv_apply(bcv_plan plan, const double *f_dev, double *u_dev, void *hip_stream)
{
    return bcv_vtv_apply_parts(plan, f_dev, u_dev, hip_stream, BCV_PART_NEAR | BCV_PART_FAR);
}

bcv_status bcv_plan_enable_timing(bcv_plan plan, int max_applies)
{
    return guard([&] {
        check_plan(plan);
        BCV_REQUIRE(max_applies >= 0 && max_applies <= 1000000, BCV_EINVAL, "max_applies out of range");
        on_device(plan->device, [&] { bcv::set_timing(plan, max_applies); });
    });
}

bcv_status bcv_plan_phase_times(bcv_plan plan, double *ms, int64_t *n_applies)
{
    return guard([&] {
        check_plan(plan);
        BCV_REQUIRE(ms != nullptr && n_applies != nullptr, BCV_EINVAL, "NULL argument");
        on_device(plan->device, [&] { bcv::phase_times(plan, ms, n_applies); });
    });
}

bcv_status bcv_vtb_apply(bcv_plan plan, const double *f_dev, double *u_face_dev, void *hip_stream)
{
    return guard([&] {
        check_plan(plan);
        BCV_REQUIRE(f_dev != nullptr && u_face_dev != nullptr, BCV_EINVAL, "NULL density or face pointer");
        BCV_REQUIRE(plan->boundary, BCV_ESTATE, "the plan was built without boundary structures (opts.boundary)");
        on_device(plan->device, [&] { bcv::launch_vtb(*plan, f_dev, u_face_dev, (hipStream_t)hip_stream); });
    });
}

bcv_status bcv_btv_apply(bcv_plan plan, const double *q_face_dev, const double *g_face_dev, double *u_dev,
                         void *hip_stream)
{
    return guard([&] {
        check_plan(plan);
        BCV_REQUIRE(q_face_dev != nullptr && g_face_dev != nullptr && u_dev != nullptr, BCV_EINVAL,
                    "NULL face data or potential pointer");
        BCV_REQUIRE(plan->boundary, BCV_ESTATE, "the plan was built without boundary structures (opts.boundary)");
        on_device(plan->device, [&] { bcv::launch_btv(*plan, q_face_dev, g_face_dev, u_dev, (hipStream_t)hip_stream); });
    });
}

bcv_status bcv_tree_num_faces(bcv_tree tree, int64_t *n_faces)
{
    return guard([&] {
        check_tree(tree);
        BCV_REQUIRE(n_faces != nullptr, BCV_EINVAL, "NULL argument");
        *n_faces = (int64_t)bcv::tree_faces(*tree).size() / 3;
    });
}

bcv_status bcv_tree_faces(bcv_tree tree, int32_t *leaf_axis_side)
{
    return guard([&] {
        check_tree(tree);
        BCV_REQUIRE(leaf_axis_side != nullptr, BCV_EINVAL, "NULL argument");
        const std::vector<int32_t> f = bcv::tree_faces(*tree);
        std::copy(f.begin(), f.end(), leaf_axis_side);
    });
}

bcv_status bcv_boundary_touching_integrals(double *V, double *K)
{
    return guard([&] {
        BCV_REQUIRE(V != nullptr && K != nullptr, BCV_EINVAL, "NULL argument");
        bcv::boundary_touching_integrals(V, K);
    });
}

bcv_status bcv_touching_integrals(int device, double *out)
{
    return guard([&] {
        BCV_REQUIRE(out != nullptr, BCV_EINVAL, "NULL argument");
        int n_dev = 0;
        BCV_HIP(hipGetDeviceCount(&n_dev));
        BCV_REQUIRE(device >= 0 && device < n_dev, BCV_EINVAL, "no such HIP device");
        on_device(device, [&] { bcv::touching_integrals(device, out); });
    });
}

bcv_status bcv_touching_basis_block(int p_t, int p_s, int side_t, int side_s, const int *offset, double *out)
{
    return guard([&] {
        BCV_REQUIRE(offset != nullptr && out != nullptr, BCV_EINVAL, "NULL argument");
        BCV_REQUIRE(p_t >= 0 && p_s >= 0 && p_t <= bcv::kMaxBasisDegree && p_s <= bcv::kMaxBasisDegree, BCV_EINVAL,
                    "basis degrees must be 0..8");
        const bool equal = side_t == 1 && side_s == 1;
        BCV_REQUIRE(equal || (side_t == 1 && side_s == 2) || (side_t == 2 && side_s == 1), BCV_EINVAL,
                    "sides must be (1, 1), (1, 2) or (2, 1)");
        // b: lower corner of the side-2 cube relative to the side-1 cube (pairs of sides 1 and 2)
        int b[3];
        for (int ax = 0; ax < 3; ++ax) b[ax] = side_t == 2 ? -offset[ax] : offset[ax];
        bool ok = true, inside = true;
        for (int ax = 0; ax < 3; ++ax) {
            ok = ok && (equal ? (b[ax] >= -1 && b[ax] <= 1) : (b[ax] >= -2 && b[ax] <= 1));
            inside = inside && (b[ax] == -1 || b[ax] == 0);
        }
        BCV_REQUIRE(ok && (equal || !inside), BCV_EINVAL, "the cubes do not touch (or overlap)");
        const bcv::BasisTouchTable &tab = bcv::basis_touch_table(std::max(p_t, p_s));
        const int nt = bcv::ncoef(p_t), ns = bcv::ncoef(p_s), nb = tab.nb;
        const double *blk = equal ? &tab.equal[(size_t)((b[0] + 1) + 3 * (b[1] + 1) + 9 * (b[2] + 1)) * nb * nb]
                                  : &tab.small_big[(size_t)((b[0] + 2) + 4 * (b[1] + 2) + 16 * (b[2] + 2)) * nb * nb];
        for (int a = 0; a < nt; ++a)
            for (int c = 0; c < ns; ++c)
                out[(size_t)a * ns + c] = side_t == 2 ? blk[(size_t)c * nb + a] : blk[(size_t)a * nb + c];
    });
}

bcv_status bcv_box_pair_integrals(int device, int64_t n, const double *geom, int n_gauss, double *out)
{
    return guard([&] {
        BCV_REQUIRE(n >= 0 && (n == 0 || (geom != nullptr && out != nullptr)), BCV_EINVAL, "bad arguments");
        check_device(device);
        on_device(device, [&] { bcv::box_pair_integrals(device, n, geom, n_gauss, out); });
    });
}

bcv_status bcv_touch_pair_quadrature(int device, int64_t n, const bcv_touch_pair *pairs, int n_gauss, double *out)
{
    return guard([&] {
        BCV_REQUIRE(n >= 0 && (n == 0 || (pairs != nullptr && out != nullptr)), BCV_EINVAL, "bad arguments");
        BCV_REQUIRE(n_gauss >= 1 && n_gauss <= 16, BCV_EINVAL, "Gauss order must be 1..16");
        check_device(device);
        on_device(device, [&] { bcv::touch_pair_quadrature(device, n, pairs, n_gauss, out); });
    });
}

bcv_status bcv_mlp_create(int width, uint64_t seed, int device, bcv_mlp *out)
{
    return guard([&] {
        BCV_REQUIRE(out != nullptr, BCV_EINVAL, "NULL argument");
        *out = nullptr;
        check_device(device);
        on_device(device, [&] { *out = bcv::mlp_create(width, seed, device); });
    });
}

bcv_status bcv_mapped_pair_entries(int device, int64_t n, const double *geom_t, const double *geom_s, double *value)
{
    return guard([&] {
        check_device(device);
        BCV_REQUIRE(n >= 0 && (n == 0 || (geom_t && geom_s && value)), BCV_EINVAL, "bad arguments");
        for (int64_t i = 0; i < n; ++i) {
            const double *g[2] = {geom_t + 4 * i, geom_s + 4 * i};
            for (const double *c : g) {
                BCV_REQUIRE(c[3] > 0.0, BCV_EINVAL, "sides must be 2^-l, l in 0..12");
                const int lev = -std::ilogb(c[3]);
                BCV_REQUIRE(std::ldexp(1.0, -lev) == c[3] && lev >= 0 && lev <= 12, BCV_EINVAL,
                            "sides must be 2^-l, l in 0..12");
                for (int ax = 0; ax < 3; ++ax)
                    BCV_REQUIRE(c[ax] >= 0.0 && c[ax] + c[3] <= 1.0 &&
                                    std::ldexp(c[ax], lev) == std::floor(std::ldexp(c[ax], lev)),
                                BCV_EINVAL, "a cube of the reference octree inside [0,1]^3");
            }
            const double big = std::max(g[0][3], g[1][3]), small = std::min(g[0][3], g[1][3]);
            BCV_REQUIRE(big == small || big == 2.0 * small, BCV_EINVAL, "sides equal or in ratio 2");
            bool touch = true, overlap = true;
            for (int ax = 0; ax < 3; ++ax) {
                const double lo = std::max(g[0][ax], g[1][ax]), hi = std::min(g[0][ax] + g[0][3], g[1][ax] + g[1][3]);
                touch = touch && lo <= hi;
                overlap = overlap && lo < hi;
            }
            BCV_REQUIRE(touch && (!overlap || big == small), BCV_EINVAL,
                        "the closed cubes must touch (equal cubes, or a smaller cube outside the larger)");
        }
        on_device(device, [&] { bcv::mapped_rule_values(n, geom_t, geom_s, bcv::kMappedRule, value); });
    });
}

void bcv_mlp_destroy(bcv_mlp mlp)
{
    if (mlp && mlp->magic == bcv_mlp_s::kMagic) bcv::mlp_destroy(mlp);
}

bcv_status bcv_mlp_num_params(bcv_mlp mlp, int64_t *n)
{
    return guard([&] {
        check_mlp(mlp);
        BCV_REQUIRE(n != nullptr, BCV_EINVAL, "NULL argument");
        *n = bcv::mlp_n_params(*mlp);
    });
}

bcv_status bcv_mlp_get_params(bcv_mlp mlp, float *params)
{
    return guard([&] {
        check_mlp(mlp);
        BCV_REQUIRE(params != nullptr, BCV_EINVAL, "NULL argument");
        on_device(mlp->device, [&] { bcv::mlp_get_params(*mlp, params); });
    });
}

bcv_status bcv_mlp_set_params(bcv_mlp mlp, const float *params)
{
    return guard([&] {
        check_mlp(mlp);
        BCV_REQUIRE(params != nullptr, BCV_EINVAL, "NULL argument");
        on_device(mlp->device, [&] { bcv::mlp_set_params(*mlp, params); });
    });
}

bcv_status bcv_mlp_forward(bcv_mlp mlp, int64_t n, const float *X, float *Y)
{
    return guard([&] {
        check_mlp(mlp);
        BCV_REQUIRE(n >= 0 && (n == 0 || (X != nullptr && Y != nullptr)), BCV_EINVAL, "bad arguments");
        on_device(mlp->device, [&] { bcv::mlp_forward_host(*mlp, n, X, Y); });
    });
}

bcv_status bcv_mlp_forward_noalloc(bcv_mlp mlp, int64_t n, const float *X_dev, float *Y_dev, void *hip_stream)
{
    return guard([&] {
        check_mlp(mlp);
        BCV_REQUIRE(n >= 0 && (n == 0 || (X_dev != nullptr && Y_dev != nullptr)), BCV_EINVAL, "bad arguments");
        on_device(mlp->device, [&] { bcv::mlp_forward_noalloc(*mlp, n, X_dev, Y_dev, (hipStream_t)hip_stream); });
    });
}

bcv_status bcv_mlp_loss_grad(bcv_mlp mlp, int64_t n, const float *X, const float *r, double *loss, float *grad)
{
    return guard([&] {
        check_mlp(mlp);
        BCV_REQUIRE(n >= 1 && X && r && loss && grad, BCV_EINVAL, "bad arguments");
        on_device(mlp->device, [&] { *loss = bcv::mlp_loss_grad_host(*mlp, n, X, r, grad); });
    });
}

bcv_status bcv_mlp_train(bcv_mlp mlp, const bcv_mlp_train_opts *opts, bcv_mlp_train_report *report)
{
    return guard([&] {
        check_mlp(mlp);
        BCV_REQUIRE(opts != nullptr, BCV_EINVAL, "NULL argument");
        on_device(mlp->device, [&] { bcv::mlp_train(*mlp, *opts, report); });
    });
}

bcv_status bcv_surrogate_eval(bcv_mlp mlp, int64_t n, const bcv_touch_pair *pairs, double tol, double *value,
                              double *est_err, int32_t *fallback, int64_t *n_fallback)
{
    return guard([&] {
        check_mlp(mlp);
        BCV_REQUIRE(n >= 0 && (n == 0 || (pairs && value && est_err && fallback)), BCV_EINVAL, "bad arguments");
        on_device(mlp->device, [&] { bcv::surrogate_eval(*mlp, n, pairs, tol, value, est_err, fallback, n_fallback); });
    });
}

bcv_status bcv_mlp_save(bcv_mlp mlp, const char *path)
{
    return guard([&] {
        check_mlp(mlp);
        BCV_REQUIRE(path != nullptr, BCV_EINVAL, "NULL argument");
        on_device(mlp->device, [&] { bcv::mlp_save(*mlp, path); });
    });
}

bcv_status bcv_mlp_load(const char *path, int device, bcv_mlp *out)
{
    return guard([&] {
        BCV_REQUIRE(path != nullptr && out != nullptr, BCV_EINVAL, "NULL argument");
        *out = nullptr;
        check_device(device);
        on_device(device, [&] { *out = bcv::mlp_load(path, device); });
    });
}

bcv_status bcv_vtv_graph_create(bcv_plan plan, const double *f_dev, double *u_dev, bcv_graph *out)
{
    return guard([&] {
        check_plan(plan);
        BCV_REQUIRE(f_dev != nullptr && u_dev != nullptr && out != nullptr, BCV_EINVAL, "NULL argument");
        *out = nullptr;
        on_device(plan->device, [&] { *out = bcv::graph_create(*plan, f_dev, u_dev); });
    });
}

bcv_status bcv_graph_launch(bcv_graph graph, void *hip_stream)
{
    return guard([&] {
        BCV_REQUIRE(graph != nullptr, BCV_EINVAL, "graph handle is NULL");
        BCV_REQUIRE(graph->magic == bcv_graph_s::kMagic, BCV_ESTATE, "not a live bcv_graph");
        on_device(graph->device, [&] { bcv::graph_launch(*graph, static_cast<hipStream_t>(hip_stream)); });
    });
}

void bcv_graph_destroy(bcv_graph graph)
{
    if (graph && graph->magic == bcv_graph_s::kMagic) bcv::graph_destroy(graph);
}

bcv_status bcv_autotune(bcv_tree tree, const bcv_plan_opts *base, int device, int n_applies, bcv_plan_opts *best,
                        double *best_ms)
{
    return guard([&] {
        check_tree(tree);
        BCV_REQUIRE(base != nullptr && best != nullptr && best_ms != nullptr, BCV_EINVAL, "NULL argument");
        check_plan_opts(*base, device);
        on_device(device, [&] { *best_ms = bcv::autotune(*tree, *base, device, n_applies, *best); });
    });
}

const char *bcv_last_error(void) { return g_error.c_str(); }

}  // extern "C"
