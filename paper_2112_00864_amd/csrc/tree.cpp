// BC octree of a cube (Sec. 2, Boundary Concentrated Mesh, with cube cells).
//
// In reference coordinates level 0 is [0,1]^3 and a level-l cell (i, j, k) is the cube
// [i, i+1] x [j, j+1] x [k, k+1] times 2^-l; the physical domain is lo + side [0,1]^3 (mesh_lo,
// mesh_side), and every operator follows from the reference one by the scalings stated in bcv.h.
// For l < L the marked cells M_l are, by marking rule,
//   0: the cells with a face on the boundary (B_l);
//   1: the cells with a boundary cell among their neighbours, N(w) meeting B_l (the rule of Sec. 2);
// the leaves of level l are L_l = C_l minus M_l; C_{l+1} consists of the children of M_l; every
// level-L cell is a leaf.
#include <algorithm>
#include <numeric>

#include "internal.hpp"

namespace bcv {

// Cells between the cell and the nearest boundary plane, along the axis where it is closest (0
// for a boundary cell).
static int32_t boundary_distance(int lev, int32_t i, int32_t j, int32_t k)
{
    const int32_t top = (1 << lev) - 1;
    return std::min({i, j, k, top - i, top - j, top - k});
}

// Marking rule 1: does N(w) contain a boundary cell? Every boundary cell of level l exists (its
// ancestors are boundary cells, which both rules refine). A boundary cell at integer offset o is a
// neighbour iff |o|^2 < 12 (eq. def:neighbors with eta0 = 1/2 and rho = a sqrt(3)/2). A boundary
// cell has a coordinate on a boundary plane, so its offset along that axis is at least d (the
// distance above) and |o| >= d; the boundary cell straight across the closest plane has |o| = d.
// So the test is d^2 < 12, i.e. d <= 3.
static bool near_boundary(int lev, int32_t i, int32_t j, int32_t k)
{
    const int32_t d = boundary_distance(lev, i, j, k);
    return d * d < 12;
}

// A forest of n unit-cube BC meshes with finest levels L[m]: mesh m occupies [4m, 4m + 1) x [0, 1)^2
// (in units of a level-0 cell), so cells of different meshes are never neighbours at any level
// (their integer offsets are at least 4 * 2^l - 2^l > sqrt(12) apart at level l) and the planner
// treats the forest as one mesh. With n = 1 this is the single mesh of the unit cube.
// lo (3 per mesh) and side (1 per mesh) place each mesh's cube in physical space; NULL: unit cubes.
bcv_tree_s *build_forest(int n, const int *Ls, const int *markings, const double *lo, const double *side,
                         const int *geoms)
{
    auto *t = new bcv_tree_s;
    t->L = 0;
    for (int m = 0; m < n; ++m) t->L = std::max(t->L, Ls[m]);
    t->n_meshes = n;
    t->mesh_L.assign(Ls, Ls + n);
    t->mesh_lo.assign(3 * (size_t)n, 0.0);
    t->mesh_side.assign(n, 1.0);
    if (lo) std::copy(lo, lo + 3 * n, t->mesh_lo.begin());
    if (side) std::copy(side, side + n, t->mesh_side.begin());
    t->mesh_geom.assign(n, 0);
    if (geoms)
        for (int m = 0; m < n; ++m) t->mesh_geom[m] = (int8_t)geoms[m];
    auto push = [&](int32_t i, int32_t j, int32_t k, int lev, int32_t par) {
        t->ijk.push_back(i);
        t->ijk.push_back(j);
        t->ijk.push_back(k);
        t->level.push_back((int8_t)lev);
        t->refined.push_back(0);
        t->parent.push_back(par);
        t->first_child.push_back(-1);
        t->leaf_of_cell.push_back(-1);
    };
    for (int m = 0; m < n; ++m) push(4 * m, 0, 0, 0, -1);
    t->lvl_start.push_back(0);
    for (int lev = 0; lev <= t->L; ++lev) {
        const int32_t b = t->lvl_start[lev], e = (int32_t)t->level.size();
        t->lvl_start.push_back(e);  // start of level lev + 1 (children appended below)
        if (lev == t->L) break;
        for (int32_t c = b; c < e; ++c) {
            const int32_t i = t->ijk[3 * c], j = t->ijk[3 * c + 1], k = t->ijk[3 * c + 2];
            const int m = (i >> lev) / 4;
            const int32_t il = i - ((4 * m) << lev);  // coordinates within mesh m
            const bool mark = markings[m] ? near_boundary(lev, il, j, k) : boundary_distance(lev, il, j, k) == 0;
            if (lev >= Ls[m] || !mark) continue;
            t->refined[c] = 1;
            t->first_child[c] = (int32_t)t->level.size();
            for (int ch = 0; ch < 8; ++ch)
                push(2 * i + (ch & 1), 2 * j + ((ch >> 1) & 1), 2 * k + ((ch >> 2) & 1), lev + 1, c);
        }
    }
    // lvl_start now has L + 2 entries: level l occupies [lvl_start[l], lvl_start[l + 1]).
    std::vector<int32_t> leaves;
    for (int32_t c = 0; c < (int32_t)t->level.size(); ++c)
        if (!t->refined[c]) leaves.push_back(c);
    int bits = t->L;  // enough bits for every coordinate at level-L resolution
    while ((int64_t(4 * (n - 1) + 1) << t->L) > (int64_t(1) << bits)) ++bits;
    std::vector<uint64_t> key(t->level.size());
    for (int32_t c : leaves) {
        const int sh = t->L - t->level[c];
        key[c] = morton3((uint32_t)t->ijk[3 * c] << sh, (uint32_t)t->ijk[3 * c + 1] << sh,
                         (uint32_t)t->ijk[3 * c + 2] << sh, bits);
    }
    std::sort(leaves.begin(), leaves.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    t->leaf_cell = leaves;
    for (size_t q = 0; q < leaves.size(); ++q) t->leaf_of_cell[leaves[q]] = (int32_t)q;
    return t;
}

bcv_tree_s *build_tree(int L, int marking) { return build_forest(1, &L, &marking, nullptr, nullptr, nullptr); }

// Boundary faces of the unit cube: the faces of level-L leaves in the planes x, y, z = 0 or 1
// (a cell meeting the boundary has a face on it and is refined down to level L).
std::vector<int32_t> tree_faces(const bcv_tree_s &t)
{
    BCV_REQUIRE(t.n_meshes == 1, BCV_ENOTSUP, "boundary faces: single-mesh trees only");
    const int32_t top = (1 << t.L) - 1;
    std::vector<int32_t> out;
    for (int64_t q = 0; q < t.n_leaves(); ++q) {
        const int32_t c = t.leaf_cell[q];
        if (t.level[c] != t.L) continue;
        for (int ax = 0; ax < 3; ++ax) {
            const int32_t v = t.ijk[3 * c + ax];
            for (int side = 0; side < 2; ++side)
                if (v == (side ? top : 0)) {
                    out.push_back((int32_t)q);
                    out.push_back(ax);
                    out.push_back(side);
                }
        }
    }
    return out;
}

}  // namespace bcv
