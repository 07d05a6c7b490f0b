// Interaction plan of the BC-FMM (Sec. 3 of the paper), built on the host and uploaded once.
//
//  * Neighbours N(w) (eq. def:neighbors): same-level cubes at integer offset o with
//    eta = sqrt(3)/|o| > eta0 = 1/2, i.e. |o|^2 < 12 (rho = a sqrt(3)/2 from eq. def:diam).
//  * Interaction lists I(w): children of the parent's neighbours that are not neighbours of w.
//  * Near field of a leaf w: N*(w) = N_M(w) plus N_L(pi_l(w)) for every ancestor level l
//    (Sec. 3, before Lemma 1); a marked cell of N_M(w) stands for all of its leaves. The
//    decomposition eq. spaceDecomp:OmOm then covers every ordered leaf pair exactly once.
//  * Near pairs whose closed cubes touch get one of seven singular classes; all others use the
//    2x2x2 point rule on both cells.
//  * M2L work is packed into 64-lane tasks: 64 targets of one level sharing their position in
//    the parent, so that each interaction offset of the union of their lists is valid for every
//    lane that has a source there; the lanes of a slot share the offset (one derivative table)
//    and each lane reads its own source moments.
#include <omp.h>

#include <algorithm>
#include <array>
#include <unordered_map>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "ballmap.hpp"
#include "internal.hpp"
#include "kernels.hpp"
#include "multiindex.hpp"

namespace bcv {

void derivative_table(int q, const int o[3], double *out);
void touching_integrals(int device, double out[kTouchClasses]);

namespace {

struct Grid {  // dense (i, j, k) -> cell index of one level, over the bounding box of its cells
    int nx = 0, ny = 0, nz = 0;
    std::vector<int32_t> idx;
    int32_t at(int i, int j, int k) const
    {
        if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz) return -1;
        return idx[((size_t)k * ny + j) * nx + i];
    }
};

std::vector<Grid> make_grids(const bcv_tree_s &t)
{
    std::vector<Grid> g(t.L + 1);
    for (int lev = 0; lev <= t.L; ++lev) {
        Grid &G = g[lev];
        for (int32_t c = t.lvl_start[lev]; c < t.lvl_start[lev + 1]; ++c) {
            G.nx = std::max(G.nx, t.ijk[3 * c] + 1);
            G.ny = std::max(G.ny, t.ijk[3 * c + 1] + 1);
            G.nz = std::max(G.nz, t.ijk[3 * c + 2] + 1);
        }
        G.idx.assign((size_t)G.nx * G.ny * G.nz, -1);
        for (int32_t c = t.lvl_start[lev]; c < t.lvl_start[lev + 1]; ++c)
            G.idx[((size_t)t.ijk[3 * c + 2] * G.ny + t.ijk[3 * c + 1]) * G.nx + t.ijk[3 * c]] = c;
    }
    return g;
}

bool is_neighbour_offset(int a, int b, int c) { return a * a + b * b + c * c < 12; }

const std::vector<std::array<int, 3>> &stencil()
{
    static const std::vector<std::array<int, 3>> s = [] {
        std::vector<std::array<int, 3>> v;
        for (int c = -3; c <= 3; ++c)
            for (int b = -3; b <= 3; ++b)
                for (int a = -3; a <= 3; ++a)
                    if (is_neighbour_offset(a, b, c)) v.push_back({a, b, c});
        return v;
    }();
    return s;
}

constexpr uint32_t kBadTouch = 0xFFu;

// Touch code of two cubes given at level-L resolution: 0 if the closed cubes are disjoint, else
// 1 + class (0 self, 1 face, 2 edge, 3 vertex with equal sides; 4 face, 5 edge, 6 vertex with
// sides 1:2). The mesh is 2:1 balanced, so any other touching pair (kBadTouch) is an internal error.
uint32_t touch_code(const int64_t lo_a[3], int64_t sa, const int64_t lo_b[3], int64_t sb)
{
    int contacts = 0;
    for (int ax = 0; ax < 3; ++ax) {
        const int64_t lo = std::max(lo_a[ax], lo_b[ax]);
        const int64_t hi = std::min(lo_a[ax] + sa, lo_b[ax] + sb);
        if (lo > hi) return 0;
        if (lo == hi) ++contacts;
    }
    if (sa == sb) return 1u + (uint32_t)contacts;
    if (std::max(sa, sb) != 2 * std::min(sa, sb) || contacts == 0) return kBadTouch;
    return 4u + (uint32_t)contacts;
}

struct LeafGeo {
    std::vector<int64_t> lo;  // 3 per leaf, level-L resolution
    std::vector<int64_t> size;
};

LeafGeo leaf_geometry(const bcv_tree_s &t)
{
    LeafGeo g;
    const int64_t n = t.n_leaves();
    g.lo.resize(3 * n);
    g.size.resize(n);
    for (int64_t l = 0; l < n; ++l) {
        const int32_t c = t.leaf_cell[l];
        const int s = t.L - t.level[c];
        for (int ax = 0; ax < 3; ++ax) g.lo[3 * l + ax] = (int64_t)t.ijk[3 * c + ax] << s;
        g.size[l] = (int64_t)1 << s;
    }
    return g;
}

// Leaves y with (w, y) in w x N*(w) for the leaf cell w (marked sources expanded to leaves).
void near_sources(const bcv_tree_s &t, const std::vector<Grid> &g, int32_t cell, std::vector<int32_t> &out,
                  std::vector<int32_t> &stack)
{
    out.clear();
    const int lev = t.level[cell];
    const int i = t.ijk[3 * cell], j = t.ijk[3 * cell + 1], k = t.ijk[3 * cell + 2];
    for (const auto &o : stencil()) {  // N(w) = N_L(w) + N_M(w)
        const int32_t s = g[lev].at(i + o[0], j + o[1], k + o[2]);
        if (s < 0) continue;
        if (!t.refined[s]) {
            out.push_back(t.leaf_of_cell[s]);
            continue;
        }
        stack.assign(1, s);  // all leaves below a marked neighbour
        while (!stack.empty()) {
            const int32_t c = stack.back();
            stack.pop_back();
            if (!t.refined[c]) {
                out.push_back(t.leaf_of_cell[c]);
            } else {
                for (int ch = 7; ch >= 0; --ch) stack.push_back(t.first_child[c] + ch);
            }
        }
    }
    for (int lp = lev - 1; lp >= 0; --lp) {  // N_L of every proper ancestor
        const int sh = lev - lp;
        const int ai = i >> sh, aj = j >> sh, ak = k >> sh;
        for (const auto &o : stencil()) {
            const int32_t s = g[lp].at(ai + o[0], aj + o[1], ak + o[2]);
            if (s >= 0 && !t.refined[s]) out.push_back(t.leaf_of_cell[s]);
        }
    }
}

struct NearCSR {
    std::vector<int64_t> row;
    std::vector<int64_t> split;  // first non-touching entry of each row
    std::vector<uint32_t> col;
    int64_t n_touch = 0;
};

NearCSR build_near(const bcv_tree_s &t, const std::vector<Grid> &g, const LeafGeo &geo, bool direct)
{
    const int64_t nl = t.n_leaves();
    NearCSR r;
    r.row.assign(nl + 1, 0);
    auto gen = [&](int64_t n, std::vector<int32_t> &src, std::vector<int32_t> &stack) {
        if (direct) {
            src.resize(nl);
            for (int64_t s = 0; s < nl; ++s) src[s] = (int32_t)s;
        } else {
            near_sources(t, g, t.leaf_cell[n], src, stack);
        }
    };
#pragma omp parallel
    {
        std::vector<int32_t> src, stack;
#pragma omp for schedule(dynamic, 256)
        for (int64_t n = 0; n < nl; ++n) {
            gen(n, src, stack);
            r.row[n + 1] = (int64_t)src.size();
        }
    }
    for (int64_t n = 0; n < nl; ++n) r.row[n + 1] += r.row[n];
    r.col.resize(r.row[nl]);
    r.split.assign(nl, 0);
    int64_t touch = 0, bad = 0;
#pragma omp parallel reduction(+ : touch, bad)
    {
        std::vector<int32_t> src, stack;
        std::vector<uint32_t> codes;
#pragma omp for schedule(dynamic, 256)
        for (int64_t n = 0; n < nl; ++n) {
            gen(n, src, stack);
            codes.resize(src.size());
            for (size_t e = 0; e < src.size(); ++e) {
                const int32_t s = src[e];
                uint32_t tc = touch_code(&geo.lo[3 * n], geo.size[n], &geo.lo[3 * s], geo.size[s]);
                bad += tc == kBadTouch;
                touch += tc != 0;
                if (tc != 0 && tc != kBadTouch && geo.size[s] < geo.size[n]) tc |= 8u;  // the source is the smaller cube
                codes[e] = (uint32_t)s | ((tc & 15u) << 28);
            }
            // touching pairs first (they are cheap), then by source leaf
            std::sort(codes.begin(), codes.end(), [](uint32_t a, uint32_t b) {
                const bool ta = (a >> 28) != 0, tb = (b >> 28) != 0;
                if (ta != tb) return ta;
                return (a & 0x0FFFFFFFu) < (b & 0x0FFFFFFFu);
            });
            std::copy(codes.begin(), codes.end(), r.col.begin() + r.row[n]);
            int64_t n_t = 0;
            while (n_t < (int64_t)codes.size() && (codes[n_t] >> 28) != 0) ++n_t;
            r.split[n] = r.row[n] + n_t;
        }
    }
    if (bad) fail(BCV_ESTATE, "internal: touching leaves violate 2:1 balance");
    r.n_touch = touch;
    return r;
}

// Near-field work units of at most `unit` entries (by default a whole row up to 2048 entries per
// wave: at h = 1/256 a two-stream mixed apply took 5.42 ms with 2048 or 4096, 5.45 with 1024, 5.52
// with 512 and 5.91 with 256). A row is cut into equal pieces; units are ordered longest first so
// that the long units start early.
constexpr int kDefaultNearUnit = 2048;

struct NearUnits {
    std::vector<NearUnit> units;
    std::vector<NearSplit> splits;
    int64_t n_partial = 0;
    int32_t xcd_begin[kXcds + 1] = {};  // with xcd ranges: the units of XCD x are [xcd_begin[x], xcd_begin[x + 1])
};

// xcd: the units are grouped in kXcds contiguous target ranges (leaf order, so spatially compact)
// of about equal entry counts, one per XCD, so that each XCD's L2 holds the densities of its own
// region; within a range the longest units come first. Otherwise all units are longest first.
NearUnits build_near_units(const NearCSR &near, int64_t n_leaves, int64_t unit, bool xcd = false)
{
    NearUnits r;
    for (int64_t t = 0; t < n_leaves; ++t) {
        const int64_t b = near.row[t], len = near.row[t + 1] - b;
        const int64_t pieces = std::max<int64_t>(1, (len + unit - 1) / unit);
        if (pieces == 1) {
            r.units.push_back(NearUnit{b, b + len, (int32_t)t, -1});
            continue;
        }
        BCV_REQUIRE(r.n_partial + pieces < INT32_MAX, BCV_ENOTSUP, "near field too large");
        r.splits.push_back(NearSplit{(int32_t)t, (int32_t)r.n_partial, (int32_t)pieces, 0});
        for (int64_t k = 0; k < pieces; ++k)
            r.units.push_back(NearUnit{b + len * k / pieces, b + len * (k + 1) / pieces, (int32_t)t,
                                       (int32_t)(r.n_partial + k)});
        r.n_partial += pieces;
    }
    const auto longer = [](const NearUnit &x, const NearUnit &y) { return x.end - x.begin > y.end - y.begin; };
    if (xcd) {
        // units are in target order here; cut them at equal shares of the entries
        const int64_t total = near.row[n_leaves];
        int64_t acc = 0;
        int x = 0;
        r.xcd_begin[0] = 0;
        for (size_t k = 0; k < r.units.size(); ++k) {
            while (x < kXcds - 1 && acc >= total * (x + 1) / kXcds) r.xcd_begin[++x] = (int32_t)k;
            acc += r.units[k].end - r.units[k].begin;
        }
        while (x < kXcds) r.xcd_begin[++x] = (int32_t)r.units.size();
        BCV_REQUIRE(r.units.size() < (size_t)INT32_MAX, BCV_ENOTSUP, "near field too large");
        for (int y = 0; y < kXcds; ++y)
            std::stable_sort(r.units.begin() + r.xcd_begin[y], r.units.begin() + r.xcd_begin[y + 1], longer);
    } else {
        std::stable_sort(r.units.begin(), r.units.end(), longer);
    }
    // every entry of every row is covered by exactly one unit
    std::vector<int64_t> covered(n_leaves, 0);
    for (const NearUnit &u : r.units) {
        BCV_REQUIRE(u.target >= 0 && u.target < n_leaves && u.begin >= near.row[u.target] &&
                        u.end <= near.row[u.target + 1] && u.begin <= u.end && u.out < r.n_partial,
                    BCV_ESTATE, "internal: near unit out of range");
        covered[u.target] += u.end - u.begin;
    }
    for (int64_t t = 0; t < n_leaves; ++t)
        BCV_REQUIRE(covered[t] == near.row[t + 1] - near.row[t], BCV_ESTATE, "internal: near units do not tile a row");
    return r;
}

struct M2LPlan {
    std::vector<M2LTask> tasks;
    std::vector<int32_t> targets;   // 64 per task
    std::vector<int32_t> slot_key;  // offset key per slot | gather bit 31, later the offset id | bit 31
    // 64 per slot: source row | (offset in the lane's own list) << 31 (not zero-filled: every word
    // is written by the builder, each task's block by one thread)
    std::unique_ptr<uint32_t[]> slot_src;
    std::vector<M2LSplit> splits;
    int32_t n_pieces = 0;           // partial blocks of split tasks
    int32_t xcd_begin[kXcds + 1] = {};
    int32_t level_xcd[kMaxLevel + 1][kXcds + 1] = {};  // per_level: the XCD ranges of each level's tasks
    int64_t n_pairs = 0;
    int64_t n_read_lanes = 0;       // lanes that read their source row in a lane-shifting kernel
};

// Default longest slot list of one interaction task: longer lists (the remainder tasks, whose
// lanes belong to many signature classes) are cut into pieces so that no wave outlasts the others.
// Most tasks of a face-marked mesh hold 224-287 slots; at 320 those stay whole (measured 3.5% faster
// than 256 at h = 1/128 and 1/256; shorter pieces add partial sums and gathering first slots). With
// level-dependent orders each level is its own launch, and 256 measured faster (4% in FP64); so
// did small meshes, whose few tasks need the shorter pieces to fill the GPU.
constexpr int kDefaultMaxSlots = 320;
constexpr int kDefaultMaxSlotsSchedule = 256;

int offset_key(int a, int b, int c) { return ((a + 7) * 15 + (b + 7)) * 15 + (c + 7); }

// Sorted interaction-offset keys of cell c at level lev (its I list, eq. after spaceDecomp:Om);
// with source_ok, only the sources s with source_ok[s] (the BtV interaction sources I(w) ∩ B_l).
void interaction_keys(const bcv_tree_s &t, const std::vector<Grid> &g, int lev, int32_t c, std::vector<int32_t> &keys,
                      const uint8_t *source_ok = nullptr)
{
    keys.clear();
    const int i = t.ijk[3 * c], j = t.ijk[3 * c + 1], k = t.ijk[3 * c + 2];
    for (const auto &o : stencil()) {
        const int32_t pn = g[lev - 1].at((i >> 1) + o[0], (j >> 1) + o[1], (k >> 1) + o[2]);
        if (pn < 0 || !t.refined[pn]) continue;  // only marked parent-neighbours have children
        for (int d = 0; d < 8; ++d) {
            const int32_t s = t.first_child[pn] + d;
            if (source_ok && !source_ok[s]) continue;
            const int a = i - t.ijk[3 * s], b = j - t.ijk[3 * s + 1], cc = k - t.ijk[3 * s + 2];
            if (!is_neighbour_offset(a, b, cc)) keys.push_back(offset_key(a, b, cc));
        }
    }
    std::sort(keys.begin(), keys.end());
}

uint64_t hash_keys(const std::vector<int32_t> &keys)
{
    uint64_t h = 1469598103934665603ull;
    for (int32_t k : keys) h = (h ^ (uint64_t)(uint32_t)k) * 1099511628211ull;
    return h ^ keys.size();
}

// Packs the interaction phase into 64-lane tasks. Targets of one level are grouped by the
// signature of their interaction list (cells in the interior of a face share it, cells along an
// edge share it with the other cells at the same distance from the edge): each signature class
// fills whole 64-lane tasks, and the remainders are packed together in Morton order. Members of a class share their child position, so along a row of the mesh
// they are two cells apart; a class is laid out row by row along the axis where it has the most
// such pairs (lane l + 1 two cells after lane l except where a row ends: the task's "heads"). A
// task's slots are the union of its targets' offsets o = t - s, sorted so that consecutive slots
// step o by two cells along that axis. Then the source of a non-head lane at a slot is the
// previous slot's source of the lane before it, and the interaction kernel can shift registers
// across lanes instead of gathering again; the plan checks this for every slot and lane, and marks
// the slots where it fails (and the first one) as gathering. Every slot records the source row of
// every lane (the zero row where there is no cell) and, in bit 31, whether the offset is in that
// lane's own list.
// max_slots: the longest slot list of a task piece, per level. per_level: each level's tasks get XCD
// ranges of their own (the levels are launched one by one, at their own expansion orders).
// small_slots > 0: the limit for phases of fewer than 2^20 slots (about 256 per wave slot of the
// GPU), where shorter pieces give more waves.
// source_ok: only these sources enter the lists (the BtV plan: boundary cells); target_ok: only
// these cells are targets (the VtB plan: boundary cells, whose local coefficients the faces need).
M2LPlan build_m2l(const bcv_tree_s &t, const std::vector<Grid> &g, const std::vector<int32_t> &max_slots,
                  bool per_level = false, int32_t small_slots = 0, const uint8_t *source_ok = nullptr,
                  const uint8_t *target_ok = nullptr, bool merge = true)
{
    M2LPlan m;
    const int32_t zero_row = (int32_t)t.n_cells();
    BCV_REQUIRE(zero_row < (1 << 30), BCV_ENOTSUP, "more than 2^30 cells");
    struct Chunk {
        int lev;
        int axis;  // rows of the task run along this axis
        int step;  // consecutive lanes of a row are this many cells apart (1 or 2)
        std::vector<int32_t> cells;
    };
    std::vector<Chunk> chunks;
    for (int lev = t.L; lev >= 2; --lev) {
        const int32_t b = t.lvl_start[lev], n = t.lvl_start[lev + 1] - b;
        std::vector<uint64_t> sig(n);
        std::vector<char> is_t(n, 1);
        if (target_ok)
            for (int32_t q = 0; q < n; ++q) is_t[q] = target_ok[b + q] != 0;
#pragma omp parallel
        {
            std::vector<int32_t> keys;
#pragma omp for schedule(dynamic, 256)
            for (int32_t q = 0; q < n; ++q) {
                interaction_keys(t, g, lev, b + q, keys, source_ok);
                sig[q] = hash_keys(keys);
            }
        }
        // classes in order of their first (Morton-smallest) member
        std::vector<int32_t> order;
        for (int32_t q = 0; q < n; ++q)
            if (is_t[q]) order.push_back(q);
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return sig[x] < sig[y]; });
        const int32_t nt = (int32_t)order.size();
        struct Class {
            int32_t s0, s1;  // range in order
            int axis;
        };
        std::vector<Class> classes;
        std::unordered_map<uint64_t, int32_t> class_of_sig;
        for (int32_t s0 = 0; s0 < nt;) {
            int32_t s1 = s0;
            while (s1 < nt && sig[order[s1]] == sig[order[s0]]) ++s1;
            // the class in rows along the axis with the most member pairs two cells apart (x first on
            // ties); a class may span several separate patches of the level
            int axis = 0;
            int64_t pairs[3] = {0, 0, 0};
            for (int32_t r = s0; r < s1; ++r) {
                const int32_t *c = &t.ijk[3 * (b + order[r])];
                for (int ax = 0; ax < 3; ++ax) {
                    const int32_t nb = g[lev].at(c[0] + 2 * (ax == 0), c[1] + 2 * (ax == 1), c[2] + 2 * (ax == 2));
                    pairs[ax] += nb >= 0 && is_t[nb - b] && sig[nb - b] == sig[order[s0]];
                }
            }
            for (int ax = 1; ax < 3; ++ax)
                if (pairs[ax] > pairs[axis]) axis = ax;
            class_of_sig[sig[order[s0]]] = (int32_t)classes.size();
            classes.push_back(Class{s0, s1, axis});
            s0 = s1;
        }
        // merge: a class of at least 64 cells whose members' neighbours one cell further along its
        // axis form one other class of the same size and axis (the cells of the other child
        // position, e.g. in the interior of a face) is merged with it: rows then step by one cell,
        // so runs of offsets are twice as long and rows twice as dense (fewer row reads), for a
        // larger union of lists (more masked lanes). FP64 plans merge (their rows cost twice the
        // bytes), and so do the matrix-core plans (6.15 against 6.28 ms per apply); FP32 lane-shift
        // plans do not (h = 1/256: FP32 interaction phase 4.01 ms unmerged against 4.41 merged, apply
        // 5.21 against 5.44 ms; FP64 7.15 against 7.56 ms per apply the other way).
        std::vector<int32_t> partner(classes.size(), -1);
        auto class_of = [&](int32_t cell) -> int32_t {
            const int32_t *c = &t.ijk[3 * cell];
            (void)c;
            return class_of_sig.at(sig[cell - b]);
        };
        for (size_t k = 0; k < classes.size(); ++k) {
            const Class &C = classes[k];
            if (!merge || C.s1 - C.s0 < 64 || partner[k] >= 0) continue;
            const int ax = C.axis;
            int32_t cand = -1;
            bool ok = true;
            for (int32_t r = C.s0; r < C.s1 && ok; ++r) {
                const int32_t *c = &t.ijk[3 * (b + order[r])];
                const int32_t nb = g[lev].at(c[0] + (ax == 0), c[1] + (ax == 1), c[2] + (ax == 2));
                if (nb < 0) continue;
                if (!is_t[nb - b]) {
                    ok = false;
                    break;
                }
                const int32_t pc = class_of(nb);
                if (cand < 0) cand = pc;
                ok = pc == cand;
            }
            if (!ok || cand < 0 || cand == (int32_t)k || partner[cand] >= 0) continue;
            const Class &P = classes[cand];
            if (P.axis != ax || P.s1 - P.s0 != C.s1 - C.s0) continue;
            partner[k] = cand;
            partner[cand] = (int32_t)k;
        }
        std::vector<Chunk> level_chunks;
        std::vector<Chunk> remainders;
        for (size_t k = 0; k < classes.size(); ++k) {
            if (partner[k] >= 0 && partner[k] < (int32_t)k) continue;  // merged into its partner's rows
            const Class &C = classes[k];
            const int axis = C.axis, step = partner[k] >= 0 ? 1 : 2;
            std::vector<int32_t> cells;
            for (int32_t r = C.s0; r < C.s1; ++r) cells.push_back(b + order[r]);
            if (partner[k] >= 0)
                for (int32_t r = classes[partner[k]].s0; r < classes[partner[k]].s1; ++r) cells.push_back(b + order[r]);
            const int u = axis == 0 ? 2 : (axis == 1 ? 2 : 1), v = axis == 0 ? 1 : 0;
            std::sort(cells.begin(), cells.end(), [&](int32_t x, int32_t y) {
                const int32_t *a = &t.ijk[3 * x], *c = &t.ijk[3 * y];
                if (a[u] != c[u]) return a[u] < c[u];
                if (a[v] != c[v]) return a[v] < c[v];
                return a[axis] < c[axis];
            });
            size_t q = 0;
            for (; q + 64 <= cells.size(); q += 64)
                level_chunks.push_back(Chunk{lev, axis, step, std::vector<int32_t>(cells.begin() + q, cells.begin() + q + 64)});
            if (q < cells.size())
                remainders.push_back(Chunk{lev, axis, step, std::vector<int32_t>(cells.begin() + q, cells.end())});
        }
        // the remainders (most are whole classes: the rows of cells along the edges of the domain,
        // single cells near its corners and on the coarse levels) share tasks with remainders of
        // the same row axis, in Morton order, which keeps similar lists together (a first fit by
        // decreasing size that minimised the added offsets saved under 1% of the slots)
        std::sort(remainders.begin(), remainders.end(), [](const Chunk &x, const Chunk &y) {
            if (x.step != y.step) return x.step < y.step;
            return x.axis != y.axis ? x.axis < y.axis : x.cells[0] < y.cells[0];
        });
        Chunk cur{lev, 0, 2, {}};
        for (auto &rem : remainders) {
            if (!cur.cells.empty() &&
                (cur.axis != rem.axis || cur.step != rem.step || cur.cells.size() + rem.cells.size() > 64)) {
                level_chunks.push_back(std::move(cur));
                cur = Chunk{lev, rem.axis, rem.step, {}};
            }
            cur.axis = rem.axis;
            cur.step = rem.step;
            cur.cells.insert(cur.cells.end(), rem.cells.begin(), rem.cells.end());
        }
        if (!cur.cells.empty()) level_chunks.push_back(std::move(cur));
        // spatial order of tasks within the level (Morton order of the first target)
        std::sort(level_chunks.begin(), level_chunks.end(),
                  [](const Chunk &x, const Chunk &y) { return x.cells[0] < y.cells[0]; });
        for (auto &ch : level_chunks) chunks.push_back(std::move(ch));
    }
    // Pass 1: each task's slots (the union of its targets' offsets, in slot order) and heads.
    struct Out {
        std::vector<int32_t> keys;  // offset key per slot | (the slot gathers) << 31
        uint64_t heads = 0;
        int64_t pairs = 0;
    };
    std::vector<Out> outs(chunks.size());
#pragma omp parallel
    {
        std::vector<int32_t> keys;
        std::vector<char> used(15 * 15 * 15);
        std::vector<std::array<int, 5>> order;  // across 1, across 2, along parity, along, key
#pragma omp for schedule(dynamic, 4)
        for (size_t q = 0; q < chunks.size(); ++q) {
            const Chunk &ch = chunks[q];
            const int ax = ch.axis, u = ax == 0 ? 1 : 0, v = ax == 2 ? 1 : 2;
            const int nl = (int)ch.cells.size();
            std::fill(used.begin(), used.end(), 0);
            for (int lane = 0; lane < nl; ++lane) {
                interaction_keys(t, g, ch.lev, ch.cells[lane], keys, source_ok);
                for (int32_t key : keys) used[key] = 1;
            }
            Out &o = outs[q];
            for (int lane = 0; lane < nl; ++lane) {  // heads: the previous lane is not `step` cells back
                bool head = lane == 0;
                if (!head) {
                    const int32_t a = ch.cells[lane - 1], c = ch.cells[lane];
                    for (int k = 0; k < 3; ++k)
                        head = head || t.ijk[3 * c + k] - t.ijk[3 * a + k] != (k == ax ? ch.step : 0);
                }
                if (head) o.heads |= 1ull << lane;
            }
            order.clear();
            for (int key = 0; key < 15 * 15 * 15; ++key) {
                if (!used[key]) continue;
                const int d[3] = {key / 225 - 7, (key / 15) % 15 - 7, key % 15 - 7};
                order.push_back({d[u], d[v], ch.step == 2 ? d[ax] & 1 : 0, d[ax], key});
            }
            std::sort(order.begin(), order.end());
            o.keys.resize(order.size());
            for (size_t k = 0; k < order.size(); ++k) o.keys[k] = order[k][4];
        }
    }
    std::vector<int64_t> chunk_base(chunks.size() + 1, 0);
    for (size_t q = 0; q < chunks.size(); ++q) chunk_base[q + 1] = chunk_base[q] + (int64_t)outs[q].keys.size();
    BCV_REQUIRE(chunk_base.back() < (int64_t)INT32_MAX, BCV_ENOTSUP, "interaction plan too large");
    const int64_t n_slots = chunk_base.back();
    m.slot_key.resize(n_slots);
    m.slot_src.reset(new (std::nothrow) uint32_t[std::max<int64_t>(n_slots, 1) * 64]);
    if (!m.slot_src) fail(BCV_ENOMEM, "host allocation failed for the interaction plan");
    // Pass 2: every lane's source at every slot, written in place (first touch by the filling
    // thread), and the gather bit.
#pragma omp parallel
    {
        std::vector<std::vector<int32_t>> lane_keys(64);
#pragma omp for schedule(dynamic, 4)
        for (size_t q = 0; q < chunks.size(); ++q) {
            const Chunk &ch = chunks[q];
            const int nl = (int)ch.cells.size();
            for (int lane = 0; lane < nl; ++lane)
                interaction_keys(t, g, ch.lev, ch.cells[lane], lane_keys[lane], source_ok);
            Out &o = outs[q];
            uint32_t *src = m.slot_src.get() + chunk_base[q] * 64;
            for (size_t k = 0; k < o.keys.size(); ++k) {
                const int key = o.keys[k];
                const int d[3] = {key / 225 - 7, (key / 15) % 15 - 7, key % 15 - 7};
                uint32_t *at = src + k * 64;
                for (int lane = 0; lane < 64; ++lane) {
                    int32_t s = -1;
                    bool valid = false;
                    if (lane < nl) {
                        const int32_t c = ch.cells[lane];
                        s = g[ch.lev].at(t.ijk[3 * c] - d[0], t.ijk[3 * c + 1] - d[1], t.ijk[3 * c + 2] - d[2]);
                        valid = std::binary_search(lane_keys[lane].begin(), lane_keys[lane].end(), key);
                        if (valid && s < 0) o.pairs = INT64_MIN;  // a listed source must exist
                    }
                    o.pairs += valid;
                    at[lane] = (uint32_t)(s >= 0 ? s : zero_row) | (valid ? 1u << 31 : 0u);
                }
                // the slot can shift if every non-head lane finds its source one lane down
                bool shift = k > 0;
                for (int lane = 1; shift && lane < nl; ++lane)
                    if (!((o.heads >> lane) & 1))
                        shift = (at[lane] & 0x7FFFFFFFu) == (at[lane - 64 - 1] & 0x7FFFFFFFu);
                m.slot_key[chunk_base[q] + k] = shift ? key : (int32_t)((uint32_t)key | (1u << 31));
            }
        }
    }
    for (const Out &o : outs) BCV_REQUIRE(o.pairs >= 0, BCV_ESTATE, "internal: interaction source missing");
    // Pieces of at most max_slots slots, in task order.
    struct Piece {
        M2LTask task;
        int32_t chunk;
    };
    std::vector<Piece> pieces;
    std::vector<M2LSplit> split_of_chunk(chunks.size(), M2LSplit{-1, 0, 0, 0});
    for (size_t q = 0; q < chunks.size(); ++q) {
        const int32_t base = (int32_t)chunk_base[q];
        const int32_t n = (int32_t)(chunk_base[q + 1] - chunk_base[q]);
        const int32_t ms = small_slots > 0 && n_slots < (1 << 20) ? std::min(small_slots, max_slots[chunks[q].lev])
                                                                   : max_slots[chunks[q].lev];
        const int32_t np = std::max<int32_t>(1, (n + ms - 1) / ms);
        if (np > 1) split_of_chunk[q] = M2LSplit{-1, m.n_pieces, np, 0};
        for (int32_t k = 0; k < np; ++k) {
            const int32_t b = base + (int32_t)((int64_t)n * k / np), e = base + (int32_t)((int64_t)n * (k + 1) / np);
            pieces.push_back(
                Piece{M2LTask{b, e - b, chunks[q].lev, np > 1 ? m.n_pieces + k : -1, outs[q].heads}, (int32_t)q});
            if (e > b) m.slot_key[b] = (int32_t)((uint32_t)m.slot_key[b] | (1u << 31));  // a piece starts by gathering
            for (int32_t j = b; j < e; ++j)
                m.n_read_lanes += m.slot_key[j] < 0 ? 64 : __builtin_popcountll(outs[q].heads);
        }
        if (np > 1) m.n_pieces += np;
        m.n_pairs += outs[q].pairs;
    }
    // XCD ranges: contiguous runs of pieces (spatially ordered, so an XCD's L2 sees neighbouring
    // sources) with about equal slot totals; inside a range the longest pieces go first. per_level:
    // each level's pieces (contiguous: the chunks go level by level) get ranges of their own.
    auto deal = [&](size_t pb, size_t pe, int32_t *begin) {
        int64_t total = 0;
        for (size_t i = pb; i < pe; ++i) total += pieces[i].task.n_slots;
        std::vector<size_t> cut(kXcds + 1, pe);
        cut[0] = pb;
        int64_t acc = 0;
        int x = 1;
        for (size_t i = pb; i < pe && x < kXcds; ++i) {
            acc += pieces[i].task.n_slots;
            while (x < kXcds && acc * kXcds >= total * x) cut[x++] = i + 1;
        }
        for (int y = 0; y < kXcds; ++y)
            std::stable_sort(pieces.begin() + cut[y], pieces.begin() + cut[y + 1],
                             [](const Piece &a, const Piece &b) { return a.task.n_slots > b.task.n_slots; });
        for (int y = 0; y <= kXcds; ++y) begin[y] = (int32_t)cut[y];
    };
    if (!per_level) {
        deal(0, pieces.size(), m.xcd_begin);
    } else {
        BCV_REQUIRE(t.L <= kMaxLevel, BCV_ENOTSUP, "too many levels");
        size_t pb = 0;
        for (int lev = t.L; lev >= 0; --lev) {
            size_t pe = pb;
            while (pe < pieces.size() && pieces[pe].task.level == lev) ++pe;
            deal(pb, pe, m.level_xcd[lev]);
            pb = pe;
        }
        BCV_REQUIRE(pb == pieces.size(), BCV_ESTATE, "internal: interaction tasks not grouped by level");
        m.xcd_begin[0] = 0;
        for (int x = 1; x <= kXcds; ++x) m.xcd_begin[x] = (int32_t)pieces.size();
    }
    for (const Piece &pc : pieces) {
        const int32_t ti = (int32_t)m.tasks.size();
        m.tasks.push_back(pc.task);
        const Chunk &ch = chunks[pc.chunk];
        for (int lane = 0; lane < 64; ++lane) m.targets.push_back(lane < (int)ch.cells.size() ? ch.cells[lane] : -1);
        M2LSplit &sp = split_of_chunk[pc.chunk];
        if (pc.task.out == sp.first && sp.count > 1) sp.task = ti;  // the first piece carries the targets
    }
    for (const M2LSplit &sp : split_of_chunk)
        if (sp.count > 1) m.splits.push_back(sp);
    for (const M2LTask &tk : m.tasks)
        BCV_REQUIRE(tk.slot_begin >= 0 && tk.n_slots >= 0 && (size_t)tk.slot_begin + tk.n_slots <= m.slot_key.size() &&
                        tk.out < m.n_pieces,
                    BCV_ESTATE, "internal: interaction task out of range");
    for (const M2LSplit &sp : m.splits)
        BCV_REQUIRE(sp.task >= 0 && sp.task < (int32_t)m.tasks.size() && sp.first >= 0 &&
                        sp.first + sp.count <= m.n_pieces,
                    BCV_ESTATE, "internal: split interaction task out of range");
    BCV_REQUIRE(m.xcd_begin[kXcds] == (int32_t)m.tasks.size(), BCV_ESTATE, "internal: XCD ranges");
    return m;
}

template <class T>
T *upload(bcv_plan_s *p, const std::vector<T> &v)
{
    if (v.empty()) return nullptr;
    T *d = nullptr;
    const size_t bytes = v.size() * sizeof(T);
    if (hipMalloc(&d, bytes) != hipSuccess) fail(BCV_ENOMEM, "hipMalloc failed for a plan buffer");
    p->device_bytes += (int64_t)bytes;
    BCV_HIP(hipMemcpy(d, v.data(), bytes, hipMemcpyHostToDevice));
    return d;
}

template <class T>
T *upload(bcv_plan_s *p, const T *v, size_t count)
{
    if (count == 0) return nullptr;
    T *d = nullptr;
    const size_t bytes = count * sizeof(T);
    if (hipMalloc(&d, bytes) != hipSuccess) fail(BCV_ENOMEM, "hipMalloc failed for a plan buffer");
    p->device_bytes += (int64_t)bytes;
    BCV_HIP(hipMemcpy(d, v, bytes, hipMemcpyHostToDevice));
    return d;
}

template <class T>
T *alloc_zero(bcv_plan_s *p, size_t count)
{
    T *d = nullptr;
    const size_t bytes = count * sizeof(T);
    if (hipMalloc(&d, bytes) != hipSuccess) fail(BCV_ENOMEM, "hipMalloc failed for plan workspace");
    p->device_bytes += (int64_t)bytes;
    BCV_HIP(hipMemset(d, 0, bytes));
    return d;
}

// BtV (Algorithm 3) near field. For a leaf w of level l, the pair (w, face) is near when the
// level-l ancestor of the face's cell is a neighbour of w: then no ancestor pair meets in an
// interaction list (the parents of neighbours are neighbours), so the far field never covers it.
// Otherwise the ancestors meet in an interaction list at exactly one level <= l, as in the volume
// calculation, and there the source is a boundary cell. Every face lies in the subtree of one
// boundary cell per level; a subtree's leaves are consecutive in leaf (Morton) order, so its faces
// are one range of the face list.
struct BtvNear {
    std::vector<uint32_t> faces;     // leaf | (2 axis + side) << 28
    std::vector<int32_t> leaf_faces; // n_leaves + 1
    NearCSR near;                    // col: face | (touching class + 1) << 24
    NearCSR vtb;                     // rows: faces; col: source leaf | (touching class + 1) << 24
};

// The class of the boundary face (type, of the level-L cell fc) against the volume cell c, or -1
// if the closed cell and face do not meet.
int face_touch_class(const bcv_tree_s &t, int32_t c, int32_t fc, int type)
{
    if (t.level[c] != t.level[fc]) return -1;  // cells meeting the boundary all have level L
    const int ax = type >> 1, side = type & 1;
    int o[3];
    for (int d = 0; d < 3; ++d) {
        o[d] = t.ijk[3 * fc + d] - t.ijk[3 * c + d];
        if (o[d] < -1 || o[d] > 1) return -1;
    }
    for (int d = 0; d < 3; ++d) {
        const int flo = d == ax ? o[d] + side : o[d], fhi = d == ax ? o[d] + side : o[d] + 1;
        if (std::max(flo, 0) > std::min(fhi, 1)) return -1;
    }
    return face_class(o, ax, side);
}

// VtB (Algorithm 2) near rows: a face's target is its level-L cell w, whose near sources are the
// leaves of N*(w), the volume near row of w; the entries are the single-layer ones of BtV.
void build_vtb_near(const bcv_tree_s &t, const NearCSR &vol, BtvNear &r)
{
    const int64_t nf = (int64_t)r.faces.size();
    BCV_REQUIRE(t.n_leaves() < (1 << 24), BCV_ENOTSUP, "VtB: more than 2^24 leaves");
    r.vtb.row.assign(nf + 1, 0);
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t leaf = (int32_t)(r.faces[f] & 0x0FFFFFFFu);
        r.vtb.row[f + 1] = r.vtb.row[f] + (vol.row[leaf + 1] - vol.row[leaf]);
    }
    r.vtb.col.resize(r.vtb.row[nf]);
    int64_t touch = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : touch)
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t leaf = (int32_t)(r.faces[f] & 0x0FFFFFFFu);
        const int type = (int)(r.faces[f] >> 28);
        const int32_t fc = t.leaf_cell[leaf];
        int64_t out = r.vtb.row[f];
        for (int64_t e = vol.row[leaf]; e < vol.row[leaf + 1]; ++e) {
            const int32_t s = (int32_t)(vol.col[e] & 0x0FFFFFFFu);
            const int cls = face_touch_class(t, t.leaf_cell[s], fc, type);
            touch += cls >= 0;
            r.vtb.col[out++] = (uint32_t)s | ((uint32_t)(cls + 1) << 24);
        }
    }
    r.vtb.n_touch = touch;
}

BtvNear build_btv_near(const bcv_tree_s &t, const std::vector<Grid> &g, bool direct)
{
    BtvNear r;
    const std::vector<int32_t> fl = tree_faces(t);
    const int64_t nf = (int64_t)fl.size() / 3, nl = t.n_leaves();
    BCV_REQUIRE(nf < (1 << 24), BCV_ENOTSUP, "more than 2^24 boundary faces");
    r.faces.resize(nf);
    r.leaf_faces.assign(nl + 1, 0);
    for (int64_t f = 0; f < nf; ++f) {
        r.faces[f] = (uint32_t)fl[3 * f] | ((uint32_t)(2 * fl[3 * f + 1] + fl[3 * f + 2]) << 28);
        ++r.leaf_faces[fl[3 * f] + 1];
    }
    for (int64_t q = 0; q < nl; ++q) r.leaf_faces[q + 1] += r.leaf_faces[q];
    // leaf range [lo, hi) of every cell's subtree, finest level first
    const int64_t nc = t.n_cells();
    std::vector<int32_t> lo(nc), hi(nc), count(nc);
    for (int lev = t.L; lev >= 0; --lev)
        for (int32_t c = t.lvl_start[lev]; c < t.lvl_start[lev + 1]; ++c) {
            if (!t.refined[c]) {
                lo[c] = t.leaf_of_cell[c];
                hi[c] = lo[c] + 1;
                count[c] = 1;
                continue;
            }
            lo[c] = INT32_MAX, hi[c] = 0, count[c] = 0;
            for (int d = 0; d < 8; ++d) {
                const int32_t ch = t.first_child[c] + d;
                lo[c] = std::min(lo[c], lo[ch]);
                hi[c] = std::max(hi[c], hi[ch]);
                count[c] += count[ch];
            }
            BCV_REQUIRE(hi[c] - lo[c] == count[c], BCV_ESTATE, "internal: subtree leaves not consecutive");
        }
    auto on_boundary = [](int lev, const int32_t *c) {
        const int32_t top = (1 << lev) - 1;
        return c[0] == 0 || c[1] == 0 || c[2] == 0 || c[0] == top || c[1] == top || c[2] == top;
    };
    // class of (leaf cell c, face f), or -1 if they do not meet
    auto touch_class = [&](int32_t c, int64_t f) {
        return face_touch_class(t, c, t.leaf_cell[r.faces[f] & 0x0FFFFFFFu], (int)(r.faces[f] >> 28));
    };
    auto gen = [&](int64_t q, std::vector<uint32_t> &out) {
        out.clear();
        const int32_t c = t.leaf_cell[q];
        const int lev = t.level[c];
        auto add = [&](int64_t f0, int64_t f1) {
            for (int64_t f = f0; f < f1; ++f) {
                const int cls = touch_class(c, f);
                out.push_back((uint32_t)f | ((uint32_t)(cls + 1) << 24));
            }
        };
        if (direct) {
            add(0, nf);
            return;
        }
        const int32_t *ijk = &t.ijk[3 * c];
        for (const auto &o : stencil()) {
            const int32_t nb[3] = {ijk[0] + o[0], ijk[1] + o[1], ijk[2] + o[2]};
            const int32_t n = g[lev].at(nb[0], nb[1], nb[2]);
            if (n < 0 || !on_boundary(lev, nb)) continue;
            add(r.leaf_faces[lo[n]], r.leaf_faces[hi[n]]);
        }
    };
    r.near.row.assign(nl + 1, 0);
#pragma omp parallel
    {
        std::vector<uint32_t> buf;
#pragma omp for schedule(dynamic, 256)
        for (int64_t q = 0; q < nl; ++q) {
            gen(q, buf);
            r.near.row[q + 1] = (int64_t)buf.size();
        }
    }
    for (int64_t q = 0; q < nl; ++q) r.near.row[q + 1] += r.near.row[q];
    r.near.col.resize(r.near.row[nl]);
    int64_t touch = 0;
#pragma omp parallel reduction(+ : touch)
    {
        std::vector<uint32_t> buf;
#pragma omp for schedule(dynamic, 256)
        for (int64_t q = 0; q < nl; ++q) {
            gen(q, buf);
            std::copy(buf.begin(), buf.end(), r.near.col.begin() + r.near.row[q]);
            for (uint32_t e : buf) touch += (e >> 24) != 0;
        }
    }
    r.near.n_touch = touch;
    return r;
}

}  // namespace

// Degree-p leaf bases: coefficient layout, the block rows of the near field (columns = source
// coefficients, shared by the target's rows), the apply's work items, and per near entry its target
// and the position of its block in the target's row (for the plan-time assembly).
void build_basis_near(bcv_plan_s &p, const bcv_tree_s &t, const NearCSR &near, std::vector<int32_t> &pair_t,
                      std::vector<int32_t> &pair_pos)
{
    const int64_t nl = p.n_leaves;
    std::vector<int32_t> nb(nl);
    std::vector<int64_t> hi_off(nl + 1, 0);
    for (int64_t w = 0; w < nl; ++w) {
        nb[w] = ncoef(t.L - t.level[t.leaf_cell[w]]);
        hi_off[w + 1] = hi_off[w] + (nb[w] - 1);
    }
    p.n_dofs = nl + hi_off[nl];
    BCV_REQUIRE(p.n_dofs < (int64_t(1) << 31), BCV_ENOTSUP, "degree-p leaf bases: more than 2^31 coefficients");
    std::vector<int32_t> dof_leaf(std::max<int64_t>(hi_off[nl], 1));
    for (int64_t w = 0; w < nl; ++w)
        for (int64_t k = hi_off[w]; k < hi_off[w + 1]; ++k) dof_leaf[k] = (int32_t)w;
    std::vector<int64_t> cb(nl + 1, 0), vb(nl, 0);
    pair_t.resize(near.col.size());
    pair_pos.resize(near.col.size());
    for (int64_t w = 0; w < nl; ++w) {
        int64_t len = 0;
        for (int64_t e = near.row[w]; e < near.row[w + 1]; ++e) {
            pair_t[e] = (int32_t)w;
            BCV_REQUIRE(len < (int64_t(1) << 31), BCV_ENOTSUP, "degree-p leaf bases: near row too long");
            pair_pos[e] = (int32_t)len;
            len += nb[near.col[e] & 0x0FFFFFFFu];
        }
        cb[w + 1] = cb[w] + len;
    }
    int64_t nv = 0;
    for (int64_t w = 0; w < nl; ++w) {
        vb[w] = nv;
        nv += (int64_t)nb[w] * (cb[w + 1] - cb[w]);
    }
    std::vector<int32_t> bcol(std::max<int64_t>(cb[nl], 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t w = 0; w < nl; ++w) {
        int64_t j = cb[w];
        for (int64_t e = near.row[w]; e < near.row[w + 1]; ++e) {
            const int32_t s = (int32_t)(near.col[e] & 0x0FFFFFFFu);
            bcol[j++] = s;
            for (int k = 1; k < nb[s]; ++k) bcol[j++] = (int32_t)(nl + hi_off[s] + (k - 1));
        }
    }
    // Work units: kBasisRows rows of one target over at most `unit` columns (each unit streams at most
    // kBasisRows * unit block entries); longer rows are cut into equal pieces with partial sums.
    const int64_t unit = 4096;
    std::vector<BasisUnit> work;
    std::vector<BasisSplit> splits;
    int32_t n_partial = 0;
    for (int64_t w = 0; w < nl; ++w) {
        const int64_t len = cb[w + 1] - cb[w];
        const int64_t pieces = std::max<int64_t>(1, (len + unit - 1) / unit);
        for (int a0 = 0; a0 < nb[w]; a0 += kBasisRows) {
            if (pieces == 1) {
                work.push_back({0, (int32_t)w, a0, (int32_t)len, -1});
                continue;
            }
            splits.push_back({(int32_t)w, a0, n_partial, (int32_t)pieces});
            for (int64_t k = 0; k < pieces; ++k) {
                const int64_t j0 = len * k / pieces, j1 = len * (k + 1) / pieces;
                work.push_back({j0, (int32_t)w, a0, (int32_t)(j1 - j0), n_partial});
                n_partial += kBasisRows;
            }
        }
    }
    std::stable_sort(work.begin(), work.end(), [](const BasisUnit &a, const BasisUnit &b) { return a.len > b.len; });
    p.n_bvals = nv;
    p.n_bcols = cb[nl];
    p.n_bwork = (int64_t)work.size();
    p.n_bsplits = (int64_t)splits.size();
    p.d_bsplits = upload(&p, splits);
    if (n_partial > 0) p.d_bpartial = alloc_zero<double>(&p, (size_t)n_partial);
    p.d_hi_off = upload(&p, hi_off);
    p.d_dof_leaf = upload(&p, dof_leaf);
    p.d_bcb = upload(&p, cb);
    p.d_bvb = upload(&p, vb);
    p.d_bcol = upload(&p, bcol);
    p.d_bwork = upload(&p, work);
    p.d_bval = alloc_zero<double>(&p, (size_t)std::max<int64_t>(nv, 1));
    const BasisTables tb = basis_tables();
    p.d_btab = upload(&p, &tb, 1);
}

void destroy_plan(bcv_plan_s *p);

// Mapped meshes: the per-leaf and per-cell geometry of the apply (see mapped.hip) and the touching
// near entries of ball leaves for the singular rule. Reference frame of the forest: mesh m occupies
// [4m, 4m + 1) x [0,1)^2, and a ball mesh's cells are the images of its reference cubes under the
// cube-to-ball map of its unit cube, shifted back by 4m along x.
template <int Q>
void mapped_rows(const std::vector<double> &pts, const std::vector<double> &cen, const bcv_tree_s &t,
                 std::vector<double> &kap, std::vector<double> &kapr)
{
    constexpr int K = ncoef(Q), R = nreduced(Q);
    constexpr MultiIndex<Q> mi{};
    constexpr FoldTable<Q> fold{};
    const int64_t nl = t.n_leaves();
    kap.assign((size_t)nl * K, 0.0);
    kapr.assign((size_t)nl * R, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < nl; ++l) {
        const int32_t c = t.leaf_cell[l];
        const double a = std::ldexp(1.0, -t.level[c]);
        double row[K] = {};
        for (int g = 0; g < 8; ++g) {
            const double *x = &pts[(8 * l + g) * 4];
            double pw[3][Q + 1];
            for (int ax = 0; ax < 3; ++ax) {
                const double d = (x[ax] - cen[4 * c + ax]) / a;
                pw[ax][0] = 1.0;
                for (int k = 1; k <= Q; ++k) pw[ax][k] = pw[ax][k - 1] * d / k;
            }
            for (int b = 0; b < K; ++b) row[b] += x[3] * pw[0][mi.e[b][0]] * pw[1][mi.e[b][1]] * pw[2][mi.e[b][2]];
        }
        for (int b = 0; b < K; ++b) kap[(size_t)l * K + b] = row[b];
        for (int r = 0; r < R; ++r) {
            double v = 0.0;
            for (int k = 0; k < fold.n[r]; ++k) {
                const int src = fold.src[r][k];
                v += fold.c[r][k] * ((mi.deg[src] & 1) ? -row[src] : row[src]);
            }
            kapr[(size_t)l * R + r] = v;
        }
    }
}

struct MappedTouch {
    std::vector<int64_t> entry;                 // every touching entry of a ball leaf
    std::vector<int64_t> work_entry, work_mirror;  // the pairs the rule runs on, and the (s, t) entry or -1
    std::vector<int32_t> work_target;
};

void setup_mapped(bcv_plan_s *p, const bcv_tree_s &t, const std::vector<Grid> &g, const NearCSR &near, bool direct,
                  MappedTouch &mt)
{
    const int64_t nl = t.n_leaves(), nc = t.n_cells();
    const double node[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
    auto mesh_of = [&](int32_t c) { return (t.ijk[3 * c] >> t.level[c]) / 4; };
    // the image of a reference point (forest frame) and the Jacobian determinant there
    auto place = [&](int m, const double x[3], double out[3]) {
        double jac = 1.0;
        const double sh = 4.0 * m;
        if (t.mesh_geom[m] == BCV_GEOM_BALL) {
            const double xl[3] = {x[0] - sh, x[1], x[2]};
            ball_map(xl, out, &jac);
            out[0] += sh;
        } else {
            out[0] = x[0], out[1] = x[1], out[2] = x[2];
        }
        return jac;
    };
    std::vector<double> pts((size_t)nl * 32), cen((size_t)nc * 4);
    std::vector<uint8_t> lm(nl);
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < nl; ++l) {
        const int32_t c = t.leaf_cell[l];
        const double a = std::ldexp(1.0, -t.level[c]);
        const int m = mesh_of(c);
        lm[l] = t.mesh_geom[m] == BCV_GEOM_BALL;
        for (int gi = 0; gi < 8; ++gi) {
            const double x[3] = {a * (t.ijk[3 * c] + node[gi & 1]), a * (t.ijk[3 * c + 1] + node[(gi >> 1) & 1]),
                                 a * (t.ijk[3 * c + 2] + node[(gi >> 2) & 1])};
            double *o = &pts[(size_t)(8 * l + gi) * 4];
            const double jac = place(m, x, o);
            o[3] = a * a * a * 0.125 * jac;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        const double a = std::ldexp(1.0, -t.level[c]);
        const double x[3] = {a * (t.ijk[3 * c] + 0.5), a * (t.ijk[3 * c + 1] + 0.5), a * (t.ijk[3 * c + 2] + 0.5)};
        place(mesh_of((int32_t)c), x, &cen[4 * c]);
        cen[4 * c + 3] = a;
    }
    std::vector<double> kap, kapr;
    switch (p->q) {
    case 4: mapped_rows<4>(pts, cen, t, kap, kapr); break;
    case 6: mapped_rows<6>(pts, cen, t, kap, kapr); break;
    case 8: mapped_rows<8>(pts, cen, t, kap, kapr); break;
    default: fail(BCV_ENOTSUP, "mapped meshes: q must be 4, 6 or 8");
    }
    p->d_leaf_pts = upload(p, pts);
    p->d_centre = upload(p, cen);
    p->d_kap = upload(p, kap);
    p->d_kapr = upload(p, kapr);
    p->d_leaf_mapped = upload(p, lm);
    // touching entries of ball leaves (they come first in each row); the rule is symmetric, so a pair
    // and its mirror (s, t) are computed once
    auto find = [&](int32_t row, int32_t col) -> int64_t {
        for (int64_t e = near.row[row]; e < near.split[row]; ++e)
            if ((int32_t)(near.col[e] & 0x0FFFFFFFu) == col) return e;
        return -1;
    };
    for (int64_t l = 0; l < nl; ++l)
        if (lm[l])
            for (int64_t e = near.row[l]; e < near.split[l]; ++e) {
                const int32_t s = (int32_t)(near.col[e] & 0x0FFFFFFFu);
                mt.entry.push_back(e);
                const int64_t m = s == (int32_t)l ? -1 : find(s, (int32_t)l);
                if (m >= 0 && s < (int32_t)l) continue;  // computed with its mirror
                mt.work_entry.push_back(e);
                mt.work_target.push_back((int32_t)l);
                mt.work_mirror.push_back(m);
            }
    p->n_mapped_touch = (int64_t)mt.entry.size();
    p->n_mapped_pairs = (int64_t)mt.work_entry.size();
    if (direct) return;
    // interaction lists of the ball cells of levels >= 2 (cell order), CSR; the cells of cube meshes
    // take the lattice interaction plan
    const int32_t c0 = t.L >= 2 ? t.lvl_start[2] : (int32_t)nc;
    std::vector<int32_t> tgt;
    for (int64_t c = c0; c < nc; ++c)
        if (t.mesh_geom[mesh_of((int32_t)c)] == BCV_GEOM_BALL) tgt.push_back((int32_t)c);
    std::vector<int64_t> off(tgt.size() + 1, 0);
    std::vector<std::vector<int32_t>> lists(tgt.size());
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < (int64_t)tgt.size(); ++q) {
        const int32_t c = tgt[q];
        const int lev = t.level[c];
        const int i = t.ijk[3 * c], j = t.ijk[3 * c + 1], k = t.ijk[3 * c + 2];
        auto &out = lists[(size_t)q];
        for (const auto &o : stencil()) {
            const int32_t pn = g[lev - 1].at((i >> 1) + o[0], (j >> 1) + o[1], (k >> 1) + o[2]);
            if (pn < 0 || !t.refined[pn]) continue;
            for (int d = 0; d < 8; ++d) {
                const int32_t s = t.first_child[pn] + d;
                if (!is_neighbour_offset(i - t.ijk[3 * s], j - t.ijk[3 * s + 1], k - t.ijk[3 * s + 2])) out.push_back(s);
            }
        }
    }
    for (size_t q = 0; q < lists.size(); ++q) off[q + 1] = off[q] + (int64_t)lists[q].size();
    std::vector<int32_t> src((size_t)off.back());
    for (size_t q = 0; q < lists.size(); ++q) std::copy(lists[q].begin(), lists[q].end(), src.begin() + off[q]);
    p->n_ilist = off.back();
    p->n_m2l = p->n_ilist;
    p->n_ilist_targets = (int64_t)tgt.size();
    p->d_ilist_tgt = upload(p, tgt);
    p->d_ilist_off = upload(p, off);
    p->d_ilist_src = upload(p, src);
}

bcv_plan_s *build_plan(const bcv_tree_s &t, const bcv_plan_opts &opts, int device)
{
    BCV_HIP(hipSetDevice(device));
    std::unique_ptr<bcv_plan_s, void (*)(bcv_plan_s *)> p(new bcv_plan_s, destroy_plan);
    p->device = device;
    p->L = t.L;
    p->q = opts.q;

    p->direct = opts.direct;
    p->nearfield = opts.nearfield;
    p->near_order = opts.near_order;
    p->precision = opts.precision;
    if (opts.precision == BCV_MIXED_SPLIT16)
        BCV_REQUIRE(opts.q == 6 && !opts.q_schedule, BCV_ENOTSUP,
                    "BCV_MIXED_SPLIT16 supports the fixed order q = 6 only");
    for (int lev = 0; lev <= t.L + 1 && lev <= kMaxLevel + 1; ++lev) p->lvl_start[lev] = t.lvl_start[lev];
    for (int m = 0; m < t.n_meshes; ++m) p->mapped = p->mapped || t.mesh_geom[m] == BCV_GEOM_BALL;
    if (p->mapped) {
        BCV_REQUIRE(opts.nearfield == BCV_NEAR_ASSEMBLED, BCV_ENOTSUP,
                    "mapped (ball) meshes need the assembled near field (BCV_NEAR_ASSEMBLED)");
        BCV_REQUIRE(opts.q == 4 || opts.q == 6 || opts.q == 8, BCV_ENOTSUP, "mapped (ball) meshes: q = 4, 6 or 8");
        BCV_REQUIRE(!opts.q_schedule && opts.near_order == 0 && opts.basis_degree == 0 && !opts.boundary &&
                        !opts.surrogate && opts.precision != BCV_MIXED_SPLIT16,
                    BCV_ENOTSUP,
                    "mapped (ball) meshes: fixed order, the 2x2x2 near rule, BCV_FP64 or BCV_MIXED_F32, no "
                    "basis, boundary or surrogate");
    }
    if (opts.basis_degree != 0) {
        BCV_REQUIRE(opts.basis_degree == 1, BCV_EINVAL, "basis_degree must be 0 or 1");
        BCV_REQUIRE(opts.precision == BCV_FP64, BCV_ENOTSUP, "degree-p leaf bases: BCV_FP64 only");
        BCV_REQUIRE(t.n_meshes == 1 && t.mesh_side[0] == 1.0, BCV_ENOTSUP,
                    "degree-p leaf bases: a single mesh of side 1");
        BCV_REQUIRE(!opts.boundary && !opts.surrogate, BCV_ENOTSUP,
                    "degree-p leaf bases: no boundary structures, no surrogate");
        int coarsest = t.L;
        for (int64_t l = 0; l < t.n_leaves(); ++l) coarsest = std::min<int>(coarsest, t.level[t.leaf_cell[l]]);
        BCV_REQUIRE(t.L - coarsest <= kMaxBasisDegree, BCV_ENOTSUP, "degree-p leaf bases: leaf degrees above 8");
        p->basis = 1;
        p->basis_P = t.L - coarsest;
        p->near_order = 0;
    }
    p->streams = opts.streams;
    if (p->streams == 2) {
        BCV_HIP(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
        BCV_HIP(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
        BCV_HIP(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
        BCV_HIP(hipEventCreateWithFlags(&p->ev_fork2, hipEventDisableTiming));
    }
    // expansion orders per level and the row strides of the coefficient arrays. Orders without
    // kernels of their own (fixed q other than 4, 6, 8) run the level-by-level kernels of the
    // level-dependent orders with the same order on every level.
    const bool per_level = opts.q_schedule || !(opts.q == 4 || opts.q == 6 || opts.q == 8);
    p->q_schedule = per_level;
    p->exact_moments = opts.exact_moments;
    int q_max = opts.q;
    for (int lev = 0; lev <= kMaxLevel; ++lev) {
        p->q_level[lev] = opts.q_schedule ? opts.q + t.L - std::max(lev, 2) : opts.q;
        if (lev <= t.L) q_max = std::max(q_max, p->q_level[lev]);
    }
    if (per_level) {
        BCV_REQUIRE(t.n_meshes == 1, BCV_ENOTSUP,
                    "level-dependent orders and fixed orders other than 4, 6, 8: single-mesh trees only");
        BCV_REQUIRE(q_max <= kMaxSchedQ, BCV_EINVAL, "level-dependent orders: q + L - 2 must not exceed 10");
    }
    // meshes whose cube is not the unit cube: the apply scales u by side^5 (boundary plans: unit side only)
    bool scaled = false;
    for (int m = 0; m < t.n_meshes; ++m) scaled = scaled || t.mesh_side[m] != 1.0;
    BCV_REQUIRE(!scaled || !opts.boundary, BCV_ENOTSUP, "the boundary (BtV/VtB) structures need a domain of side 1");
    p->K = ncoef(q_max);
    p->R = (q_max + 1) * (q_max + 1);
    p->n_leaves = t.n_leaves();
    p->n_cells = t.n_cells();
    BCV_REQUIRE(p->n_leaves < (1 << 28), BCV_ENOTSUP, "more than 2^28 leaves");
    if (opts.direct) BCV_REQUIRE(p->n_leaves <= 20000, BCV_EINVAL, "direct mode is limited to 20000 leaves");

    double touch[kTouchClasses];
    touching_integrals(device, touch);
    if (opts.surrogate) {
        // the six contact classes as canonical pairs (smaller cube [0,1]^3, the other of side 1 or 2)
        const bcv_touch_pair cls[6] = {{BCV_CONTACT_FACE, 0, 1.0, {0.0, 0.0}},   {BCV_CONTACT_EDGE, 0, 1.0, {0.0, 0.0}},
                                       {BCV_CONTACT_VERTEX, 0, 1.0, {0.0, 0.0}}, {BCV_CONTACT_FACE, 0, 2.0, {0.0, 0.0}},
                                       {BCV_CONTACT_EDGE, 0, 2.0, {0.0, 0.0}},   {BCV_CONTACT_VERTEX, 0, 2.0, {0.0, 0.0}}};
        double value[6], est[6];
        int32_t fb[6];
        int64_t n_fb = 0;
        surrogate_eval(*opts.surrogate, 6, cls, opts.surrogate_tol, value, est, fb, &n_fb);
        // a class takes the network's value only where it is accepted; a rejected class keeps the
        // exact table value (its fallback, the high-order quadrature, is less accurate than that)
        p->surrogate_classes = 0;
        for (int c = 0; c < 6; ++c)
            if (!fb[c]) {
                touch[1 + c] = value[c];
                ++p->surrogate_classes;
            }
    }
    for (int c = 0; c < kTouchClasses; ++c) p->touch_value[c] = touch[c] / (4.0 * M_PI);

    const std::vector<Grid> grids = make_grids(t);
    const LeafGeo geo = leaf_geometry(t);

    // Leaf geometry (lower corner and side, exact dyadic values) and leaf -> cell map.
    std::vector<double> lg(4 * p->n_leaves);
    for (int64_t l = 0; l < p->n_leaves; ++l) {
        const int32_t c = t.leaf_cell[l];
        const double a = std::ldexp(1.0, -t.level[c]);
        for (int ax = 0; ax < 3; ++ax) lg[4 * l + ax] = t.ijk[3 * c + ax] * a;
        lg[4 * l + 3] = a;
    }
    p->d_leaf_geom = upload(p.get(), lg);
    p->d_leaf_cell = upload(p.get(), t.leaf_cell);
    {
        std::vector<int32_t> rest;
        for (int64_t l = 0; l < p->n_leaves; ++l)
            if (t.level[t.leaf_cell[l]] != p->L) rest.push_back((int32_t)l);
        p->n_rest_leaves = (int64_t)rest.size();
        if (!rest.empty()) p->d_rest_leaves = upload(p.get(), rest);
    }
    if (scaled) {
        std::vector<double> us(p->n_leaves);
        for (int64_t l = 0; l < p->n_leaves; ++l) {
            const int32_t c = t.leaf_cell[l];
            const double sd = t.mesh_side[(t.ijk[3 * c] >> t.level[c]) / 4];
            us[l] = sd * sd * sd * sd * sd;
        }
        p->d_uscale = upload(p.get(), us);
    }

    NearCSR vol_near;  // kept for the VtB rows
    MappedTouch mapped_touch;  // mapped meshes: touching entries of ball leaves
    std::vector<int32_t> basis_pair_t, basis_pair_pos;  // degree-p leaf bases: per near entry
    // Level-dependent near-field rule: per-leaf Gauss orders and the entries that need them.
    std::vector<int8_t> near_order;
    std::vector<int64_t> ordered_entry;
    std::vector<int32_t> ordered_target;
    {
        NearCSR near = build_near(t, grids, geo, opts.direct != 0);
        if (opts.near_order == 1) {
            // n_l = 2 + L - l points per axis, L the finest level of the leaf's mesh
            near_order.resize(p->n_leaves);
            for (int64_t l = 0; l < p->n_leaves; ++l) {
                const int32_t c = t.leaf_cell[l];
                const int m = (t.ijk[3 * c] >> t.level[c]) / 4;
                near_order[l] = (int8_t)(2 + t.mesh_L[m] - t.level[c]);
            }
            for (int64_t n = 0; n < p->n_leaves; ++n)
                for (int64_t e = near.split[n]; e < near.row[n + 1]; ++e) {  // the non-touching entries
                    const int32_t s = (int32_t)(near.col[e] & 0x0FFFFFFFu);
                    if (near_order[n] != 2 || near_order[s] != 2) {
                        ordered_entry.push_back(e);
                        ordered_target.push_back((int32_t)n);
                    }
                }
        }
        if (p->basis) build_basis_near(*p, t, near, basis_pair_t, basis_pair_pos);
        p->n_near = (int64_t)near.col.size();
        p->n_touch = near.n_touch;
        p->d_split = upload(p.get(), near.split);
        p->d_col = upload(p.get(), near.col);
        const NearUnits nu =
            build_near_units(near, p->n_leaves, opts.near_unit > 0 ? opts.near_unit : kDefaultNearUnit, true);
        p->n_units = (int64_t)nu.units.size();
        for (int x = 0; x <= kXcds; ++x) p->near_xcd[x] = nu.xcd_begin[x];
        p->n_splits = (int64_t)nu.splits.size();
        p->d_units = upload(p.get(), nu.units);
        p->d_splits = upload(p.get(), nu.splits);
        if (nu.n_partial > 0) p->d_partial = alloc_zero<double>(p.get(), (size_t)nu.n_partial);
        if (p->mapped) setup_mapped(p.get(), t, grids, near, opts.direct != 0, mapped_touch);
        if (opts.boundary) vol_near = std::move(near);
    }

    if (!opts.direct) {
        // Per-level lists of marked cells for the upward and downward passes.
        std::vector<int32_t> parents;
        p->parent_begin.assign(t.L + 2, 0);
        for (int lev = 0; lev <= t.L; ++lev) {
            p->parent_begin[lev] = (int32_t)parents.size() / 2;
            for (int32_t c = t.lvl_start[lev]; c < t.lvl_start[lev + 1]; ++c)
                if (t.refined[c]) {
                    parents.push_back(c);
                    parents.push_back(t.first_child[c]);
                }
        }
        p->parent_begin[t.L + 1] = (int32_t)parents.size() / 2;
        p->d_parents = upload(p.get(), parents);
        p->d_cell_leaf = upload(p.get(), t.leaf_of_cell);

        // Longest slot list per task piece. With level-dependent orders a coarse level's slot costs
        // (q_l / q)^4 times more and its few tasks would run as a handful of long waves: its pieces
        // are halved per order above q (at least 8 slots), so more waves share the work.
        const int32_t slots = opts.m2l_max_slots > 0 ? opts.m2l_max_slots
                                                     : (per_level ? kDefaultMaxSlotsSchedule : kDefaultMaxSlots);
        std::vector<int32_t> level_slots(t.L + 1, slots);
        if (per_level)
            for (int lev = 0; lev <= t.L; ++lev)
                level_slots[lev] = std::max<int32_t>(8, slots >> std::min(16, p->q_level[lev] - opts.q));
        // The lattice interaction plan: every cell, or with mapped meshes the cells of the cube
        // meshes (ball cells take the pair lists of setup_mapped).
        std::vector<uint8_t> lattice_target;
        bool lattice = !p->mapped;
        if (p->mapped) {
            lattice_target.assign(t.n_cells(), 0);
            for (int64_t c = 0; c < t.n_cells(); ++c) {
                lattice_target[c] = t.mesh_geom[(t.ijk[3 * c] >> t.level[c]) / 4] == BCV_GEOM_BOX;
                lattice = lattice || lattice_target[c];
            }
        }
        if (lattice) {
        M2LPlan m2l = build_m2l(t, grids, level_slots, per_level,
                                opts.m2l_max_slots == 0 && !per_level ? kDefaultMaxSlotsSchedule : 0, nullptr,
                                p->mapped ? lattice_target.data() : nullptr, opts.precision != BCV_MIXED_F32);
        std::vector<int32_t> id_of_key(15 * 15 * 15, -1);
        for (int32_t key : m2l.slot_key) id_of_key[key & 0x7FFFFFFF] = 0;
        std::vector<double> G;
        int32_t n_off = 0;
        for (int key = 0; key < 15 * 15 * 15; ++key) {
            if (id_of_key[key] < 0) continue;
            id_of_key[key] = n_off++;
            const int o[3] = {key / 225 - 7, (key / 15) % 15 - 7, key % 15 - 7};
            const size_t at = G.size();
            G.resize(at + p->K);
            derivative_table(q_max, o, &G[at]);  // a level of order q_l reads the first ncoef(q_l) entries
        }
        for (int32_t &s : m2l.slot_key) s = id_of_key[s & 0x7FFFFFFF] | (s & (int32_t)0x80000000);
        p->n_offsets = n_off;
        p->n_m2l = m2l.n_pairs + p->n_ilist;
        p->n_m2l_lanes = (int64_t)m2l.slot_key.size() * 64;
        p->n_m2l_read_lanes = m2l.n_read_lanes;
        p->n_tasks = (int64_t)m2l.tasks.size();
        p->d_G = upload(p.get(), G);
        if (p->precision != BCV_FP64) {
            std::vector<float> G32(G.begin(), G.end());
            p->d_G32 = upload(p.get(), G32);
        }
        if (p->precision == BCV_MIXED_SPLIT16) {
            // matrix-core operands of every offset, and per slot the targets whose list holds it
            std::vector<uint16_t> A;
            std::vector<float> G48;
            split16_tables(p->K, G, n_off, A, G48);
            p->d_m2l_A = reinterpret_cast<uint32_t *>(upload(p.get(), A));
            p->d_G48 = upload(p.get(), G48);
            const int64_t n_slots = (int64_t)m2l.slot_key.size();
            std::vector<uint64_t> mask(std::max<int64_t>(n_slots, 1), 0);
#pragma omp parallel for schedule(static)
            for (int64_t sl = 0; sl < n_slots; ++sl) {
                uint64_t mk = 0;
                for (int lane = 0; lane < 64; ++lane)
                    if (m2l.slot_src[sl * 64 + lane] >> 31) mk |= 1ull << lane;
                mask[sl] = mk;
            }
            p->d_slot_mask = upload(p.get(), mask);
        }
        p->d_tasks = upload(p.get(), m2l.tasks);
        p->d_task_targets = upload(p.get(), m2l.targets);
        p->d_slot_off = upload(p.get(), m2l.slot_key);
        p->d_slot_src = upload(p.get(), m2l.slot_src.get(), (size_t)m2l.slot_key.size() * 64);
        p->n_m2l_splits = (int64_t)m2l.splits.size();
        p->d_m2l_splits = upload(p.get(), m2l.splits);
        if (m2l.n_pieces > 0)
            p->d_m2l_partial = alloc_zero<double>(p.get(), (size_t)m2l.n_pieces * 64 * p->K);
        int32_t longest = 0;
        for (int x = 0; x <= kXcds; ++x) p->xcd_begin[x] = m2l.xcd_begin[x];
        for (int x = 0; x < kXcds; ++x) longest = std::max(longest, m2l.xcd_begin[x + 1] - m2l.xcd_begin[x]);
        p->m2l_groups = (int64_t)kXcds * longest;
        for (int lev = 0; lev <= kMaxLevel; ++lev)
            for (int x = 0; x <= kXcds; ++x) p->level_xcd[lev][x] = m2l.level_xcd[lev][x];
        if (opts.boundary) {
            // BtV: sources restricted to the boundary cells B_l; VtB: targets restricted to them.
            std::vector<uint8_t> on_b(t.n_cells(), 0);
            for (int64_t c = 0; c < t.n_cells(); ++c) {
                const int lev = t.level[c];
                const int32_t top = (1 << lev) - 1;
                const int32_t *x = &t.ijk[3 * c];
                on_b[c] = std::min({x[0], x[1], x[2], top - x[0], top - x[1], top - x[2]}) == 0;
            }
            const int32_t small = opts.m2l_max_slots == 0 ? kDefaultMaxSlotsSchedule : 0;
            auto make_set = [&](const uint8_t *src_ok, const uint8_t *tgt_ok, M2LSet &ms) {
                M2LPlan b = build_m2l(t, grids, level_slots, false, small, src_ok, tgt_ok, opts.precision != BCV_MIXED_F32);
                for (int32_t &k : b.slot_key) {
                    const int32_t id = id_of_key[k & 0x7FFFFFFF];
                    BCV_REQUIRE(id >= 0, BCV_ESTATE, "internal: boundary interaction offset without a table");
                    k = id | (k & (int32_t)0x80000000);
                }
                ms.n_tasks = (int64_t)b.tasks.size();
                ms.n_pairs = b.n_pairs;
                ms.d_tasks = upload(p.get(), b.tasks);
                ms.d_task_targets = upload(p.get(), b.targets);
                ms.d_slot_off = upload(p.get(), b.slot_key);
                ms.d_slot_src = upload(p.get(), b.slot_src.get(), (size_t)b.slot_key.size() * 64);
                ms.n_m2l_splits = (int64_t)b.splits.size();
                ms.d_m2l_splits = upload(p.get(), b.splits);
                if (b.n_pieces > 0) ms.d_m2l_partial = alloc_zero<double>(p.get(), (size_t)b.n_pieces * 64 * p->K);
                int32_t lg = 0;
                for (int x = 0; x <= kXcds; ++x) ms.xcd_begin[x] = b.xcd_begin[x];
                for (int x = 0; x < kXcds; ++x) lg = std::max(lg, b.xcd_begin[x + 1] - b.xcd_begin[x]);
                ms.m2l_groups = (int64_t)kXcds * lg;
            };
            make_set(on_b.data(), nullptr, p->btv_m2l);
            make_set(nullptr, on_b.data(), p->vtb_m2l);
        }
        }
        p->d_M = alloc_zero<double>(p.get(), (size_t)(p->n_cells + 1) * p->K);
        p->d_Lam = alloc_zero<double>(p.get(), (size_t)p->n_cells * p->K);
        const size_t n_folded = (size_t)(p->n_cells + 1) * (size_t)p->R;
        if (p->precision != BCV_FP64)
            p->d_M32 = alloc_zero<float>(p.get(), n_folded);
        else
            p->d_Mr = alloc_zero<double>(p.get(), n_folded);
        if (p->precision == BCV_MIXED_SPLIT16) {
            p->d_M16 = alloc_zero<uint16_t>(p.get(), (size_t)(p->n_cells + 1) * kSplitRowHalves);
            p->d_fscale = alloc_zero<float>(p.get(), kFscaleParts + 1);
        }
    }

    if (opts.boundary) {
        BtvNear bn = build_btv_near(t, grids, opts.direct != 0);
        p->boundary = 1;
        p->n_faces = (int64_t)bn.faces.size();
        p->n_btv_near = (int64_t)bn.near.col.size();
        p->n_btv_touch = bn.near.n_touch;
        p->d_faces = upload(p.get(), bn.faces);
        p->d_leaf_faces = upload(p.get(), bn.leaf_faces);
        p->d_btv_col = upload(p.get(), bn.near.col);
        const NearUnits nu =
            build_near_units(bn.near, p->n_leaves, opts.near_unit > 0 ? opts.near_unit : kDefaultNearUnit);
        p->n_btv_units = (int64_t)nu.units.size();
        p->n_btv_splits = (int64_t)nu.splits.size();
        p->d_btv_units = upload(p.get(), nu.units);
        p->d_btv_splits = upload(p.get(), nu.splits);
        if (nu.n_partial > 0) p->d_btv_partial = alloc_zero<double>(p.get(), (size_t)nu.n_partial);
        std::vector<double> tv(2 * kFaceClasses);
        boundary_touching_integrals(tv.data(), tv.data() + kFaceClasses);
        p->d_btv_touch = upload(p.get(), tv);
        build_vtb_near(t, vol_near, bn);
        p->n_vtb_near = (int64_t)bn.vtb.col.size();
        p->d_vtb_col = upload(p.get(), bn.vtb.col);
        const NearUnits vu =
            build_near_units(bn.vtb, p->n_faces, opts.near_unit > 0 ? opts.near_unit : kDefaultNearUnit);
        p->n_vtb_units = (int64_t)vu.units.size();
        p->n_vtb_splits = (int64_t)vu.splits.size();
        p->d_vtb_units = upload(p.get(), vu.units);
        p->d_vtb_splits = upload(p.get(), vu.splits);
        if (vu.n_partial > 0) p->d_vtb_partial = alloc_zero<double>(p.get(), (size_t)vu.n_partial);
    }

    if (p->basis) {
        launch_basis_assemble(*p, basis_pair_t, basis_pair_pos, basis_touch_table(p->basis_P));
    } else if (opts.nearfield == BCV_NEAR_ASSEMBLED) {
        p->d_val = alloc_zero<double>(p.get(), (size_t)p->n_near);
        launch_near_assemble(*p, nullptr);
        BCV_HIP(hipDeviceSynchronize());
        if (opts.near_order == 1) launch_near_assemble_ordered(*p, ordered_entry, ordered_target, near_order);
        if (p->mapped) {
            launch_mapped_assemble(*p, mapped_touch.entry, mapped_touch.work_entry, mapped_touch.work_target,
                                   mapped_touch.work_mirror, kMappedRule, t.mapped_touch_cache[opts.direct != 0]);
        }
        if (p->precision != BCV_FP64) {  // the apply reads FP32 entries (touching pairs stay exact)
            p->d_val32 = alloc_zero<float>(p.get(), (size_t)p->n_near);
            launch_near_narrow(*p, nullptr);
            BCV_HIP(hipDeviceSynchronize());
            if (!p->mapped) {  // mapped meshes keep the FP64 entries: their touching values are per pair
                BCV_HIP(hipFree(p->d_val));
                p->d_val = nullptr;
                p->device_bytes -= (int64_t)(sizeof(double) * p->n_near);
            }
        }
    }
    p->n_near_ordered = (int64_t)ordered_entry.size();
    BCV_HIP(hipDeviceSynchronize());
    return p.release();
}

void destroy_plan(bcv_plan_s *p)
{
    if (!p) return;
    (void)hipSetDevice(p->device);
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->ev_fork2) (void)hipEventDestroy(p->ev_fork2);
    if (p->side) (void)hipStreamDestroy(p->side);
    void *bufs[] = {p->d_leaf_geom, p->d_leaf_cell, p->d_cell_leaf, p->d_rest_leaves, p->d_split, p->d_col, p->d_val, p->d_val32, p->d_units,
                    p->d_splits, p->d_partial, p->d_M, p->d_Lam, p->d_G,
                    p->d_M32, p->d_Mr, p->d_G32,
                    p->d_parents, p->d_tasks, p->d_task_targets, p->d_slot_off, p->d_slot_src,
                    p->d_slot_mask, p->d_m2l_A, p->d_G48, p->d_M16, p->d_fscale, p->d_uscale,
                    p->d_m2l_splits, p->d_m2l_partial, p->d_faces, p->d_leaf_faces, p->d_btv_col,
                    p->d_btv_units, p->d_btv_splits, p->d_btv_partial, p->d_btv_touch, p->d_vtb_col,
                    p->d_vtb_units, p->d_vtb_splits, p->d_vtb_partial, p->d_hi_off, p->d_dof_leaf, p->d_bcb,
                    p->d_bvb, p->d_bcol, p->d_bval, p->d_bwork, p->d_bsplits, p->d_bpartial, p->d_btab,
                    p->btv_m2l.d_tasks, p->btv_m2l.d_task_targets, p->btv_m2l.d_slot_off, p->btv_m2l.d_slot_src,
                    p->btv_m2l.d_m2l_splits, p->btv_m2l.d_m2l_partial, p->vtb_m2l.d_tasks,
                    p->vtb_m2l.d_task_targets, p->vtb_m2l.d_slot_off, p->vtb_m2l.d_slot_src,
                    p->vtb_m2l.d_m2l_splits, p->vtb_m2l.d_m2l_partial, p->d_leaf_pts, p->d_centre, p->d_kap,
                    p->d_kapr, p->d_leaf_mapped, p->d_ilist_tgt, p->d_ilist_off, p->d_ilist_src};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    p->magic = 0;
    delete p;
}

void set_timing(bcv_plan_s *p, int max_applies)
{
    for (hipEvent_t e : p->events) BCV_HIP(hipEventDestroy(e));
    p->events.clear();
    p->timing_cap = 0;
    p->timing_used = 0;
    for (int64_t n = 0; n < 2 * BCV_N_PHASES * (int64_t)max_applies; ++n) {
        hipEvent_t e;
        BCV_HIP(hipEventCreate(&e));
        p->events.push_back(e);
    }
    p->timing_cap = max_applies;
}

void phase_times(const bcv_plan_s *p, double *ms, int64_t *n)
{
    for (int k = 0; k < BCV_N_PHASES; ++k) ms[k] = 0.0;
    for (int s = 0; s < p->timing_used; ++s)
        for (int k = 0; k < BCV_N_PHASES; ++k) {
            const hipEvent_t a = p->events[2 * (BCV_N_PHASES * s + k)], b = p->events[2 * (BCV_N_PHASES * s + k) + 1];
            BCV_HIP(hipEventSynchronize(b));
            float t = 0.0f;
            BCV_HIP(hipEventElapsedTime(&t, a, b));
            ms[k] += t;
        }
    *n = p->timing_used;
}

}  // namespace bcv
