// Captured applies (one HIP graph launch per apply, for batched meshes and tight loops) and the
// autotuner of the plan's work decomposition.
#include <algorithm>
#include <memory>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace bcv {

bcv_plan_s *build_plan(const bcv_tree_s &t, const bcv_plan_opts &opts, int device);
void destroy_plan(bcv_plan_s *p);

bcv_graph_s *graph_create(const bcv_plan_s &p, const double *f, double *u)
{
    BCV_REQUIRE(p.timing_cap == 0, BCV_ESTATE, "phase timing is enabled on this plan; disable it before capturing");
    auto g = std::make_unique<bcv_graph_s>();
    g->device = p.device;
    g->plan = &p;
    hipStream_t cs = nullptr;
    BCV_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        try {
            launch_apply(p, f, u, BCV_PART_NEAR | BCV_PART_FAR, cs);
        } catch (...) {
            (void)hipStreamEndCapture(cs, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipStreamDestroy(cs);
            throw;
        }
        e = hipStreamEndCapture(cs, &graph);
    }
    (void)hipStreamDestroy(cs);
    BCV_HIP(e);
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        BCV_HIP(e);
    }
    return g.release();
}

void graph_launch(const bcv_graph_s &g, hipStream_t st) { BCV_HIP(hipGraphLaunch(g.exec, st)); }

void graph_destroy(bcv_graph_s *g)
{
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->magic = 0;
    delete g;
}

namespace {

struct PlanDeleter {
    void operator()(bcv_plan_s *p) const { destroy_plan(p); }
};

// Milliseconds per apply of a plan built with opts (density 1, two warm-up applies).
double time_plan(const bcv_tree_s &t, const bcv_plan_opts &opts, int device, int n_applies, double *f, double *u,
                 hipStream_t st)
{
    std::unique_ptr<bcv_plan_s, PlanDeleter> p(build_plan(t, opts, device));
    for (int k = 0; k < 2; ++k) launch_apply(*p, f, u, BCV_PART_NEAR | BCV_PART_FAR, st);
    hipEvent_t e0, e1;
    BCV_HIP(hipEventCreate(&e0));
    BCV_HIP(hipEventCreate(&e1));
    float ms = 0.0f;
    try {
        BCV_HIP(hipEventRecord(e0, st));
        for (int k = 0; k < n_applies; ++k) launch_apply(*p, f, u, BCV_PART_NEAR | BCV_PART_FAR, st);
        BCV_HIP(hipEventRecord(e1, st));
        BCV_HIP(hipEventSynchronize(e1));
        BCV_HIP(hipEventElapsedTime(&ms, e0, e1));
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)ms / n_applies;
}

}  // namespace

// Coordinate search: near_unit first (with the base piece length), then m2l_max_slots (not for forests
// of ball meshes only, whose interaction phase works pair by pair).
double autotune(const bcv_tree_s &t, const bcv_plan_opts &base, int device, int n_applies, bcv_plan_opts &best)
{
    BCV_REQUIRE(n_applies >= 1 && n_applies <= 1000, BCV_EINVAL, "n_applies must be 1..1000");
    const int64_t n = t.n_leaves();
    double *f = nullptr, *u = nullptr;
    if (hipMalloc(&f, n * sizeof(double)) != hipSuccess) fail(BCV_ENOMEM, "hipMalloc failed");
    if (hipMalloc(&u, n * sizeof(double)) != hipSuccess) {
        (void)hipFree(f);
        fail(BCV_ENOMEM, "hipMalloc failed");
    }
    double best_ms = 0.0;
    try {
        const std::vector<double> ones(n, 1.0);
        BCV_HIP(hipMemcpy(f, ones.data(), n * sizeof(double), hipMemcpyHostToDevice));
        hipStream_t st = nullptr;
        best = base;
        best_ms = time_plan(t, best, device, n_applies, f, u, st);
        for (int unit : {256, 512, 1024, 2048}) {
            bcv_plan_opts o = best;
            o.near_unit = unit;
            const double ms = time_plan(t, o, device, n_applies, f, u, st);
            if (ms < best_ms) best_ms = ms, best = o;
        }
        bool lattice = false;  // forests of ball meshes only have no lattice interaction tasks
        for (int m = 0; m < t.n_meshes; ++m) lattice = lattice || t.mesh_geom[m] == BCV_GEOM_BOX;
        for (int slots : {128, 256, 320, 512, 1024}) {
            if (!lattice) break;
            bcv_plan_opts o = best;
            o.m2l_max_slots = slots;
            const double ms = time_plan(t, o, device, n_applies, f, u, st);
            if (ms < best_ms) best_ms = ms, best = o;
        }
    } catch (...) {
        (void)hipFree(f);
        (void)hipFree(u);
        throw;
    }
    (void)hipFree(f);
    (void)hipFree(u);
    return best_ms;
}

}  // namespace bcv
