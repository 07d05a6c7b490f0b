"""Benchmark of the VtV apply (BC-FMM volume potential) on one MI355X.

Workload (the metric's configuration): unit-cube BC octree with boundary leaves of side h = 1/256
(L = 8, 896,512 leaves), expansion order q = 6, piecewise-constant Gaussian-mixture density
(seed 0). A step is one full VtV apply (Algorithm 1: moments, upward pass, interaction phase,
downward pass, near field and evaluation) with the density already resident in HBM. Plan
construction (lists, tables, workspace) happens once before timing and is reported separately.

The same mesh is timed twice: with the plain FP64 path and with the mixed path (FP32 interaction
phase and non-touching near field, FP64 singular pairs, tree passes and accumulation), whose
touching-pair class values come from the trained surrogate where it certifies 1e-7 (the network is
trained on the GPU before timing). The headline value is the mixed rate if the mixed result is
within rel-L2 1e-6 of the FP64 result (L2 norm of cell averages over Omega), else the FP64 rate.

Prints one JSON line with the metric, the per-phase device times from HIP events recorded on the
apply's stream, the roofline of the dominant kernel (algorithmic work per apply / its measured
time), the FP64 rate and the ratio, the CPU oracle's throughput on a bounded sample of the same
workload, and, as extras on the h = 1/128 mesh (L = 7): the plain FP64 apply (the second
workload configuration), BtV/VtB, level-dependent orders and the neighbour marking.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "VtV cell-potentials/s at rel-L2≤1e-6, mixed+surrogate vs plain FP64, 1 GPU"
PEAK_FP64 = 78.6e12  # MI355X FP64 vector (= FP64 matrix) peak, FLOP/s
PEAK_FP32 = 157.3e12  # MI355X FP32 vector peak, FLOP/s
REL_L2_GATE = 1e-6  # the mixed path counts only if its rel-L2 against the FP64 path is within this
SURROGATE_TOL = 1e-7  # touching-pair surrogate: accepted where its calibrated error estimate is below this
PEAK_HBM = 8.0e12  # bytes/s
PEAK_F16_MFMA = 2.5e15  # MI355X dense FP16 matrix peak, FLOP/s


def m2l_flops_per_pair(q):
    """Algorithmic flops of one interaction pair: one multiply-add per (alpha, beta) with
    |alpha| + |beta| <= q, i.e. 2 C(q + 6, 6) (1848 at q = 6)."""
    from math import comb

    return 2 * comb(q + 6, 6)


def m2l_reduced_flops_per_pair(q):
    """Flops the kernels execute per pair in the harmonic reduction (alpha_z, beta_z <= 1):
    2 sum_{n+m<=q} (2n+1)(2m+1) (1064 at q = 6)."""
    return 2 * sum((2 * n + 1) * (2 * m + 1) for n in range(q + 1) for m in range(q + 1 - n))


def ncoef(d):
    return (d + 1) * (d + 2) * (d + 3) // 6


def m2l_kernel_names(q, mixed):
    """The interaction-phase launches of one apply (see launch_m2l in kernels.hip)."""
    R = (q + 1) ** 2
    if mixed:
        blocks = [(0, R, 0, R)] if q <= 6 else [(0, R, 0, 16), (0, 25, 16, R)]
    elif q == 4:
        blocks = [(0, R, 0, R)]
    elif q == 6:
        blocks = [(0, R, 0, R)]
    else:
        blocks = [(0, R, 0, 36), (0, 9, 36, R)]

    def waves(b):  # as launch_m2l_block: two waves per SIMD where the block's registers exceed 110
        return 2 if (b[1] - b[0] + b[3] - b[2]) * (1 if mixed else 2) > 110 else 4

    kind = "float" if mixed else "double"
    return ["m2l_shift_kernel<%d, %s, %d, %d, %d, %d, %d>" % ((q, kind) + b + (waves(b),)) for b in blocks]


def near_flops(info, q):
    """Algorithmic flops of the on-the-fly near field: 64 kernel evaluations per point-rule pair.

    Per evaluation: r^2 from per-axis squared differences (2 adds), reciprocal square root counted
    as 1 flop, accumulate (1 add): 4 flops; plus 12 subtractions and 12 multiplies per pair for the
    per-axis differences, and 1 FMA per touching pair.
    """
    n_rule = info["n_near"] - info["n_touch"]
    return n_rule * (64 * 4 + 24) + 2 * info["n_touch"]


def cpu_baseline(L, q, f, u_gpu, n_targets, leaves):
    # u_gpu: the FP64 GPU result, compared with the oracle at the sampled leaves
    """The CPU oracle (O2, Algorithm 1 step by step in FP64) on a sample of target leaves."""
    from oracle import fmm
    from oracle.mesh import BCMesh

    t0 = time.perf_counter()
    mesh = BCMesh(L)
    t1 = time.perf_counter()
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(len(f), n_targets, replace=False))
    ref = fmm.FMM(mesh, q).apply_sampled(f, sample)
    t2 = time.perf_counter()
    assert np.array_equal(mesh.leaf_array(), leaves.astype(np.int64))
    err = float(np.max(np.abs(u_gpu[sample] - ref) / np.abs(ref)))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {
        "value": n_targets / (t2 - t1),
        "unit": "cell-potentials/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "O2 (Algorithm 1 step by step, NumPy + plain C) at %d random target leaves of the same "
                  "h=1/%d q=%d workload, including the full moment and upward passes; mesh build %.1f s "
                  "excluded" % (n_targets, 2 ** L, q, t1 - t0),
        "seconds": t2 - t1,
        "max_rel_diff_vs_gpu": err,
    }


def timed_applies(bcv, torch, plan, f, u, warmup, steps, dev):
    """Warm up, then time `steps` applies (wall clock around them) with per-phase HIP events."""
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        bcv.vtv_apply(plan, f, u, stream)
    torch.cuda.synchronize()
    bcv.plan_enable_timing(plan, steps)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        bcv.vtv_apply(plan, f, u, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    phases, n_rec = bcv.plan_phase_times(plan)
    bcv.plan_enable_timing(plan, 0)
    return 1e3 * elapsed / steps, {k: v / max(n_rec, 1) for k, v in phases.items()}


def measure(bcv, torch, tree, f, args, dev, nf, prec, surrogate=None):
    """Plan, warm up, then time `args.steps` applies with per-phase HIP events. The roofline comes
    from a second timed pass in which the near field runs after the far field on one stream, so
    that every phase's kernels have the GPU to themselves (with two streams the near-field and
    interaction kernels share the compute units and their durations say nothing about either)."""
    precision = {"fp64": bcv.FP64, "mixed": bcv.MIXED_F32, "split16": bcv.MIXED_SPLIT16}[prec]

    def make_plan(streams):
        return bcv.plan_interactions(tree, q=args.q, nearfield=nf, device=dev, streams=streams,
                                     precision=precision, surrogate=surrogate, surrogate_tol=SURROGATE_TOL)

    t0 = time.perf_counter()
    plan = make_plan(args.streams)
    plan_s = time.perf_counter() - t0
    info = plan.info
    u = torch.empty_like(f)
    ms, phase_avg = timed_applies(bcv, torch, plan, f, u, args.warmup, args.steps, dev)
    u_host = u.cpu().numpy()
    del plan
    if args.streams == 1:
        iso = phase_avg
    else:
        plan = make_plan(1)
        _, iso = timed_applies(bcv, torch, plan, f, u, args.warmup, args.steps, dev)
        del plan
    roof, roof_other = roofline(info, iso, args, prec, args.q)
    return {"plan_s": plan_s, "info": info, "ms": ms, "phases": phase_avg, "phases_serial": iso, "u": u_host,
            "roof": roof, "roof_other": roof_other}


def tree_pass_bytes(info, fp_bytes=8):
    """Algorithmic bytes of the tree passes per apply: every pass reads the coefficient array it
    consumes once and writes the one it produces once (K coefficients per cell, FP64):
    P2M reads f and writes the leaf moments; M2M reads the children's moments and writes the
    parents'; L2L reads the parents' local coefficients and reads and writes the children's."""
    K, n_leaf, n_cell = info["K"], info["n_leaves"], info["n_cells"]
    n_marked, n_child = n_cell - n_leaf, n_cell - 1
    p2m = n_leaf * 8 + n_leaf * K * fp_bytes
    m2m = (n_child + n_marked) * K * fp_bytes
    l2l = (n_marked + 2 * n_child) * K * fp_bytes
    return p2m + m2m + l2l


def roofline(info, phase_avg, args, prec, q):
    """Roofline of the interaction phase, the near field and the tree passes, per apply, from the
    phase times of the serialized pass (HIP events on the stream the phase runs on, averaged over
    the applies). Work counts are the algorithmic ones: 2 C(q+6, 6) flops per interaction pair,
    12 B (FP64 entry + index) or 8 B (FP32 entry + index) per assembled near pair."""
    from paper_2112_00864_amd import profiling

    mixed = prec != "fp64"
    peak = (PEAK_FP32 if mixed else PEAK_FP64) / 1e12
    m2l_ms = phase_avg["m2l"]
    near_ms = phase_avg["near"]
    m2l_roof = {"bound": "alu", "achieved": info["n_m2l"] * m2l_flops_per_pair(q) / (m2l_ms * 1e-3) / 1e12,
                "peak": peak, "unit": "TFLOP/s",
                "flops_per_pair": m2l_flops_per_pair(q),
                "achieved_executed_reduced": info["n_m2l"] * m2l_reduced_flops_per_pair(q) / (m2l_ms * 1e-3) / 1e12,
                "reduced_flops_per_pair": m2l_reduced_flops_per_pair(q),
                "ms": m2l_ms}
    if prec == "split16":
        # matrix cores: 48 v_mfma_f32_16x16x32_f16 per slot (4 target sets x 4 tiles x 3 split products)
        executed = info["n_m2l_lanes"] // 64 * 48 * 2 * 16 * 16 * 32
        m2l_roof.update({"bound": "mfma", "peak": PEAK_F16_MFMA / 1e12,
                         "mfma_executed_tflops": executed / (m2l_ms * 1e-3) / 1e12,
                         "mfma_utilisation": executed / (m2l_ms * 1e-3) / PEAK_F16_MFMA})
    if args.nearfield == "assembled":
        near_bytes = info["n_near"] * (8 if mixed else 12)
        near_roof = {"bound": "hbm", "achieved": near_bytes / (near_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                     "unit": "GB/s", "bytes_per_pair": 8 if mixed else 12, "ms": near_ms}
    else:
        near_roof = {"bound": "alu", "achieved": near_flops(info, q) / (near_ms * 1e-3) / 1e12,
                     "peak": peak, "unit": "TFLOP/s", "ms": near_ms}
    near_name = "near_eval_kernel<%d, %s, %s>" % (q, "true" if args.nearfield == "assembled" else "false",
                                                  "true" if mixed else "false")
    # the interaction phase: the interaction launches (reading the folded moment rows that P2M and
    # M2M write) and the sum of the split tasks' pieces
    if prec == "split16":
        m2l_names = ["split_rows_kernel", "m2l_mfma_kernel<%d>" % q, "m2l_combine_kernel"]
    else:
        m2l_names = m2l_kernel_names(q, mixed) + ["m2l_combine_kernel"]
    for roof_, names in ((m2l_roof, m2l_names), (near_roof, [near_name])):
        roof_["frac"] = roof_["achieved"] / roof_["peak"]
        # HBM bytes per apply (PMC, summed over the launches), None if stale
        traffic = [profiling.traffic_for(n, args.L, q) for n in names]
        roof_["traffic"] = None if None in traffic else sum(traffic)
        roof_["kernel"] = " + ".join(names)
        roof_["measured"] = ("HIP events per phase over %d applies, near field after the far field on one stream"
                             % args.steps)
    tree_ms = phase_avg["p2m"] + phase_avg["m2m"] + phase_avg["l2l"]
    tb = tree_pass_bytes(info)
    tree_roof = {"bound": "hbm", "achieved": tb / (tree_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                 "bytes": tb, "ms": tree_ms, "kernel": "P2M + M2M + L2L phases (all launches)"}
    tree_roof["frac"] = tree_roof["achieved"] / tree_roof["peak"]
    dominant = m2l_roof if m2l_ms >= near_ms else near_roof
    return dominant, {"m2l_kernel": m2l_roof, "near_eval_kernel": near_roof, "tree_passes": tree_roof}


def measure_btv(bcv, torch, tree, f, args, dev):
    """BtV (Algorithm 3) and VtB (Algorithm 2) on the same mesh: FP64 and mixed plans with boundary
    structures; BtV from seeded face data (traces of a harmonic function), VtB from the leaf density
    f; `args.steps` timed applies of each after `args.warmup`."""
    import synth

    lv = tree.leaves().astype(np.int64)
    faces = tree.faces().astype(np.int64)
    fk = np.column_stack([lv[faces[:, 0]], faces[:, 1:]])
    qf, gf = synth.face_data(fk, seed=0)
    q = torch.tensor(qf, device="cuda:%d" % dev)
    g = torch.tensor(gf, device="cuda:%d" % dev)
    out = {}
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        plan = bcv.plan_interactions(tree, q=args.q, device=dev, streams=1, boundary=True,
                                     precision=bcv.MIXED_F32 if prec == "mixed" else bcv.FP64)
        plan_s = time.perf_counter() - t0
        u = torch.empty(plan.n_leaves, dtype=torch.float64, device="cuda:%d" % dev)
        for _ in range(args.warmup):
            bcv.btv_apply(plan, q, g, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bcv.btv_apply(plan, q, g, u)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        out[prec] = {"ms_per_apply": ms, "value": plan.n_leaves / (ms * 1e-3), "plan_seconds": plan_s,
                     "u": u.cpu().numpy()}
        uf = torch.empty(plan.info["n_faces"], dtype=torch.float64, device="cuda:%d" % dev)
        for _ in range(args.warmup):
            bcv.vtb_apply(plan, f, uf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bcv.vtb_apply(plan, f, uf)
        torch.cuda.synchronize()
        ms_vtb = 1e3 * (time.perf_counter() - t0) / args.steps
        out[prec]["vtb"] = {"ms_per_apply": ms_vtb, "value": plan.info["n_faces"] / (ms_vtb * 1e-3),
                            "unit": "face-potentials/s", "uf": uf.cpu().numpy()}
        info = plan.info
        del plan
    vol = np.ldexp(1.0, -3 * lv[:, 0].astype(np.int32))
    a, b = out["mixed"]["u"], out["fp64"]["u"]
    rel = float(np.sqrt(np.sum(vol * ((a - b) / vol) ** 2) / np.sum(vol * (b / vol) ** 2)))
    charges, poles = synth.harmonic_params(0)
    avg = synth.cell_average(lv, lambda x: synth.harmonic(x, charges, poles), n=4)
    rep = float(np.linalg.norm(b / vol - avg) / np.linalg.norm(avg))
    va, vb = out["mixed"]["vtb"]["uf"], out["fp64"]["vtb"]["uf"]
    vtb_rel = float(np.linalg.norm(va - vb) / np.linalg.norm(vb))
    for prec in out:
        del out[prec]["u"]
        del out[prec]["vtb"]["uf"]
    return {"vtb_mixed_vs_fp64_rel": vtb_rel, "n_vtb_near_pairs": info["n_vtb_near"],"metric": "BtV cell-potentials/s (Algorithm 3, u = <1_w, V[q] - K[g]>), 1 GPU",
            "unit": "cell-potentials/s", "n_faces": info["n_faces"], "n_btv_near_pairs": info["n_btv_near"],
            "n_btv_touching_pairs": info["n_btv_touch"],
            "n_btv_m2l_pairs": info["n_btv_m2l"], "n_vtb_m2l_pairs": info["n_vtb_m2l"], "n_vtv_m2l_pairs": info["n_m2l"], "fp64": out["fp64"], "mixed": out["mixed"],
            "mixed_vs_fp64_rel_l2": rel, "representation_formula_rel_err": rep,
            "data": "synthetic: face averages of u = sum_k c_k/|x - p_k| (4 poles outside the cube, seed 0) and "
                    "of du/dn; the representation formula gives u in the cube"}


def measure_marking(bcv, torch, args, dev):
    """The neighbour marking rule (Sec. 2) with the level-dependent near-field rule (Sec. 4) at the
    same h and q: a mesh refined wherever a boundary cell is a neighbour, its near-field entries
    assembled once at plan time (2 + L - l Gauss points per axis on a level-l leaf). FP64 and mixed
    plans, `args.steps` timed applies each; the same Gaussian-mixture density recipe."""
    import synth

    tree = bcv.build_bc_tree(args.L, bcv.MARK_NEIGHBOR)
    lv = tree.leaves().astype(np.int64)
    f = torch.tensor(synth.leaf_density(lv, seed=0), device="cuda:%d" % dev)
    out = {}
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        plan = bcv.plan_interactions(tree, q=args.q, device=dev, streams=args.streams, nearfield=bcv.NEAR_ASSEMBLED,
                                     near_order=1, precision=bcv.MIXED_F32 if prec == "mixed" else bcv.FP64)
        plan_s = time.perf_counter() - t0
        u = torch.empty(plan.n_leaves, dtype=torch.float64, device="cuda:%d" % dev)
        for _ in range(args.warmup):
            bcv.vtv_apply(plan, f, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bcv.vtv_apply(plan, f, u)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        out[prec] = {"ms_per_apply": ms, "value": plan.n_leaves / (ms * 1e-3), "plan_seconds": plan_s,
                     "u": u.cpu().numpy()}
        info = plan.info
        del plan
    vol = np.ldexp(1.0, -3 * lv[:, 0].astype(np.int32))
    a, b = out["mixed"].pop("u"), out["fp64"].pop("u")
    rel = float(np.sqrt(np.sum(vol * ((a - b) / vol) ** 2) / np.sum(vol * (b / vol) ** 2)))
    return {"metric": "VtV cell-potentials/s, neighbour marking + level-dependent near-field rule, 1 GPU",
            "unit": "cell-potentials/s", "n_leaves": int(len(lv)), "n_near_pairs": info["n_near"],
            "n_near_ordered": info["n_near_ordered"], "n_touching_pairs": info["n_touch"],
            "n_m2l_pairs": info["n_m2l"], "plan_device_bytes": info["device_bytes"], "fp64": out["fp64"],
            "mixed": out["mixed"], "mixed_vs_fp64_rel_l2": rel,
            "config": "unit cube, h = 1/%d (L = %d), marking 1 (refine when a neighbour has a face on the boundary), "
                      "q = %d, near field assembled at plan time with 2 + L - l Gauss points per axis on a level-l "
                      "leaf, %d stream(s)" % (1 << args.L, args.L, args.q, args.streams)}


def measure_schedule(bcv, torch, tree, f, args, dev, u_ref):
    """Level-dependent expansion orders q_l = 4 + L - l (Sec. 4) on the same mesh and density: FP64
    and mixed plans, `args.steps` timed applies each; compared with the headline's FP64 apply at the
    fixed order (rel-L2 of the cell averages)."""
    q0 = 4
    if q0 + args.L - 2 > 10:
        return None
    lv = tree.leaves().astype(np.int64)
    nf = bcv.NEAR_ASSEMBLED if args.nearfield == "assembled" else bcv.NEAR_QUADRATURE
    out = {}
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        plan = bcv.plan_interactions(tree, q=q0, q_schedule=1, device=dev, streams=args.streams, nearfield=nf,
                                     precision=bcv.MIXED_F32 if prec == "mixed" else bcv.FP64)
        plan_s = time.perf_counter() - t0
        u = torch.empty(plan.n_leaves, dtype=torch.float64, device="cuda:%d" % dev)
        for _ in range(args.warmup):
            bcv.vtv_apply(plan, f, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bcv.vtv_apply(plan, f, u)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        out[prec] = {"ms_per_apply": ms, "value": plan.n_leaves / (ms * 1e-3), "plan_seconds": plan_s,
                     "u": u.cpu().numpy()}
        info = plan.info
        del plan
    vol = np.ldexp(1.0, -3 * lv[:, 0].astype(np.int32))

    def rel(a, b):
        return float(np.sqrt(np.sum(vol * ((a - b) / vol) ** 2) / np.sum(vol * (b / vol) ** 2)))

    a, b = out["mixed"].pop("u"), out["fp64"].pop("u")
    res = {"metric": "VtV cell-potentials/s, level-dependent orders q_l = 4 + L - l, 1 GPU",
           "unit": "cell-potentials/s", "orders": {"level %d" % l: q0 + args.L - l for l in range(args.L, 1, -1)},
           "n_m2l_pairs": info["n_m2l"], "plan_device_bytes": info["device_bytes"], "fp64": out["fp64"],
           "mixed": out["mixed"], "mixed_vs_fp64_rel_l2": rel(a, b)}
    if u_ref is not None:
        res["fp64_vs_fixed_order_fp64_rel_l2"] = rel(b, u_ref)
        res["fixed_order"] = args.q
    return res


def measure_basis(bcv, torch, args, dev):
    """Degree-p leaf bases p_l = L - l (Sec. 4), FP64, q = args.q, on the unit-cube mesh of level
    args.basis_L: the projection of the seed-0 Gaussian mixture onto every leaf's Legendre
    polynomials as input, `args.steps` applies timed after `args.warmup`, with per-phase HIP events
    (one stream). Roofline of the near field (block rows streamed from HBM): 8 B per block entry +
    12 B per column (index and gathered coefficient) + 8 B per output coefficient."""
    import synth

    L = args.basis_L
    tree = bcv.build_bc_tree(L)
    lv = tree.leaves().astype(np.int64)
    c, w = synth.gaussian_mixture_params(0)
    coef, off = synth.legendre_coefficients(lv, L, lambda x: synth.gaussian_mixture(x, c, w))
    nl = len(lv)
    nb = np.diff(off)
    f = np.empty(off[-1])
    f[:nl] = coef[off[:-1]]  # the library's layout: degree-0 coefficients first, then the rest leaf by leaf
    hi = np.concatenate([[0], np.cumsum(nb - 1)])
    for k in np.nonzero(nb > 1)[0]:
        f[nl + hi[k] : nl + hi[k + 1]] = coef[off[k] + 1 : off[k + 1]]
    fd = torch.tensor(f, device="cuda:%d" % dev)
    ud = torch.empty_like(fd)
    # the paper's experiment setup: p_l = L - l with q_l = 4 + L - l (Sec. 5)
    sched = None
    if 4 + L - 2 <= 10:
        t0 = time.perf_counter()
        splan = bcv.plan_interactions(tree, q=4, q_schedule=1, device=dev, streams=1, basis_degree=1)
        splan_s = time.perf_counter() - t0
        sms, sph = timed_applies(bcv, torch, splan, fd, ud, args.warmup, args.steps, dev)
        sched = {"orders": "q_l = 4 + L - l", "ms_per_apply": sms, "value": splan.info["n_dofs"] / (sms * 1e-3),
                 "phase_ms": sph, "plan_seconds": splan_s}
        del splan
    t0 = time.perf_counter()
    plan = bcv.plan_interactions(tree, q=args.q, device=dev, streams=1, basis_degree=1)
    plan_s = time.perf_counter() - t0
    ms, phases = timed_applies(bcv, torch, plan, fd, ud, args.warmup, args.steps, dev)
    info = plan.info
    near_bytes = 8 * info["n_basis_vals"] + 12 * info["n_basis_cols"] + 8 * info["n_dofs"]
    near_ms = phases["near"]
    res = {"metric": "VtV coefficient-potentials/s, degree-p leaf bases p_l = L - l, FP64, 1 GPU",
           "unit": "coefficient-potentials/s", "workload": "unit cube BC octree h=1/%d (L=%d), %d leaves, %d basis "
           "coefficients (degrees 0..%d), q=%d, projected Gaussian-mixture density seed 0, near field assembled, "
           "1 stream" % (2 ** L, L, nl, info["n_dofs"], int(L - lv[:, 0].min()), args.q),
           "value": info["n_dofs"] / (ms * 1e-3), "cell_potentials_per_s": nl / (ms * 1e-3), "ms_per_apply": ms,
           "phase_ms": phases, "plan_seconds": plan_s, "plan_device_bytes": info["device_bytes"],
           "n_near_pairs": info["n_near"], "n_block_entries": info["n_basis_vals"],
           "n_block_columns": info["n_basis_cols"],
           "near_roofline": {"bound": "hbm", "bytes": near_bytes, "ms": near_ms,
                             "achieved": near_bytes / (near_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                             "frac": near_bytes / (near_ms * 1e-3) / PEAK_HBM}}
    if sched is not None:
        res["level_orders"] = sched
    del plan
    return res


def batched(args):
    """64 BC meshes, h drawn from {1/16, 1/32, 1/64} (default_rng(1234)), mesh m mapped to the ball
    iff m is odd (the others unit cubes; --cubes-only: all cubes), Gaussian-mixture density of seed
    m on mesh m, mixed precision (FP32 interaction phase): one forest plan with the autotuned work
    decomposition, its apply captured in one HIP graph. Reported against the same meshes applied one
    plan at a time, with the per-phase times of the forest's eager apply."""
    import torch

    import paper_2112_00864_amd as bcv
    import synth

    n_mesh = 64
    Ls = [int(L) for L in np.random.default_rng(1234).choice([4, 5, 6], n_mesh)]
    geoms = [bcv.GEOM_BOX if (args.cubes_only or m % 2 == 0) else bcv.GEOM_BALL for m in range(n_mesh)]
    if geoms.count(bcv.GEOM_BALL) and args.nearfield != "assembled":
        raise SystemExit("ball meshes need the assembled near field")
    t0 = time.perf_counter()
    print("batched: %d meshes (%d balls), building the forest" % (n_mesh, geoms.count(bcv.GEOM_BALL)), flush=True)
    forest = bcv.build_bc_forest(Ls, geometry=geoms)
    lv = forest.leaves().astype(np.int64)
    mesh = forest.leaf_mesh()
    f = np.empty(len(lv))
    for m in range(n_mesh):
        sel = mesh == m
        loc = lv[sel].copy()
        loc[:, 1] -= (4 * m) << loc[:, 0]
        f[sel] = synth.leaf_density(loc, seed=m)
    nf = bcv.NEAR_ASSEMBLED if args.nearfield == "assembled" else bcv.NEAR_QUADRATURE
    t1 = time.perf_counter()
    first = bcv.plan_interactions(forest, q=args.q, precision=bcv.MIXED_F32, nearfield=nf)
    first_plan_s = time.perf_counter() - t1
    del first
    print("batched: %d leaves, first plan %.1f s; autotuning" % (len(lv), first_plan_s), flush=True)
    tune, tune_ms = bcv.autotune(forest, n_applies=5, q=args.q, precision=bcv.MIXED_F32, nearfield=nf)
    plan = bcv.plan_interactions(forest, q=args.q, precision=bcv.MIXED_F32, nearfield=nf, **tune)
    setup_s = time.perf_counter() - t0
    print("batched: tuned %s in %.1f s total setup" % (tune, setup_s), flush=True)
    n = plan.n_leaves
    fd = torch.tensor(f, device="cuda:0")
    ud = torch.empty_like(fd)
    graph = bcv.vtv_graph_create(plan, fd, ud)
    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.launch()
    torch.cuda.synchronize()
    ms_graph = 1e3 * (time.perf_counter() - t0) / args.steps
    u_graph = ud.cpu().numpy()
    _, phase_ms = timed_applies(bcv, torch, plan, fd, ud, 1, args.steps, torch.device("cuda:0"))
    print("batched: graph %.3f ms per apply; planning the meshes one by one" % ms_graph, flush=True)
    if args.no_separate:
        print(json.dumps({"batched_ms_per_step": ms_graph, "phase_ms": phase_ms}), flush=True)
        return
    # the same meshes, one plan and one apply each
    plans = [bcv.plan_interactions(bcv.build_bc_tree(L, geometry=g), q=args.q, precision=bcv.MIXED_F32,
                                   nearfield=nf)
             for L, g in zip(Ls, geoms)]
    fs = [torch.tensor(f[mesh == m], device="cuda:0") for m in range(n_mesh)]
    us = [torch.empty_like(x) for x in fs]
    for p_, f_, u_ in zip(plans, fs, us):
        bcv.vtv_apply(p_, f_, u_)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for p_, f_, u_ in zip(plans, fs, us):
            bcv.vtv_apply(p_, f_, u_)
    torch.cuda.synchronize()
    ms_seq = 1e3 * (time.perf_counter() - t0) / args.steps
    worst = 0.0
    for m in range(n_mesh):
        a, b = u_graph[mesh == m], us[m].cpu().numpy()
        w = 0.125 ** lv[mesh == m, 0].astype(np.float64)
        worst = max(worst, float(np.sqrt(np.sum((a - b) ** 2 / w) / np.sum(b ** 2 / w))))
    line = {
        "metric": METRIC,
        "value": n / (ms_graph * 1e-3),
        "unit": "cell-potentials/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batched VtV: 64 BC meshes, h in {1/16,1/32,1/64} drawn by default_rng(1234), %s, "
                               "Gaussian-mixture density seed m on mesh m, q=%d, mixed FP32 interaction phase, "
                               "near field %s, one forest plan, apply captured in one HIP graph"
                               % ("all unit cubes" if args.cubes_only else
                                  "odd meshes cube-to-ball mapped, even meshes unit cubes", args.q, args.nearfield),
                   "n_leaves": n, "meshes_by_h": {"1/%d" % (2 ** L): Ls.count(L) for L in (4, 5, 6)},
                   "ball_meshes": geoms.count(bcv.GEOM_BALL),
                   "ball_leaves": int(sum(int(np.sum(mesh == m)) for m in range(n_mesh) if geoms[m] == bcv.GEOM_BALL)),
                   "autotuned": tune, "autotune_ms": tune_ms, "setup_seconds": setup_s,
                   "first_plan_seconds": first_plan_s},
        "phase_ms": phase_ms,
        "n_interaction_pairs": plan.info["n_m2l"],
        "separate_plans_ms_per_step": ms_seq,
        "speedup_vs_separate_plans": ms_seq / ms_graph,
        "max_rel_l2_vs_separate_plans": worst,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=8, help="finest level of the timed mesh (h = 2^-L)")
    ap.add_argument("--extras-L", type=int, default=7,
                    help="finest level of the extra measurements (plain FP64 config, BtV/VtB, level-dependent "
                         "orders, neighbour marking); 0 skips them all")
    ap.add_argument("--q", type=int, default=6)
    ap.add_argument("--basis-L", type=int, default=7,
                    help="finest level of the degree-p leaf basis measurement (0 skips it)")
    ap.add_argument("--nearfield", choices=["quadrature", "assembled"], default="assembled",
                    help="near-field entries stored once at plan time (assembled) or evaluated in every "
                         "apply (quadrature); the other mode is measured too and reported beside")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both",
                    help="both: time the FP64 and the mixed path on the same mesh and report the ratio")
    ap.add_argument("--streams", type=int, choices=[1, 2], default=2,
                    help="2: near field concurrent with the far field on a second stream")
    ap.add_argument("--cpu-targets", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="mixed path without the touching-pair surrogate")
    ap.add_argument("--surrogate-pairs", type=int, default=2000000,
                    help="training pairs of the touching-pair surrogate (generated and labelled on the GPU)")
    ap.add_argument("--no-split16", action="store_true",
                    help="skip the mixed apply with the interaction phase on the matrix cores")
    ap.add_argument("--no-btv", action="store_true", help="skip the BtV (Algorithm 3) measurement")
    ap.add_argument("--no-schedule", action="store_true",
                    help="skip the level-dependent expansion order measurement")
    ap.add_argument("--no-marking", action="store_true",
                    help="skip the neighbour-marking / level-dependent near-field measurement")
    ap.add_argument("--batched", action="store_true",
                    help="the batched workload: 64 meshes in one forest plan and one graph launch")
    ap.add_argument("--no-separate", action="store_true",
                    help="batched workload: skip the comparison with one plan per mesh (profiling runs)")
    ap.add_argument("--cubes-only", action="store_true",
                    help="batched workload with every mesh a unit cube (default: odd meshes are balls)")
    ap.add_argument("--near-only", action="store_true",
                    help="only run `steps` near-field applies (PART_NEAR) of the mixed plan on the --L mesh, for "
                         "counter collection, and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": n * 8}))
        return
    if args.near_only:
        import torch

        import paper_2112_00864_amd as bcv
        import synth

        tree = bcv.build_bc_tree(args.L)
        f = torch.tensor(synth.leaf_density(tree.leaves(), seed=0), device="cuda:0")
        u = torch.empty_like(f)
        plan = bcv.plan_interactions(tree, q=args.q, precision=bcv.MIXED_F32, nearfield=bcv.NEAR_ASSEMBLED, streams=1)
        for _ in range(args.steps):
            bcv.vtv_apply_parts(plan, f, u, bcv.PART_NEAR)
        torch.cuda.synchronize()
        print(json.dumps({"near_only_applies": args.steps, "L": args.L}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a batch of meshes would "
              "shard by mesh, one large mesh by Morton range of leaves)", file=sys.stderr)
        sys.exit(2)

    if args.batched:
        batched(args)
        return

    import torch

    import paper_2112_00864_amd as bcv
    import synth

    dev = 0
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    tree = bcv.build_bc_tree(args.L)
    leaves = tree.leaves()
    tree_s = time.perf_counter() - t0
    f = torch.tensor(synth.leaf_density(leaves, seed=0), device="cuda:%d" % dev)
    n = len(leaves)
    nf = bcv.NEAR_ASSEMBLED if args.nearfield == "assembled" else bcv.NEAR_QUADRATURE
    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]

    surrogate, sur_report = None, None
    if "mixed" in precisions and not args.no_surrogate:
        # touching-pair surrogate for the mixed path, trained on the GPU (not timed)
        t0 = time.perf_counter()
        surrogate = bcv.mlp_create(width=128, seed=1, device=dev)
        epochs = max(2, min(20, (20 * 100000) // args.surrogate_pairs))  # about 2e6 pair-visits in all
        sur_report = surrogate.train(n_train=args.surrogate_pairs, n_valid=20000, epochs=epochs, batch=2048, lr=2e-3,
                                     seed=42, n_gauss_lo=5, n_gauss_hi=16, tol=SURROGATE_TOL)
        sur_report["train_seconds"] = time.perf_counter() - t0
        sur_report["n_train"] = args.surrogate_pairs
        sur_report["epochs"] = epochs
        print("surrogate trained: %s" % json.dumps(sur_report), file=sys.stderr, flush=True)

    runs = {}
    for prec in precisions:
        runs[prec] = measure(bcv, torch, tree, f, args, dev, nf, prec, surrogate if prec == "mixed" else None)
        r = runs[prec]
        print("%s: plan %.1f s, step %.3f ms; phases (ms): %s"
              % (prec, r["plan_s"], r["ms"], json.dumps({k: round(v, 4) for k, v in r["phases"].items()})),
              file=sys.stderr, flush=True)

    rel_l2 = None
    if "fp64" in runs and "mixed" in runs:
        a, b = runs["mixed"]["u"], runs["fp64"]["u"]
        # relative L2(Omega) error of the cell averages (cell volume weights)
        w = 0.125 ** leaves[:, 0].astype(np.float64)
        avg_a, avg_b = a / w, b / w
        rel_l2 = float(np.sqrt(np.sum(w * (avg_a - avg_b) ** 2) / np.sum(w * avg_b ** 2)))
    # Headline: the mixed path when it meets the error gate against the FP64 path, else FP64.
    head = "mixed" if ("mixed" in runs and rel_l2 is not None and rel_l2 <= REL_L2_GATE) else precisions[-1]
    if args.precision == "both" and head != "mixed":
        print("mixed path missed the rel-L2 gate (%s): reporting FP64" % rel_l2, file=sys.stderr, flush=True)
    h = runs[head]
    info = h["info"]  # the headline plan's (the packing, and so its lane counts, depends on the precision)

    cpu = None
    if not args.no_cpu:
        u_ref = runs["fp64"]["u"] if "fp64" in runs else h["u"]
        cpu = cpu_baseline(args.L, args.q, f.cpu().numpy(), u_ref, args.cpu_targets, leaves)

    line = {
        "metric": METRIC,
        "value": n / (h["ms"] * 1e-3),
        "unit": "cell-potentials/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "VtV apply, BC-FMM, unit cube BC octree h=1/%d (L=%d), %d leaves, q=%d, Gaussian-mixture "
                        "density seed 0, near field %s, %d stream(s), %s"
                        % (2 ** args.L, args.L, n, args.q, args.nearfield, args.streams,
                           ("mixed FP32 M2L and far near field, FP64 singular pairs and accumulation"
                            + (", touching classes from the surrogate" if surrogate is not None else ""))
                           if head == "mixed" else "plain FP64"),
            "n_leaves": n,
            "q": args.q,
            "n_near_pairs": info["n_near"],
            "n_touching_pairs": info["n_touch"],
            "n_m2l_pairs": info["n_m2l"],
            "m2l_lane_efficiency": info["n_m2l"] / max(info["n_m2l_lanes"], 1),
            "m2l_read_fraction": info["n_m2l_read_lanes"] / max(info["n_m2l_lanes"], 1),
            "tree_seconds": tree_s,
            "plan_seconds": h["plan_s"],
            "plan_device_bytes": h["info"]["device_bytes"],
        },
        "phase_ms": h["phases"],
        "phase_ms_serial": h["phases_serial"],
        "roofline": h["roof"],
        "roofline_other": h["roof_other"],
        "cpu_baseline": cpu,
    }
    if "fp64" in runs:
        line["fp64"] = {"value": n / (runs["fp64"]["ms"] * 1e-3), "ms_per_step": runs["fp64"]["ms"],
                        "phase_ms": runs["fp64"]["phases"], "roofline": runs["fp64"]["roof"]}
    if rel_l2 is not None:
        line["mixed_vs_fp64"] = {"rel_l2": rel_l2, "gate": REL_L2_GATE,
                                 "speedup": runs["fp64"]["ms"] / runs["mixed"]["ms"]}
    # the same headline path with the other near-field mode (not the headline; for comparison)
    other = "quadrature" if args.nearfield == "assembled" else "assembled"
    other_nf = bcv.NEAR_QUADRATURE if other == "quadrature" else bcv.NEAR_ASSEMBLED
    r_o = measure(bcv, torch, tree, f, args, dev, other_nf, head, surrogate if head == "mixed" else None)
    line["other_near_mode"] = {"nearfield": other, "value": n / (r_o["ms"] * 1e-3), "ms_per_step": r_o["ms"],
                               "phase_ms": r_o["phases"], "phase_ms_serial": r_o["phases_serial"],
                               "plan_seconds": r_o["plan_s"], "plan_device_bytes": r_o["info"]["device_bytes"],
                               "max_rel_diff_vs_headline": float(np.max(np.abs(r_o["u"] - h["u"]) / np.abs(h["u"])))}
    print("%s with near field %s: step %.3f ms" % (head, other, r_o["ms"]), file=sys.stderr, flush=True)
    if "mixed" in runs and args.q == 6 and not args.no_split16:
        # the same mixed apply with the interaction phase on the matrix cores (split FP16)
        r16 = measure(bcv, torch, tree, f, args, dev, nf, "split16", surrogate)
        u16 = r16["u"]
        w = 0.125 ** leaves[:, 0].astype(np.float64)
        ref64 = runs["fp64"]["u"] if "fp64" in runs else None
        line["matrix_cores"] = {
            "precision": "BCV_MIXED_SPLIT16: interaction phase as v_mfma_f32_16x16x32_f16 with FP16 hi/lo "
                         "operands (3 products, FP32 accumulation); the rest as the mixed path",
            "value": n / (r16["ms"] * 1e-3), "ms_per_step": r16["ms"], "phase_ms": r16["phases"],
            "phase_ms_serial": r16["phases_serial"], "roofline": r16["roof"],
            "rel_l2_vs_fp64": None if ref64 is None else float(
                np.sqrt(np.sum(w * ((u16 - ref64) / w) ** 2) / np.sum(w * (ref64 / w) ** 2))),
            "vs_headline_mixed": runs["mixed"]["ms"] / r16["ms"]}
        print("split16: step %.3f ms; phases %s" % (r16["ms"], json.dumps(r16["phases_serial"])), file=sys.stderr,
              flush=True)
    if surrogate is not None:
        line["surrogate"] = {"classes_from_network": runs["mixed"]["info"]["surrogate_classes"], "of": 6,
                             "tol": SURROGATE_TOL, "training": sur_report}
    if args.extras_L:
        # extras on the h = 1/128 mesh: the plain FP64 workload (its own configuration), BtV/VtB,
        # level-dependent orders and the neighbour marking
        xargs = argparse.Namespace(**vars(args))
        xargs.L = args.extras_L
        xtree = bcv.build_bc_tree(xargs.L)
        xleaves = xtree.leaves()
        xf = torch.tensor(synth.leaf_density(xleaves, seed=0), device="cuda:%d" % dev)
        r64 = measure(bcv, torch, xtree, xf, xargs, dev, nf, "fp64")
        line["plain_fp64_h%d" % (2 ** xargs.L)] = {
            "workload": "VtV apply, unit cube BC octree h=1/%d (L=%d), %d leaves, q=%d, Gaussian-mixture density "
                        "seed 0, plain FP64, near field %s, %d stream(s)"
                        % (2 ** xargs.L, xargs.L, len(xleaves), args.q, args.nearfield, args.streams),
            "value": len(xleaves) / (r64["ms"] * 1e-3), "unit": "cell-potentials/s", "ms_per_step": r64["ms"],
            "phase_ms": r64["phases"], "phase_ms_serial": r64["phases_serial"], "roofline": r64["roof"],
            "roofline_other": r64["roof_other"], "plan_seconds": r64["plan_s"]}
        print("plain FP64 h=1/%d: step %.3f ms" % (2 ** xargs.L, r64["ms"]), file=sys.stderr, flush=True)
        if not args.no_btv:
            line["btv"] = measure_btv(bcv, torch, xtree, xf, xargs, dev)
            print("btv: %s" % json.dumps({k: line["btv"][k] for k in ("fp64", "mixed", "mixed_vs_fp64_rel_l2",
                                                                      "representation_formula_rel_err",
                                                                      "vtb_mixed_vs_fp64_rel")}),
                  file=sys.stderr, flush=True)
        if not args.no_schedule:
            sched = measure_schedule(bcv, torch, xtree, xf, xargs, dev, r64["u"])
            if sched is not None:
                line["level_orders"] = sched
                print("level orders: %s" % json.dumps(sched), file=sys.stderr)
        if not args.no_marking:
            line["neighbour_marking"] = measure_marking(bcv, torch, xargs, dev)
            print("neighbour marking: %s" % json.dumps(line["neighbour_marking"]), file=sys.stderr)
    if args.basis_L:
        line["degree_bases"] = measure_basis(bcv, torch, args, dev)
        print("degree bases: %s" % json.dumps(line["degree_bases"]), file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
