"""Benchmark of the VtV apply (BC-FMM volume potential) on one MI355X.

Workload: unit-cube BC octree with boundary leaves of side h = 1/128 (L = 7, 219,080 leaves),
expansion order q = 6, FP64 throughout, piecewise-constant Gaussian-mixture density (seed 0).
A step is one full VtV apply (Algorithm 1: moments, upward pass, interaction phase, downward
pass, near field and evaluation) with the density already resident in HBM. Plan construction
(lists, tables, workspace) happens once before timing and is reported separately.

Prints one JSON line with the metric, the per-phase device times from HIP events recorded on the
apply's stream, the roofline of the dominant kernel, and the CPU oracle's throughput on a bounded
sample of the same workload.
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
PEAK_HBM = 8.0e12  # bytes/s


def m2l_flops_per_pair(q):
    """Algorithmic flops of one interaction pair: one FMA (2 flops) per (alpha, beta), |alpha|+|beta| <= q."""
    from math import comb

    return 2 * comb(q + 6, 6)


def near_flops(info, q):
    """Algorithmic flops of the on-the-fly near field: 64 kernel evaluations per point-rule pair.

    Per evaluation: r^2 from per-axis squared differences (2 adds), reciprocal square root counted
    as 1 flop, accumulate (1 add): 4 flops; plus 12 subtractions and 12 multiplies per pair for the
    per-axis differences, and 1 FMA per touching pair.
    """
    n_rule = info["n_near"] - info["n_touch"]
    return n_rule * (64 * 4 + 24) + 2 * info["n_touch"]


def cpu_baseline(L, q, f, u_gpu, n_targets, leaves):
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
                  "h=1/128 q=6 workload, including the full moment and upward passes; mesh build %.1f s "
                  "excluded" % (n_targets, t1 - t0),
        "seconds": t2 - t1,
        "max_rel_diff_vs_gpu": err,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=7)
    ap.add_argument("--q", type=int, default=6)
    ap.add_argument("--nearfield", choices=["quadrature", "assembled"], default="quadrature")
    ap.add_argument("--streams", type=int, choices=[1, 2], default=2,
                    help="2: near field concurrent with the far field on a second stream")
    ap.add_argument("--cpu-targets", type=int, default=12)
    ap.add_argument("--no-cpu", action="store_true")
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
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the box has one MI355X and this build runs no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2112_00864_amd as bcv
    import synth

    dev = 0
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    tree = bcv.build_bc_tree(args.L)
    leaves = tree.leaves()
    nf = bcv.NEAR_ASSEMBLED if args.nearfield == "assembled" else bcv.NEAR_QUADRATURE
    plan = bcv.plan_interactions(tree, q=args.q, nearfield=nf, device=dev, streams=args.streams)
    plan_s = time.perf_counter() - t0
    info = plan.info
    n = info["n_leaves"]
    print("plan: %d leaves, %d near pairs, %d M2L pairs, %.1f s" % (n, info["n_near"], info["n_m2l"], plan_s),
          file=sys.stderr, flush=True)

    f = torch.tensor(synth.leaf_density(leaves, seed=0), device="cuda:%d" % dev)
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        bcv.vtv_apply(plan, f, u, stream)
    torch.cuda.synchronize()

    bcv.plan_enable_timing(plan, args.steps)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        bcv.vtv_apply(plan, f, u, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    phases, n_rec = bcv.plan_phase_times(plan)
    bcv.plan_enable_timing(plan, 0)
    ms_step = 1e3 * elapsed / args.steps
    phase_avg = {k: v / max(n_rec, 1) for k, v in phases.items()}
    u_host = u.cpu().numpy()
    print("step %.3f ms; phases (ms): %s" % (ms_step, json.dumps({k: round(v, 4) for k, v in phase_avg.items()})),
          file=sys.stderr, flush=True)

    # Roofline of the dominant kernel (per launch, averaged over the timed applies).
    m2l_ms = phase_avg["m2l"]
    near_ms = phase_avg["near"]
    m2l_fl = info["n_m2l"] * m2l_flops_per_pair(args.q)
    if args.nearfield == "assembled":
        near_bytes = info["n_near"] * (8 + 4 + 8) + n * (8 * 2 + 8 + 8 + 32)
        near_roof = {"bound": "hbm", "achieved": near_bytes / (near_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                     "unit": "GB/s"}
    else:
        near_fl = near_flops(info, args.q)
        near_roof = {"bound": "alu", "achieved": near_fl / (near_ms * 1e-3) / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s"}
    m2l_roof = {"bound": "alu", "achieved": m2l_fl / (m2l_ms * 1e-3) / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s"}
    from paper_2112_00864_amd import profiling

    m2l_name = "m2l_kernel<%d>" % args.q
    near_name = "near_eval_kernel<%d, %s>" % (args.q, "true" if args.nearfield == "assembled" else "false")
    for roof_, name in ((m2l_roof, m2l_name), (near_roof, near_name)):
        roof_["frac"] = roof_["achieved"] / roof_["peak"]
        roof_["traffic"] = profiling.traffic_for(name)  # HBM bytes per launch (PMC), None if stale
        roof_["kernel"] = name
    roof = m2l_roof if m2l_ms >= near_ms else near_roof

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.L, args.q, f.cpu().numpy(), u_host, args.cpu_targets, leaves)

    line = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "cell-potentials/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "VtV apply, plain FP64 BC-FMM, unit cube BC octree h=1/%d (L=%d), %d leaves, q=%d, "
                        "Gaussian-mixture density seed 0, near field %s, %d stream(s)"
                        % (2 ** args.L, args.L, n, args.q, args.nearfield, args.streams),
            "n_leaves": n,
            "q": args.q,
            "n_near_pairs": info["n_near"],
            "n_touching_pairs": info["n_touch"],
            "n_m2l_pairs": info["n_m2l"],
            "m2l_lane_efficiency": info["n_m2l"] / max(info["n_m2l_lanes"], 1),
            "plan_seconds": plan_s,
            "plan_device_bytes": info["device_bytes"],
        },
        "phase_ms": phase_avg,
        "roofline": roof,
        "roofline_other": {"m2l_kernel": m2l_roof, "near_eval_kernel": near_roof},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
