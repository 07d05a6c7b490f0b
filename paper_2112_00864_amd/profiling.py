"""rocprofv3 summaries for the roofline report.

* summarize_stats(): per-kernel call count and average duration from a --kernel-trace --stats
  CSV (<name>_kernel_stats.csv).
* counter_per_dispatch(): mean of one PMC counter per dispatch of a kernel from a --pmc CSV
  (<name>_counter_collection.csv), in KiB as rocprofv3 reports FETCH_SIZE / WRITE_SIZE.
* HBM traffic of a kernel = FETCH_SIZE * f_fetch + WRITE_SIZE * f_write, where each factor is
  (bytes a plain device copy of known size moves) / (what the same counter reads for that copy).
* The committed summaries under profiles/ carry a machine-readable block; traffic_for() returns a
  kernel's traffic only if the kernel source file still has the hash recorded with the counters.
"""

import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "kernels.hip")


def source_hash(path=KERNEL_SOURCE):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def short_name(name):
    """'void bcv::(anonymous namespace)::m2l_kernel<6>(int, ...)' -> 'm2l_kernel<6>'."""
    n = name.replace("bcv::(anonymous namespace)::", "").replace("void ", "")
    return n.split("(")[0].strip()


def summarize_stats(path):
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            out[short_name(r["Name"])] = {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                                          "total_ns": float(r["TotalDurationNs"]),
                                          "percent": float(r["Percentage"])}
    return out


def counter_per_dispatch(path, counter):
    acc = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def copy_factor(path, counter, copy_bytes):
    """Bytes per counter KiB, from the device copies of a calibration run (largest reading)."""
    vals = counter_per_dispatch(path, counter)
    kib = max(v for k, v in vals.items() if "copy" in k.lower() or "elementwise" in k.lower())
    return copy_bytes / kib


def traffic_for(kernel, L=None, q=None):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None if it is stale (the
    kernel source changed since), absent, or was taken on another mesh level or order."""
    path = os.path.join(PROFILES, "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    if data.get("kernel_source_sha256") != source_hash():
        return None
    if (L is not None and data.get("L") != L) or (q is not None and data.get("q") != q):
        return None
    entry = data.get("kernels", {}).get(kernel)
    return None if entry is None else entry["traffic_bytes_per_launch"]


def _csv(d, suffix):
    """The rocprofv3 CSV with the given suffix under output directory d (searched recursively)."""
    for root, _, files in os.walk(d):
        for f in sorted(files):
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError("no *%s under %s" % (suffix, d))


def write_trace_summary(stats_dir, out_md, title, command, note=""):
    """Markdown table of a --kernel-trace --stats run: calls and average duration per kernel."""
    st = summarize_stats(_csv(stats_dir, "kernel_stats.csv"))
    rows = sorted(st.items(), key=lambda kv: -kv[1]["total_ns"])
    lines = ["# " + title, "", "Command (MI355X, ROCm 7.2, committed files only):", "", "```", command, "```", ""]
    if note:
        lines += [note, ""]
    lines += ["| kernel | calls | avg (us) | total share |", "|---|---|---|---|"]
    for k, v in rows:
        lines.append("| `%s` | %d | %.1f | %.1f%% |" % (k, v["calls"], v["avg_ns"] / 1e3, v["percent"]))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def write_traffic_summary(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, copy_bytes, workload, L, q, out_json,
                          out_md, commands):
    """HBM bytes per launch from a FETCH_SIZE pass and a WRITE_SIZE pass, each scaled by what the
    same counter reads for a device copy of copy_bytes (read and written once)."""
    fetch = counter_per_dispatch(_csv(fetch_dir, "counter_collection.csv"), "FETCH_SIZE")
    write = counter_per_dispatch(_csv(write_dir, "counter_collection.csv"), "WRITE_SIZE")
    f_fetch = copy_factor(_csv(cal_fetch_dir, "counter_collection.csv"), "FETCH_SIZE", copy_bytes)
    f_write = copy_factor(_csv(cal_write_dir, "counter_collection.csv"), "WRITE_SIZE", copy_bytes)
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        fk, wk = fetch.get(k, 0.0), write.get(k, 0.0)
        kernels[k] = {"fetch_kib": fk, "write_kib": wk, "traffic_bytes_per_launch": fk * f_fetch + wk * f_write}
    data = {"workload": workload, "L": L, "q": q, "kernel_source_sha256": source_hash(),
            "fetch_bytes_per_kib": f_fetch, "write_bytes_per_kib": f_write,
            "calibration": "torch device copy of %d bytes" % copy_bytes, "kernels": kernels}
    with open(out_json, "w") as fh:
        json.dump(data, fh, indent=1)
    lines = ["# HBM traffic per launch (rocprofv3 PMC), " + workload, "",
             "Commands (one counter per run; MI355X, ROCm 7.2, committed files only):", "", "```"] + commands + [
        "```", "",
        "Calibration: a device copy of %d bytes (read once and written once) gives %.1f bytes per FETCH_SIZE KiB "
        "and %.1f bytes per WRITE_SIZE KiB; every kernel's bytes = FETCH_SIZE x %.1f + WRITE_SIZE x %.1f."
        % (copy_bytes, f_fetch, f_write, f_fetch, f_write), "",
        "Kernel source hash: `%s` (bench.py reports `traffic` only while csrc/kernels.hip has this hash and the "
        "mesh level and order match)." % data["kernel_source_sha256"], "",
        "| kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM bytes per launch |", "|---|---|---|---|"]
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["traffic_bytes_per_launch"]):
        lines.append("| `%s` | %.0f | %.0f | %.3f GB |" % (k, v["fetch_kib"], v["write_kib"],
                                                          v["traffic_bytes_per_launch"] / 1e9))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _main(argv=None):
    import argparse

    ap = argparse.ArgumentParser(description="Write the profiles/ summaries from rocprofv3 output directories.")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats_dir")
    t.add_argument("out_md")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--note", default="")
    w = sub.add_parser("traffic")
    for a in ("fetch_dir", "write_dir", "cal_fetch_dir", "cal_write_dir"):
        w.add_argument(a)
    w.add_argument("--copy-bytes", type=int, required=True)
    w.add_argument("--workload", required=True)
    w.add_argument("--L", type=int, required=True)
    w.add_argument("--q", type=int, required=True)
    w.add_argument("--out-json", default=os.path.join(PROFILES, "pmc_traffic.json"))
    w.add_argument("--out-md", required=True)
    w.add_argument("--command", action="append", default=[])
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        write_trace_summary(a.stats_dir, a.out_md, a.title, a.command, a.note)
    else:
        write_traffic_summary(a.fetch_dir, a.write_dir, a.cal_fetch_dir, a.cal_write_dir, a.copy_bytes, a.workload,
                              a.L, a.q, a.out_json, a.out_md, a.command)


if __name__ == "__main__":
    _main()
