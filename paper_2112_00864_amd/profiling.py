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


def traffic_for(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None if stale/absent."""
    path = os.path.join(PROFILES, "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    if data.get("kernel_source_sha256") != source_hash():
        return None
    entry = data.get("kernels", {}).get(kernel)
    return None if entry is None else entry["traffic_bytes_per_launch"]
