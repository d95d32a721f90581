"""Summarise rocprofv3 CSV output into the short text summaries kept under profiles/.

    python -m paper_2103_14915_amd.profile_summary --stats DIR/c2_kernel_stats.csv \\
        --fetch DIR/c2_counter_collection.csv --write DIR/c2_counter_collection.csv \\
        --copy-fetch DIR/copy_counter_collection.csv --copy-write DIR/copy_counter_collection.csv \\
        --copy-bytes 1073741824 --kernel k_process --command "..." --out profiles/NAME.md

HBM traffic of a kernel = its FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
each scaled by the factor that makes the same counter read the true byte count
of a plain device-to-device copy of known size.  Optional passes add the L2
hit rate (TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)), the share of wave
cycles spent waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES), and the copy's own
achieved bandwidth (the calibration run's JSON line).  Given the bench output
of the two counter runs (--fetch-log, --write-log), the traffic is also put
against the algorithmic bytes those runs report, per run: the number of passes
(launches) of a run can differ from run to run, the work per step does not.
The summary records
the hash of the kernel's source so that bench.py reports these figures only
while the kernel is unchanged.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources each pass kernel is built from
KERNEL_SOURCES = {
    "k_process": ("fork_pass.hip", "fork_util.h", "fork_dev.h", "fork_sched.h", "fork_mlp.h"),
    "k_gprocess": ("fork_group.hip", "fork_util.h", "fork_dev.h", "fork_sched.h"),
}


def kernel_source_hash(kernel: str = "k_process") -> str:
    h = hashlib.sha1()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def per_kernel(path, counter=None):
    agg = defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(path)):
        if counter and r.get("Counter_Name") != counter:
            continue
        name = r["Kernel_Name"] if "Kernel_Name" in r else r["Name"]
        agg[name][0] += 1
        agg[name][1] += float(r.get("Counter_Value", 0.0))
    return agg


def _bench_alg_bytes(path):
    """Algorithmic bytes of the profiled step from a bench run's JSON line."""
    for ln in open(path):
        ln = ln.strip()
        if ln.startswith("{") and '"roofline"' in ln:
            return json.loads(ln)["roofline"].get("algorithmic_bytes_per_step")
    return None


def pick(agg, key):
    for k, v in agg.items():
        if key in k:
            return k, v
    raise KeyError(key)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--copy-kernel", default="copyBuffer")
    ap.add_argument("--copy-log", help="stdout of the copy calibration run (its JSON line has copy_gbs)")
    ap.add_argument("--fetch-log", help="stdout of the FETCH_SIZE run (its bench line gives the step's algorithmic bytes)")
    ap.add_argument("--write-log", help="stdout of the WRITE_SIZE run")
    ap.add_argument("--tcc", help="counter CSV with TCC_HIT_sum and TCC_MISS_sum")
    ap.add_argument("--sq", help="counter CSV with SQ_WAIT_ANY and SQ_WAVE_CYCLES")
    ap.add_argument("--kernel", default="k_process")
    ap.add_argument("--command", default="")
    ap.add_argument("--title", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    rows = list(csv.DictReader(open(a.stats)))
    lines = [f"# {a.title or os.path.basename(a.out)}", "", f"Command: `{a.command}`", "",
             "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        lines.append(f"| {r['Name'][:70]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    out = {"kernel": a.kernel, "source_hash": kernel_source_hash(a.kernel)}
    kname, kstat = next(((r["Name"], r) for r in rows if a.kernel in r["Name"]), (None, None))
    if kstat:
        out["avg_launch_ms"] = float(kstat["AverageNs"]) / 1e6
        out["calls"] = int(kstat["Calls"])
        # the profiled command runs one step: the kernel's time per step (the number of launches,
        # and so the average per launch, varies between runs; the time per step does not)
        out["kernel_ms_total"] = float(kstat["TotalDurationNs"]) / 1e6
    if a.fetch and a.write and a.copy_fetch and a.copy_write and a.copy_bytes:
        _, (cn, cf) = pick(per_kernel(a.copy_fetch, "FETCH_SIZE"), a.copy_kernel)
        _, (cn2, cw) = pick(per_kernel(a.copy_write, "WRITE_SIZE"), a.copy_kernel)
        f_scale = a.copy_bytes / (cf / cn * 1024.0)
        w_scale = a.copy_bytes / (cw / cn2 * 1024.0)
        _, (n1, kf) = pick(per_kernel(a.fetch, "FETCH_SIZE"), a.kernel)
        _, (n2, kw) = pick(per_kernel(a.write, "WRITE_SIZE"), a.kernel)
        fetch_b = kf / n1 * 1024.0 * f_scale
        write_b = kw / n2 * 1024.0 * w_scale
        out.update({"fetch_scale": f_scale, "write_scale": w_scale, "fetch_bytes_per_launch": fetch_b,
                    "write_bytes_per_launch": write_b, "traffic_bytes_per_launch": fetch_b + write_b})
        lines += ["", f"HBM traffic of `{a.kernel}` per launch (FETCH_SIZE x {f_scale:.3f} + WRITE_SIZE x "
                      f"{w_scale:.3f}; scales from a {a.copy_bytes} B device copy): "
                      f"fetch {fetch_b / 1e6:.1f} MB, write {write_b / 1e6:.1f} MB, "
                      f"total {(fetch_b + write_b) / 1e6:.1f} MB over {n1} launches."]
        if a.fetch_log and a.write_log:
            fa, wa = _bench_alg_bytes(a.fetch_log), _bench_alg_bytes(a.write_log)
            if fa and wa:
                fr, wr = fetch_b * n1 / fa, write_b * n2 / wa
                out.update({"fetch_over_algorithmic": fr, "write_over_algorithmic": wr,
                            "traffic_over_algorithmic": fr + wr})
                lines += ["", f"Against the algorithmic bytes of the same runs ({fa / 1e9:.1f} GB and {wa / 1e9:.1f} GB "
                              f"per step): fetch {fr:.2f}x, write {wr:.2f}x, total {fr + wr:.2f}x."]
    if a.tcc:
        _, (_, hit) = pick(per_kernel(a.tcc, "TCC_HIT_sum"), a.kernel)
        _, (_, miss) = pick(per_kernel(a.tcc, "TCC_MISS_sum"), a.kernel)
        out["l2_hit_rate"] = hit / (hit + miss) if hit + miss else None
        lines += ["", f"L2 hit rate of `{a.kernel}` (TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)): "
                      f"{100.0 * out['l2_hit_rate']:.1f}%."]
    if a.sq:
        _, (_, wait) = pick(per_kernel(a.sq, "SQ_WAIT_ANY"), a.kernel)
        _, (_, cyc) = pick(per_kernel(a.sq, "SQ_WAVE_CYCLES"), a.kernel)
        out["wave_wait_share"] = wait / cyc if cyc else None
        lines += ["", f"Wave cycles of `{a.kernel}` spent waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES): "
                      f"{100.0 * out['wave_wait_share']:.1f}%."]
    if a.copy_log:
        for ln in open(a.copy_log):
            ln = ln.strip()
            if ln.startswith("{") and "copy_gbs" in ln:
                out["copy_gbs"] = json.loads(ln)["copy_gbs"]
        if "copy_gbs" in out:
            lines += ["", f"Achieved bandwidth of the plain device copy (read + write bytes / time): "
                          f"{out['copy_gbs']:.0f} GB/s."]
    lines += ["", "```json", json.dumps(out, indent=1), "```", ""]
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
