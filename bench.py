#!/usr/bin/env python3
"""Benchmark of the fork-processing hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one complete fork-processing run (state init + every pass of the
buffered execution until all buffers are empty) over the workload's whole
query batch, with the graph and sources already resident on the GPU.  The
default workload is the batched SSSP + PPR mix on R-MAT scale 20 (1,048,576
vertices, 16,777,216 edges, a/b/c/d = 0.57/0.19/0.19/0.05, weights uniform in
[1, 255]): 1,024 SSSP and 1,024 PPR forward-push queries (alpha = 0.15,
epsilon = 1e-6, push while r >= epsilon * outdeg), half of the sources
uniform and half among the top 1% by out-degree.

Prints one JSON line with queries/s under the priority rule, the learned
scheduler's speedup over it on the same queries (identical SSSP results
required), the dominant kernel's roofline figures and the CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "queries/sec for batched SSSP+PPR at 1 GPU; learned vs rule schedule speedup"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(st: dict) -> float:
    """Bytes the method must move for the work it did, counted on the device.

    SSSP/BFS: 4 B state read per edge relaxation + 4 B per improving write.
    PPR: 8 B residual read-modify-write per edge push + 24 B per vertex push
    (8 B p read-modify-write, 4 B residual reset, 8 B row bounds, 4 B degree).
    Edge data: (4 B target + weight bytes) per out-edge of every partition
    scheduled in a pass, shared by all of the pass's queries of that partition.
    Cross-partition operations: 24 B each (a 12 B <q, v, val> written and read
    back)."""
    sp_edges = st["edges"] - st["ppr_edges"]
    return (sp_edges * 4 + st["improved"] * 4 + st["ppr_edges"] * 8 + st["ppr_vertex_pushes"] * 24
            + st["selected_edges"] * (4 + st["weight_bytes"]) + st["ops_emitted"] * 24)


def measured_traffic(workload: str, kernel: str = "k_process", root: str = ""):
    """HBM bytes per launch of the pass kernel from the committed rocprofv3 summary
    of this workload, if that summary was taken from the current kernel source."""
    from paper_2103_14915_amd import profile_summary as ps
    root = root or os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", f"{kernel}_{workload}.md")
    try:
        text = open(path).read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_hash") != ps.kernel_source_hash(kernel) or "traffic_bytes_per_launch" not in blob:
        return None
    return blob


def certified_push(oracle, g, batch, alpha, eps, mode, target, threads):
    """The L1-certified mode on the CPU: the oracle's forward push, restarted
    with the GPU path's threshold rule until every query's ||r||_1 <= 0.9 * target."""
    eps = np.full(len(batch), float(eps))
    todo = np.arange(len(batch))
    while todo.size:
        left = []
        for e in np.unique(eps[todo]):
            sel = todo[eps[todo] == e]
            _, r = oracle.forward_push(g, batch[sel], alpha, e, mode, threads)
            r1 = r.sum(1)
            for k, q in enumerate(sel):
                if r1[k] > 0.9 * target:
                    eps[q] *= min(0.5, max(1e-3, 0.5 * 0.9 * target / r1[k]))
                    left.append(q)
        todo = np.asarray(left, np.int64)


def host_info():
    """CPU model and the cores this process may run on (the baseline's threads)."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    aff = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    spans, i = [], 0
    while i < len(aff):
        j = i
        while j + 1 < len(aff) and aff[j + 1] == aff[j] + 1:
            j += 1
        spans.append(f"{aff[i]}-{aff[j]}" if j > i else f"{aff[i]}")
        i = j + 1
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "affinity": ",".join(spans),
            "affinity_cpus": len(aff)}


def cpu_baseline(g, queries, spec, budget_s=15.0, l1_target=0.0):
    """The CPU oracle, untuned, one query per thread over all host cores."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    kinds = [(qt, s) for qt, s in queries]
    done, t_total = 0, 0.0
    rng = np.random.default_rng(0)
    samples = []
    work = {}  # query type -> [queries, edges the sequential algorithm scanned or pushed]
    while t_total < budget_s and done < sum(len(s) for _, s in kinds):
        for qt, s in kinds:
            batch = rng.choice(s, size=min(threads, len(s)), replace=False)
            t0 = time.perf_counter()
            w = None
            if qt == "ppr" and l1_target > 0:
                certified_push(oracle, g, batch, spec.get("alpha", 0.15), spec.get("epsilon", 1e-6),
                               spec.get("eps_mode", 0), l1_target, threads)
            elif qt == "ppr":
                _, _, w = oracle.forward_push(g, batch, spec.get("alpha", 0.15), spec.get("epsilon", 1e-6),
                                              spec.get("eps_mode", 0), threads, return_work=True)
            elif qt == "bfs":
                _, w = oracle.bfs(g, batch, threads, return_work=True)
            else:
                _, w = oracle.sssp(g, batch, threads, return_work=True)
            t_total += time.perf_counter() - t0
            done += len(batch)
            samples.append(f"{len(batch)} {qt}")
            if w is not None:
                acc = work.setdefault(qt, [0, 0])
                acc[0] += len(batch)
                acc[1] += int(np.sum(w))
    return {"value": done / t_total, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "host": host_info(),
            "sequential_edges_per_query": {qt: e / n for qt, (n, e) in work.items()},
            "sample": f"{done} queries ({', '.join(sorted(set(samples)))} per batch) of the same workload, "
                      f"{t_total:.1f} s, fp64 forward push / Dijkstra / BFS, one query per thread"
                      + (f"; PPR certified to L1 {l1_target:g} by restarted pushes at lower thresholds"
                         if l1_target > 0 else "")}


def compare_learned(fg, args, run_kw, nq, rule_value):
    """Time the learned scheduler on the same queries; SSSP/BFS digests must match the rule run's."""
    import paper_2103_14915_amd as fork
    import torch
    theta = np.load(args.compare_learned)
    kinds = fg.types
    rule_dig = [fg.digest(i) for i in range(nq)]
    kw = dict(run_kw, scheduler="learned", mlp_weights=theta)
    for _ in range(min(args.warmup, 1)):  # the rule run's first step paid the one-time allocations
        fg.run(**kw)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, args.learned_steps))
    t0 = time.perf_counter()
    for _ in range(steps):
        fg.run(**kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = fg.stats()
    learned_value = nq * steps / dt
    same = all((fg.digest(i)["hash"], fg.digest(i)["count"]) == (rule_dig[i]["hash"], rule_dig[i]["count"])
               for i in range(nq) if kinds[i] != fork.PPR)
    return {"rule_queries_per_s": rule_value, "learned_queries_per_s": learned_value,
            "speedup": learned_value / rule_value, "sssp_bfs_digests_identical": bool(same),
            "learned_passes_per_step": st["passes"], "learned_edges_per_step": st["edges"], "learned_steps": steps,
            "weights": os.path.basename(args.compare_learned)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 1 on the scale-23 batch, whose step takes over a minute; else 3)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default: 0 on the scale-23 batch; "
                    "else 1)")
    ap.add_argument("--workload", default="rmat23_sssp_ppr65536")
    ap.add_argument("--source-seed", type=int, default=-1,
                    help="draw the sources with this seed instead of the workload's (same graph, same query mix)")
    ap.add_argument("--scheduler", default="priority")
    ap.add_argument("--engine", default="", choices=["", "buffered", "grouped"],
                    help="buffered: one work item per (partition, query); grouped: per (partition, 64 queries); "
                         "default: the tuned choice")
    ap.add_argument("--parts-per-pass", type=int, default=0)
    ap.add_argument("--partition-vertices", type=int, default=0)
    ap.add_argument("--delta", type=int, default=0)
    ap.add_argument("--mu", type=float, default=0.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--scale", type=int, default=0, help="experiment: override the R-MAT scale")
    ap.add_argument("--queries", type=int, default=0, help="experiment: use only the first N queries per type")
    ap.add_argument("--max-queries", type=int, default=0, help="queries resident per wave (0 = auto)")
    ap.add_argument("--order", default="auto", choices=["auto", "none", "tiles", "rcm"],
                    help="internal vertex order: auto = square tiles for grids, the generator's order otherwise")
    ap.add_argument("--l1-target", type=float, default=0.0,
                    help="PPR queries in the L1-certified mode with this target (0 = plain push at epsilon)")
    ap.add_argument("--pool-mb", type=int, default=0, help="device memory for buffered operations (0 = auto)")
    ap.add_argument("--persistent", action="store_true", help="one persistent cooperative kernel per batch of passes")
    ap.add_argument("--items-per-pass", type=int, default=0, help="work items queued per pass (0 = auto)")
    ap.add_argument("--window-mode", type=int, default=0, help="heuristic-2 window: 0 = query-global, 1 = per visit")
    ap.add_argument("--window", type=int, default=0, help="SSSP batch width inside a visit (0 = auto)")
    ap.add_argument("--slice-slots", type=int, default=-1,
                    help="LDS slice: 0 = dense, else hash-table slots (-1 = tuned/default)")
    ap.add_argument("--tune", action="store_true", help="run the autotuner on a query sample first (cached)")
    ap.add_argument("--retune", action="store_true", help="with --tune: search again even if a result is cached")
    ap.add_argument("--tune-sample", type=int, default=1024, help="queries per autotuner trial")
    ap.add_argument("--no-tuned", action="store_true", help="ignore cached autotuner results")
    ap.add_argument("--tune-budget", type=float, default=240.0, help="seconds of autotuner trials")
    ap.add_argument("--tune-knobs", default="", help="comma-separated knobs to search (default: all)")
    ap.add_argument("--tune-from-cache", action="store_true",
                    help="with --tune: start from the cached knobs (e.g. a smaller subset's) and keep their engine")
    ap.add_argument("--compare-learned", default="auto", help="MLP weights (.npy): also time the learned scheduler "
                    "on the same workload and report the speedup over the rule-based one ('auto': the weights "
                    "shipped with the package for this graph family; 'none': skip)")
    ap.add_argument("--learned-steps", type=int, default=None,
                    help="timed steps of the learned scheduler (default: as --steps, at most 5)")
    ap.add_argument("--group-threads", type=int, default=0, help="grouped engine: workgroup size (256/512/1024)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 6,
                          "copy_gbs": 2.0 * n * 4 / (ms * 1e-3) / 1e9}), flush=True)
        return
    big = args.workload == "rmat23_sssp_ppr65536" and not (args.queries or args.scale)
    if args.steps is None:
        args.steps = 1 if big else 3
    if args.warmup is None:
        args.warmup = 0 if big else 1
    if args.learned_steps is None:
        args.learned_steps = min(args.steps, 5)
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU only; --gpus must be 1 "
                                   "(the queries would shard across GPUs with no exchange during a run)"}))
        sys.exit(2)

    import torch
    import fpp_inputs as fi
    import paper_2103_14915_amd as fork

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    spec = fi.WORKLOADS[args.workload]
    if args.source_seed >= 0:
        spec = dict(spec, seeds=(spec["seeds"][0], spec["seeds"][1], args.source_seed))
    t0 = time.perf_counter()
    g = fi.make_graph(spec, scale_override=args.scale or None)
    queries = fi.make_sources(g, spec)
    if args.queries:
        queries = [(qt, s[:args.queries]) for qt, s in queries]
    t_gen = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    # knobs: defaults <- autotuner (cached, or tuned now with --tune) <- explicit flags
    from paper_2103_14915_amd import autotune
    params, source = dict(autotune.DEFAULTS), "defaults"
    if not args.no_tuned:
        t_tune = time.perf_counter()
        start = autotune.cached(g, queries, spec) if args.tune_from_cache else None
        fixed = tuple(k for k in autotune.DEFAULTS if args.tune_knobs and k not in args.tune_knobs.split(","))
        tuned = autotune.tune(g, queries, spec, log=lambda *a: print(*a, file=sys.stderr, flush=True),
                              use_cache=not args.retune, sample=args.tune_sample, start=start,
                              fixed=fixed or (("engine",) if start else ()), budget_s=args.tune_budget) \
            if args.tune else autotune.cached(g, queries, spec)
        if tuned:
            tuned = dict(tuned)
            subset = tuned.pop("_tuned_on", None)
            params, source = tuned, ("tuned" if args.tune else "cache")
            if subset:
                source += f" (tuned on the query subset {subset} of this graph)"
            print(f"[bench] tuned params ({source}, {time.perf_counter() - t_tune:.1f}s): {params}",
                  file=sys.stderr, flush=True)
    for k, v in (("partition_vertices", args.partition_vertices), ("items_per_pass", args.items_per_pass),
                 ("window", args.window), ("delta", args.delta), ("persistent", int(args.persistent))):
        if v:
            params[k] = v
    if args.slice_slots >= 0:
        params["slice_slots"] = args.slice_slots
    if args.engine:
        params["engine"] = args.engine
    if args.mu:
        params["mu"] = args.mu
    if args.group_threads:
        params["group_threads"] = args.group_threads
    params = dict(autotune.DEFAULTS, **params)
    if params["engine"] == "grouped":
        params["persistent"] = 0
    from paper_2103_14915_amd import order as vorder
    t0 = time.perf_counter()
    if args.order == "auto":
        pos = vorder.auto(spec, g, params["partition_vertices"])
    elif args.order == "tiles":
        pos = vorder.grid_tiles(spec["rows"], spec["cols"], *vorder.tile_shape(params["partition_vertices"]))
    elif args.order == "rcm":
        pos = vorder.rcm(g)
    else:
        pos = None
    tr, tc = vorder.tile_shape(params["partition_vertices"])
    params["vertex_order"] = "none" if pos is None else ("rcm" if args.order == "rcm" else f"tiles{tr}x{tc}")
    t_order = time.perf_counter() - t0
    t0 = time.perf_counter()
    fg = fork.ForkGraph.from_graph(g, partition_vertices=params["partition_vertices"], max_queries=args.max_queries,
                                   pool_bytes=args.pool_mb << 20, vertex_order=pos)
    t_load = time.perf_counter() - t0
    nq = 0
    for qt, s in queries:
        fg.submit(qt, s, alpha=spec.get("alpha", 0.15), epsilon=spec.get("epsilon", 1e-6),
                  eps_mode=spec.get("eps_mode", 0), l1_target=args.l1_target)
        nq += len(s)
    kinds = sorted({qt for qt, _ in queries})
    kind = kinds[0] if len(kinds) == 1 else "mixed"
    run_kw = dict(autotune.run_kwargs(params), scheduler=args.scheduler, parts_per_pass=args.parts_per_pass,
                  stream=stream, profile=1, window_mode=args.window_mode)
    # device buffers of the run's waves, allocated before timing (fork_prepare): setup, like loading the graph
    t_prep = time.perf_counter()
    fg.prepare(**run_kw)
    t_prep = time.perf_counter() - t_prep
    for _ in range(args.warmup):
        fg.run(**run_kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = None
    t_call = 0.0
    step_ms = []
    for _ in range(args.steps):
        tc = time.perf_counter()
        fg.run(**run_kw)  # returns when every buffer is empty
        step_ms.append((time.perf_counter() - tc) * 1e3)
        t_call += step_ms[-1] / 1e3
        st = fg.stats()
        tot = st if tot is None else {k: tot[k] + st[k] if isinstance(st[k], (int, float))
                                      else [a + b for a, b in zip(tot[k], st[k])] if isinstance(st[k], list)
                                      else st[k] for k in st}
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for k in ("num_partitions", "weight_bytes"):
        tot[k] = st[k]
    value = nq * args.steps / dt
    abytes = algorithmic_bytes(tot)
    kernel = "k_gprocess" if params["engine"] == "grouped" else "k_process"
    prof = measured_traffic(args.workload, kernel) \
        if not (args.scale or args.queries or args.l1_target or args.source_seed >= 0) else None
    launches = max(1, tot["process_launches"])
    avg_ms = tot["process_ms"] / launches
    # HBM bytes per launch: the profiled traffic over algorithmic bytes (per run; the number of passes
    # varies between runs) times this run's algorithmic bytes per launch, else the profiled per-launch figure
    traffic = None
    if prof:
        traffic = (prof["traffic_over_algorithmic"] * abytes / launches if prof.get("traffic_over_algorithmic")
                   else prof["traffic_bytes_per_launch"])
    achieved = (abytes / launches) / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "+".join((["int32"] if {"sssp", "bfs"} & set(kinds) else []) + (["f32"] if "ppr" in kinds else [])),
        "data": "synthetic",
        "config": {"workload": args.workload + (f"@scale{args.scale}" if args.scale else "")
                   + (f"@sources{args.source_seed}" if args.source_seed >= 0 else "")
                   + (f"@q{args.queries}" if args.queries else "")
                   + (f"+l1cert{args.l1_target:g}" if args.l1_target > 0 else ""), "queries": nq, "types": kinds, "vertices": g.num_vertices,
                   "edges": g.num_edges, "partitions": tot["num_partitions"], "scheduler": args.scheduler, "engine": params["engine"], "knobs": params, "knobs_source": source,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_over_algorithmic": traffic / (abytes / launches) if traffic else None,
                     "profiled_avg_launch_ms": prof.get("avg_launch_ms") if prof else None,
                     "profiled_kernel_ms_per_step": prof.get("kernel_ms_total") if prof else None,
                     "kernel_ms_per_step": tot["process_ms"] / args.steps,
                     "l2_hit_rate": prof.get("l2_hit_rate") if prof else None,
                     "wave_wait_share": prof.get("wave_wait_share") if prof else None,
                     "achievable_copy_gbs": prof.get("copy_gbs") if prof else None,
                     "kernel": kernel,
                     "avg_launch_ms": avg_ms, "launches_per_step": launches / args.steps,
                     "algorithmic_bytes_per_launch": abytes / launches,
                     "algorithmic_bytes_per_step": abytes / args.steps},
        "detail": {"graph_gen_s": t_gen, "vertex_order_s": t_order, "graph_load_s": t_load,
                   "prepare_s": t_prep,
                   "run_wall_ms_per_step": tot["wall_ms"] / args.steps, "setup_ms_per_step": tot["setup_ms"] / args.steps,
                   "python_run_ms_per_step": t_call * 1e3 / args.steps,
                   "step_ms": step_ms, "step_ms_median": float(np.median(step_ms)),
                   "init_ms_per_step": tot["init_ms"] / args.steps, "run_ms_per_step": tot["run_ms"] / args.steps,
                   "process_ms_per_step": tot["process_ms"] / args.steps,
                   "passes_per_step": tot["passes"] / args.steps,
                   "edges_per_step": tot["edges"] / args.steps,
                   "ops_emitted_per_step": tot["ops_emitted"] / args.steps,
                   "ops_pruned_per_step": tot["pruned"] / args.steps,
                   "vertex_pushes_per_step": tot["vertex_pushes"] / args.steps,
                   "work_items_per_step": tot["work_items"] / args.steps,
                   "refine_rounds_per_step": tot["refine_rounds"] / args.steps,
                   "activations_per_step": tot["activations"] / args.steps,
                   "expansions_per_step": tot["expansions"] / args.steps,
                   "rounds_per_step": tot["rounds"] / args.steps, "edge_tasks_per_step": tot["edge_tasks"] / args.steps,
                   "ppr_edges_per_step": tot["ppr_edges"] / args.steps,
                   "ppr_vertex_pushes_per_step": tot["ppr_vertex_pushes"] / args.steps,
                   "improved_per_step": tot["improved"] / args.steps,
                   "visit_phase_share": ({n: v / max(1, sum(tot["visit_ns"])) for n, v in
                                          zip(("gather", "take", "filter", "tasks", "yield"), tot["visit_ns"])}
                                         if sum(tot["visit_ns"]) else None),
                   "spilled_per_step": tot["spilled"] / args.steps, "spill_max": st["spill_max"]},
    }
    if args.compare_learned == "auto":
        fam = "grid" if spec.get("kind") == "grid" else ""
        path = os.path.join(os.path.dirname(os.path.abspath(fork.__file__)), f"sched_mlp{'_' + fam if fam else ''}.npy")
        args.compare_learned = path if os.path.exists(path) else ""
    if args.compare_learned and args.compare_learned != "none":
        line["learned_vs_rule"] = compare_learned(fg, args, run_kw, nq, value)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(g, queries, spec, args.cpu_budget, args.l1_target)
        per_q = cb.pop("sequential_edges_per_query")
        line["cpu_baseline"] = cb
        # work efficiency: edges the GPU run scanned or pushed over the edges the
        # sequential algorithms (Dijkstra, BFS, sequential push) need for the same queries
        if per_q and all(qt in per_q for qt, _ in queries):
            seq = sum(len(s) * per_q[qt] for qt, s in queries)
            line["detail"]["sequential_edges_per_query"] = per_q
            line["detail"]["edges_vs_sequential"] = (tot["edges"] / args.steps) / seq if seq else None
    fg.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
