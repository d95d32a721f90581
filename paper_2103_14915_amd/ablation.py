"""The paper's scheduling and yielding study, run on the GPU.

Section 6.4 studies the design choices one at a time.

- Table "priority" A: the inter-partition schedule, with yielding on. The
  schedules are Random, Max #operations, FIFO and the priority functor
  (Shortest).
- Table "priority" B: yield heuristic 1 (an edge budget per visit) at
  multiples of mu, with heuristic 2 off.
- Table "priority" C: yield heuristic 2 (a value range Delta above the
  query's best pending value) at multiples of Delta, with heuristic 1 off.
- B and C each end with a run that has no yielding at all.
- Figure "acc": the design choices switched on one after another.

Here every configuration runs the same seeded queries through the library's
run options, so only the schedule changes.

- **SSSP/BFS.** Each query's digest must equal the one from the priority
  run. Exact results do not depend on the schedule, so this is checked at
  full size.
- **PPR.** Results depend on the push order. The mean residual mass ||r||_1
  is reported beside the speed.

The mapping to run options:

- mu multiplies |E_P| / |Q_P| (the partition's edges over the queries
  visiting it in the pass), which is the paper's mu for one pass.
- Delta defaults to 64 mean edge weights. Heuristic 2 is off when the
  per-query window gate is off and the in-visit range is unbounded.
- The buffers always consolidate (the flush merges operations to the same
  vertex), so Figure "acc"'s +buffer and +consolidation steps are one step
  here.

    python -m paper_2103_14915_amd.ablation --workload grid2048_sssp1024_bfs1024 --queries 256
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import ForkGraph

NO_H2 = dict(window_mode=1, delta=2_000_000_000)  # no window gate, unbounded in-visit range


def configs(kinds, delta_unit: int) -> list:
    """(group, label, run options) of the study, in run order.

    The first entry is the reference run, the priority functor with default
    yielding."""
    sp = bool(kinds & {"sssp", "bfs"})
    out = [("A", "Shortest (priority functor)", dict(scheduler="priority"))]
    out += [("A", name, dict(scheduler=s)) for name, s in
            (("FIFO", "fifo"), ("Random", "random"), ("Max #operations", "maxops"))]
    for m in (0.25, 0.5, 1.0, 2.0, 4.0):
        out.append(("B", f"{m:g} mu", dict(scheduler="priority", edge_budget_mu=m, **(NO_H2 if sp else {}))))
    no_yield = dict(scheduler="priority", edge_budget_mu=0.0, **(NO_H2 if sp else {}))
    out.append(("B", "no yielding", no_yield))
    if sp:
        for m in (0.25, 0.5, 1.0, 2.0, 4.0):
            out.append(("C", f"{m:g} Delta", dict(scheduler="priority", delta=max(1, int(round(m * delta_unit))))))
        out.append(("C", "no yielding", no_yield))
        ladder_yield = ("+yield (heuristic 2, Delta)", dict(scheduler="priority"))
    else:
        ladder_yield = ("+yield (heuristic 1, 2 mu)", dict(scheduler="priority", edge_budget_mu=2.0))
    out.append(("acc", "+buffer +consolidation (FIFO, no yielding)",
                dict(no_yield, scheduler="fifo")))
    out.append(("acc", "+priority (no yielding)", no_yield))
    out.append(("acc",) + ladder_yield)
    return out


def _digests(fg, n):
    return [fg.digest(i) for i in range(n)]


def study(g, queries, spec, base: dict, steps: int = 1, warmup: int = 1, groups: str = "A,B,C,acc",
          log=print) -> list:
    """Run every configuration of the selected groups; one row per run."""
    import torch
    kinds = {qt for qt, _ in queries}
    wmean = float(g.weight.mean()) if g.weight is not None else 1.0
    delta_unit = max(1, int(round(64.0 * wmean)))
    want = set(groups.split(","))
    fg = ForkGraph.from_graph(g, partition_vertices=base["partition_vertices"])
    rows, ref = [], None
    try:
        n = 0
        types = []
        for qt, s in queries:
            fg.submit(qt, s, alpha=spec.get("alpha", 0.15), epsilon=spec.get("epsilon", 1e-6),
                      eps_mode=spec.get("eps_mode", 0))
            n += len(s)
            types += [qt] * len(s)
        exact = [i for i, t in enumerate(types) if t != "ppr"]
        ppr = [i for i, t in enumerate(types) if t == "ppr"]
        cfgs = configs(kinds, delta_unit)
        for k, (grp, label, opt) in enumerate(cfgs):
            if k > 0 and grp not in want:
                continue
            kw = dict(items_per_pass=base["items_per_pass"], window=base["window"], delta=base["delta"],
                      persistent=0, slice_slots=base.get("slice_slots", 0))
            kw.update(opt)
            for _ in range(warmup):
                fg.run(**kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fg.run(**kw)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            st = fg.stats()
            dg = _digests(fg, n)
            if ref is None:
                ref = dg
            same = all((dg[i]["count"], dg[i]["sum"], dg[i]["hash"]) ==
                       (ref[i]["count"], ref[i]["sum"], ref[i]["hash"]) for i in exact)
            row = {"group": grp, "config": label, "queries_per_s": n / dt, "ms_per_run": dt * 1e3,
                   "passes": st["passes"], "edges": st["edges"], "ops_emitted": st["ops_emitted"],
                   "yields": st["yields"], "sssp_bfs_identical": bool(same) if exact else None,
                   "ppr_mean_residual": float(np.mean([dg[i]["fres"] for i in ppr])) if ppr else None,
                   "options": {k2: v for k2, v in opt.items()}}
            rows.append(row)
            log(f"[ablation] {grp:3s} {label:44s} {row['queries_per_s']:10.1f} q/s  {row['ms_per_run']:9.1f} ms"
                f"  passes {st['passes']:6d}  edges {st['edges']:.3e}  identical {row['sssp_bfs_identical']}")
            if exact and not same:
                raise RuntimeError(f"{label}: SSSP/BFS results differ from the priority run")
    finally:
        fg.close()
    return rows


def markdown(rows: list) -> str:
    ref = rows[0]["queries_per_s"]
    out = ["| group | configuration | queries/s | ms per run | vs priority | passes | edges | exact |",
           "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        ex = {True: "identical", False: "DIFFERENT", None: "—"}[r["sssp_bfs_identical"]]
        if r["ppr_mean_residual"] is not None:
            ex += f"; mean ‖r‖₁ {r['ppr_mean_residual']:.3g}"
        out.append(f"| {r['group']} | {r['config']} | {r['queries_per_s']:.1f} | {r['ms_per_run']:.1f} | "
                   f"{r['queries_per_s'] / ref:.2f}× | {r['passes']} | {r['edges']:.3g} | {ex} |")
    return "\n".join(out)


def main(argv=None) -> int:
    import fpp_inputs as fi
    from . import autotune
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="grid2048_sssp1024_bfs1024")
    ap.add_argument("--queries", type=int, default=0, help="the first N queries of each type (0 = all)")
    ap.add_argument("--groups", default="A,B,C,acc")
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--json", default="", help="also write the rows to this file")
    args = ap.parse_args(argv)
    spec = fi.WORKLOADS[args.workload]
    g = fi.make_graph(spec)
    full = fi.make_sources(g, spec)
    queries = [(qt, s[:args.queries] if args.queries else s) for qt, s in full]
    base = autotune.cached(g, full) or dict(autotune.DEFAULTS)
    print(f"[ablation] {args.workload}, {sum(len(s) for _, s in queries)} queries, knobs {base}", flush=True)
    rows = study(g, queries, spec, base, steps=args.steps, warmup=args.warmup, groups=args.groups,
                 log=lambda *a: print(*a, flush=True))
    print(markdown(rows), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"workload": args.workload, "queries": sum(len(s) for _, s in queries), "knobs": base,
                       "rows": rows}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
