"""Autotuner for the fork-processing pass.

Picks the knobs that the paper fixes by hand (Section 6.1: partition size =
LLC size; yield thresholds; one partition processed at a time) for the
MI355X: the engine (one query per work item, or 64 queries per work item in
vertex-major rows), partition size (vertices per LDS-staged slice), work
items queued per pass (how many visits run between two scheduling steps),
the SSSP batch window, the heuristic-2 range Delta and the heuristic-1 edge
budget mu, whether the pass loop runs in one persistent kernel, and the LDS
slice shape (dense, or a hash table of touched vertices that lets more
workgroups share a CU).  It times short runs on a seeded sample
of the workload's queries and does coordinate descent from the defaults.
Results are cached in JSON keyed by graph shape, query mix and device.

    from paper_2103_14915_amd import autotune
    params = autotune.tune(graph, [("sssp", sources), ...], spec)
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Optional

import numpy as np

from . import ForkGraph

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.environ.get("FORK_TUNE_CACHE", os.path.join(HERE, "tune_cache.json"))

DEFAULTS = {"engine": "buffered", "partition_vertices": 16384, "items_per_pass": 0, "window": 0, "delta": 0,
            "mu": 0.0, "persistent": 0, "slice_slots": 0, "group_threads": 0}
GROUPED_PVMAX = 16384  # largest partition the grouped engine visits


def valid(p) -> bool:
    """Knob combinations the library accepts."""
    if p.get("engine") == "grouped":  # the persistent kernel and the LDS slice shape belong to the other engine
        return p["partition_vertices"] <= GROUPED_PVMAX and not p["persistent"] and not p.get("slice_slots")
    return not p.get("group_threads")  # the workgroup size is a grouped-engine knob


def run_kwargs(p) -> dict:
    """fork_run keyword arguments of a knob set."""
    return dict(engine=p.get("engine", "buffered"), items_per_pass=p["items_per_pass"], window=p["window"],
                delta=p["delta"], edge_budget_mu=float(p.get("mu", 0.0)), persistent=p["persistent"],
                slice_slots=p.get("slice_slots", 0), group_threads=int(p.get("group_threads", 0)))


def device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:  # noqa: BLE001 - the name only keys the cache
        return "unknown"


def signature(g, queries, spec=None) -> str:
    """Cache key of a graph and query mix.  PPR queries with the absolute
    threshold (eps_mode 0) are marked 'ppr@abs': they push far more than the
    degree-scaled ones and tune differently."""
    h = hashlib.sha1()
    h.update(np.asarray([g.num_vertices, g.num_edges], np.int64).tobytes())
    h.update(np.ascontiguousarray(g.row_ptr[:: max(1, g.num_vertices // 4096)]).tobytes())
    if g.weight is not None:
        h.update(np.ascontiguousarray(g.weight[:4096]).tobytes())
    absolute = spec is not None and spec.get("eps_mode", 1) == 0
    mix = ",".join(f"{qt}{'@abs' if qt == 'ppr' and absolute else ''}:{len(s)}" for qt, s in queries)
    return f"V{g.num_vertices}-E{g.num_edges}-{mix}-{h.hexdigest()[:12]}"


def _load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _split(sig: str):
    """(graph part, {query type: count}, hash) of a cache signature."""
    head, mix, hsh = sig.split("-")[0:2], sig.split("-")[2:-1], sig.split("-")[-1]
    counts = {}
    for part in "-".join(mix).split(","):
        qt, _, n = part.partition(":")
        counts[qt] = int(n) if n.isdigit() else 0
    return "-".join(head), counts, hsh


def cached(g, queries, spec=None) -> Optional[dict]:
    """Tuned knobs for this graph and query mix: this device's entry, else any
    device's; else the entry tuned on the largest query subset of the same
    graph with the same query types (a batch too large to tune in full takes
    the knobs of a seeded subset of itself)."""
    cache = _load_cache()
    sig = signature(g, queries, spec)
    hit = cache.get(f"{sig}|{device_name()}")
    if hit is None:
        hit = next((v for k, v in cache.items() if k.split("|")[0] == sig), None)
    if hit is None:
        graph, counts, hsh = _split(sig)
        best = None
        for k, v in cache.items():
            g2, c2, h2 = _split(k.split("|")[0])
            if g2 == graph and h2 == hsh and set(c2) == set(counts) and all(c2[t] <= counts[t] for t in counts):
                n = sum(c2.values())
                if best is None or n > best[0]:
                    best = (n, v, ",".join(f"{t}:{c2[t]}" for t in c2))
        hit = dict(best[1], params=dict(best[1].get("params", {}), _tuned_on=best[2])) if best else None
    return None if hit is None else dict(DEFAULTS, **hit.get("params", {}))


def _sample(queries, n):
    out = []
    for qt, s in queries:
        k = max(1, min(len(s), int(round(n * len(s) / sum(len(x) for _, x in queries)))))
        idx = np.random.default_rng(12345).choice(len(s), k, replace=False)
        out.append((qt, np.asarray(s)[np.sort(idx)]))
    return out


def _trial(g, sample, spec, p, stream=None) -> float:
    from . import order
    # the workload's vertex order follows the partition size (one tile per partition on grids)
    fg = ForkGraph.from_graph(g, partition_vertices=p["partition_vertices"],
                              vertex_order=order.auto(spec, g, p["partition_vertices"]))
    try:
        n = 0
        for qt, s in sample:
            fg.submit(qt, s, alpha=spec.get("alpha", 0.15), epsilon=spec.get("epsilon", 1e-6),
                      eps_mode=spec.get("eps_mode", 0))
            n += len(s)
        kw = dict(run_kwargs(p), stream=stream)
        fg.run(**kw)
        t0 = time.perf_counter()
        fg.run(**kw)
        return n / (time.perf_counter() - t0)
    finally:
        fg.close()


def candidates(g, queries) -> dict:
    kinds = {qt for qt, _ in queries}
    wmean = float(g.weight.mean()) if g.weight is not None else 1.0
    c = {
        "engine": ["buffered", "grouped"],
        "partition_vertices": [2048, 4096, 8192, 16384, 32768, 65536],
        "items_per_pass": [0, 2048, 16384, 65536],
        "persistent": [0, 1],
        "slice_slots": [0, 1024, 2048, 2560, 4096],
        "mu": [0.0, 1.0, 2.0, 4.0],
        "group_threads": [0, 512, 1024],
    }
    if kinds & {"sssp", "bfs"}:
        w = max(1, int(round(wmean)))
        c["window"] = [0, max(1, w // 8), max(1, w // 2), 2 * w, 8 * w, 32 * w, 128 * w]
        c["delta"] = [0, 4 * w, 16 * w, 64 * w, 256 * w]
    return c


def tune(g, queries, spec, sample=256, rounds=1, budget_s=240.0, log=print, use_cache=True, start=None,
         fixed=()) -> dict:
    """Coordinate descent from `start` (default: the defaults) over every
    knob not named in `fixed`.  A large batch starts from the knobs of a tuned
    subset and fixes the engine, so that no trial runs minutes on a slow
    configuration."""
    key = f"{signature(g, queries, spec)}|{device_name()}"
    cache = _load_cache()
    if use_cache and key in cache:
        return cache[key]["params"]
    smp = _sample(queries, sample)
    best = dict(DEFAULTS, **{k: v for k, v in (start or {}).items() if k in DEFAULTS})
    best_v = _trial(g, smp, spec, best)
    log(f"[tune] start {best} -> {best_v:.1f} q/s")
    trials = [{"params": dict(best), "qps": best_v}]
    t_start = time.time()
    space = candidates(g, queries)
    for _ in range(rounds):
        for name, values in space.items():
            if name in fixed:
                continue
            for v in values:
                if v == best[name] or time.time() - t_start > budget_s:
                    continue
                p = dict(best, **{name: v})
                if not valid(p):
                    continue
                try:
                    q = _trial(g, smp, spec, p)
                except Exception as e:  # noqa: BLE001 - a configuration that fails is just not chosen
                    log(f"[tune] {p} failed: {e}")
                    continue
                trials.append({"params": p, "qps": q})
                log(f"[tune] {name}={v} -> {q:.1f} q/s")
                if q > best_v:
                    best, best_v = p, q
    cache = _load_cache()
    cache[key] = {"params": best, "qps_sample": best_v, "sample_queries": int(sum(len(s) for _, s in smp)),
                  "default_qps_sample": trials[0]["qps"], "trials": trials}
    with open(CACHE, "w") as f:
        json.dump(cache, f, indent=1)
    log(f"[tune] best {best} -> {best_v:.1f} q/s (default {trials[0]['qps']:.1f})")
    return best
