"""Learned partition scheduler: trace collection and GPU training.

The paper schedules partitions with a user priority functor: a partition's
priority is the best priority among its buffered operations (Section 5.2).
The learned scheduler replaces that functor by an MLP (16 -> 64 -> 64 -> 1)
that scores each partition from its buffer statistics.  Training data comes
from the rule-based scheduler itself: a traced run records, for every
partition a pass visited, the 16 features it had when it was selected and the
useful work the visit did (SSSP/BFS: vertex expansions whose distance was
already final; PPR: vertex pushes).  The network learns to predict
log(1 + useful work); at run time the partitions with the highest predicted
useful work are processed first.  Any processing order gives the same exact
SSSP/BFS answers, so the network changes only speed.

    python -m paper_2103_14915_amd.learn --out paper_2103_14915_amd/sched_mlp.npy

Training runs entirely on the GPU through the library's own forward /
backward / Adam kernels (fork_mlp_train).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import MLP_NPARAM, ForkGraph, mlp_train

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "sched_mlp.npy")

# Training graphs: R-MAT scales 20 and 21 with seeds distinct from every
# benchmark and test graph (those use seeds 1..5 and 9..21).
TRAIN_SPECS = [
    dict(scale=20, seed=41, wseed=141, sseed=241),
    dict(scale=21, seed=42, wseed=142, sseed=242),
    dict(scale=20, seed=43, wseed=143, sseed=243),
]


def init_theta(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (same layout as the library)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((64, 16), (64, None), (64, 64), (64, None), (1, 64), (1, None)):
        if fan_in is None:
            parts.append(np.zeros(fan_out))
        else:
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
    th = np.concatenate(parts).astype(np.float32)
    assert th.size == MLP_NPARAM
    return th


LABELS = ("useful", "ratio", "net")


def target_of(records: np.ndarray, label: str = "useful") -> np.ndarray:
    """Regression target of a trace record (column 16 = useful work of the
    partition's visits in the pass, column 17 = all their work):
    useful: log(1 + useful); ratio: useful / work, the share of the visit that
    was not redundant; net: log(1 + useful) - log(1 + redundant)."""
    u, w = records[:, 16].astype(np.float64), records[:, 17].astype(np.float64)
    if label == "ratio":
        t = np.where(w > 0, u / np.maximum(w, 1.0), 0.0)
    elif label == "net":
        t = np.log1p(u) - np.log1p(np.maximum(w - u, 0.0))
    elif label == "useful":
        t = np.log1p(u)
    else:
        raise ValueError(label)
    return t.astype(np.float32)


# run knobs for traces and for learned runs of the SSSP+PPR mix (the autotuned
# setting of the scale-20 mix: 8,192-vertex partitions, SSSP window 16,
# Delta 32768, 64K items per pass, 4,096-slot hashed slices)
PARTITION_VERTICES = 8192
RUN_KW = dict(window=16, delta=32768, items_per_pass=65536, slice_slots=4096)


def collect(spec: dict, n_sssp: int, n_ppr: int, partition_vertices: int = PARTITION_VERTICES, log=print,
            **run_kw) -> np.ndarray:
    import fpp_inputs as fi

    g = fi.rmat(spec["scale"], seed=spec["seed"], weights=(1, 255), weight_seed=spec["wseed"])
    fg = ForkGraph.from_graph(g, partition_vertices=partition_vertices)
    if n_sssp:
        fg.submit("sssp", fi.sources_mixed(g, n_sssp, spec["sseed"]))
    if n_ppr:
        fg.submit("ppr", fi.sources_mixed(g, n_ppr, spec["sseed"] + 1), alpha=0.15, epsilon=1e-6, eps_mode=1)
    t0 = time.time()
    fg.run(scheduler="priority", trace=1, **(run_kw or RUN_KW))
    rec = fg.trace()
    fg.close()
    log(f"[learn] traced rmat{spec['scale']} seed {spec['seed']}: {rec.shape[0]} visits in {time.time() - t0:.1f}s")
    return rec


# Grid family (the road-network stand-in): grids whose weight and source
# seeds differ from every test and benchmark grid, traced with the knobs tuned
# for the 2048 x 2048 workload in its tile order.
GRID_SPECS = [
    dict(rows=1024, cols=1024, wseed=161, sseed=261),
    dict(rows=1536, cols=1536, wseed=162, sseed=262),
    dict(rows=1024, cols=2048, wseed=163, sseed=263),
]
GRID_PARTITION_VERTICES = 8192
GRID_RUN_KW = dict(window=0, delta=128256, items_per_pass=65536, slice_slots=0)


def collect_grid(spec: dict, n_sssp: int, n_bfs: int, log=print) -> np.ndarray:
    import fpp_inputs as fi
    from . import order

    g = fi.grid(spec["rows"], spec["cols"], weights=(1, 1000), weight_seed=spec["wseed"])
    pos = order.grid_tiles(spec["rows"], spec["cols"], *order.tile_shape(GRID_PARTITION_VERTICES))
    fg = ForkGraph.from_graph(g, partition_vertices=GRID_PARTITION_VERTICES, vertex_order=pos)
    if n_sssp:
        fg.submit("sssp", fi.sources_uniform(g, n_sssp, spec["sseed"]))
    if n_bfs:
        fg.submit("bfs", fi.sources_uniform(g, n_bfs, spec["sseed"] + 1))
    t0 = time.time()
    fg.run(scheduler="priority", trace=1, **GRID_RUN_KW)
    rec = fg.trace()
    fg.close()
    log(f"[learn] traced grid {spec['rows']}x{spec['cols']}: {rec.shape[0]} visits in {time.time() - t0:.1f}s")
    return rec


def train(records: np.ndarray, steps: int = 3000, batch: int = 256, lr: float = 1e-3, seed: int = 7,
          label: str = "useful"):
    x = records[:, :16]
    t = target_of(records, label)
    theta = init_theta(seed)
    theta, losses = mlp_train(theta, x, t, steps=steps, batch=batch, lr=lr, seed=seed)
    return theta, losses


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--family", default="rmat", choices=["rmat", "grid"],
                    help="training graphs: R-MAT SSSP+PPR mixes, or grids with SSSP+BFS")
    ap.add_argument("--sssp", type=int, default=512)
    ap.add_argument("--ppr", type=int, default=512)
    ap.add_argument("--bfs", type=int, default=256, help="BFS queries per grid (grid family)")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--specs", type=int, default=0, help="training graphs to use (0 = all of the family)")
    ap.add_argument("--label", default="useful", choices=LABELS)
    ap.add_argument("--save-trace", default="", help="also save the trace records (.npy)")
    ap.add_argument("--load-trace", default="", help="train on saved trace records instead of tracing")
    args = ap.parse_args(argv)
    specs = (GRID_SPECS if args.family == "grid" else TRAIN_SPECS)
    specs = specs[:args.specs] if args.specs else specs
    if args.load_trace:
        records = np.load(args.load_trace)
    elif args.family == "grid":
        records = np.concatenate([collect_grid(s, args.sssp, args.bfs) for s in specs])
    else:
        records = np.concatenate([collect(s, args.sssp, args.ppr) for s in specs])
    if args.save_trace:
        np.save(args.save_trace, records)
    t0 = time.time()
    theta, losses = train(records, steps=args.steps, label=args.label)
    print(f"[learn] trained on {records.shape[0]} visits, {args.steps} steps in {time.time() - t0:.1f}s: "
          f"loss {losses[:50].mean():.4f} -> {losses[-50:].mean():.4f}", flush=True)
    np.save(args.out, theta)
    grid = args.family == "grid"
    meta = {"records": int(records.shape[0]), "steps": args.steps, "loss_first": float(losses[:50].mean()),
            "loss_last": float(losses[-50:].mean()), "family": args.family, "specs": specs, "label": args.label,
            "run_knobs": dict(GRID_RUN_KW, partition_vertices=GRID_PARTITION_VERTICES) if grid
            else dict(RUN_KW, partition_vertices=PARTITION_VERTICES),
            "queries": {"sssp": args.sssp, "bfs": args.bfs} if grid else {"sssp": args.sssp, "ppr": args.ppr}}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
