"""The scheduling/yielding study on a small grid: every schedule, yield
setting and ladder step returns SSSP/BFS results identical to the priority
run's (the paper's exactness under any processing order)."""
import sys

import numpy as np
import pytest

import fpp_inputs as fi
import oracle

pytestmark = pytest.mark.gpu


def test_ablation_study_is_exact_under_every_schedule():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_14915_amd import ablation as ab
    g = fi.grid(96, 96, weights=(1, 1000), weight_seed=5)
    s_sp = fi.sources_uniform(g, 12, 6)
    s_bf = fi.sources_uniform(g, 12, 7)
    base = {"partition_vertices": 1024, "items_per_pass": 0, "window": 0, "delta": 0, "slice_slots": 0}
    lines = []
    rows = ab.study(g, [("sssp", s_sp), ("bfs", s_bf)], {}, base, steps=1, warmup=0,
                    log=lambda *a: (lines.append(" ".join(map(str, a))), print(*a, flush=True)))
    assert [r["group"] for r in rows].count("A") == 4 and len(rows) == len(ab.configs({"sssp"}, 1))
    assert all(r["sssp_bfs_identical"] for r in rows)
    # the reference itself is exact
    from paper_2103_14915_amd import ForkGraph
    fg = ForkGraph.from_graph(g, partition_vertices=1024)
    fg.submit("sssp", s_sp)
    fg.run()
    d = np.stack([fg.fetch(i) for i in range(len(s_sp))])
    fg.close()
    np.testing.assert_array_equal(d, oracle.sssp(g, s_sp))
    sys.stdout.flush()
