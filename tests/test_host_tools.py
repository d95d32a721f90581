"""Host-side logic that needs no GPU: the autotuner's search and cache, the
rocprofv3 summariser, bench.py's one-GPU guard and traffic lookup."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import fpp_inputs as fi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def autotune(tmp_path, monkeypatch):
    from paper_2103_14915_amd import autotune as at
    monkeypatch.setattr(at, "CACHE", str(tmp_path / "cache.json"))
    monkeypatch.setattr(at, "device_name", lambda: "test-device")
    return at


def test_autotune_coordinate_descent_and_cache(autotune, monkeypatch):
    """With a synthetic cost model the search finds the best value of every
    knob, caches it under (graph, mix, device), and later calls reuse it."""
    g = fi.rmat(10, seed=1, weights=(1, 9), weight_seed=2)
    queries = [("sssp", fi.sources_uniform(g, 40, 3)), ("ppr", fi.sources_uniform(g, 20, 4))]
    best = {"partition_vertices": 32768, "items_per_pass": 16384, "persistent": 1, "slice_slots": 2048,
            "window": 4, "delta": 80}
    calls = []

    def trial(g_, sample, spec, p, stream=None):
        calls.append(dict(p))
        assert sum(len(s) for _, s in sample) <= 24  # the sample, not the whole batch
        return 100.0 + 10.0 * sum(k in best and p[k] == best[k] for k in p)  # more matches, more q/s

    monkeypatch.setattr(autotune, "_trial", trial)
    cand = autotune.candidates(g, queries)
    w = max(1, int(round(float(g.weight.mean()))))
    best["window"], best["delta"] = cand["window"][2], cand["delta"][1]
    p = autotune.tune(g, queries, {}, sample=24, log=lambda *a: None)
    for k, v in best.items():
        assert p[k] == v, (k, p[k], v)
    assert autotune.cached(g, queries) == p
    n = len(calls)
    assert autotune.tune(g, queries, {}, sample=24, log=lambda *a: None) == p
    assert len(calls) == n  # served from the cache
    cache = json.load(open(autotune.CACHE))
    (key,) = cache
    assert key.endswith("|test-device") and cache[key]["trials"][0]["params"] == autotune.DEFAULTS
    assert w >= 1


def test_autotune_cache_falls_back_to_other_device(autotune):
    g = fi.rmat(9, seed=5)
    queries = [("ppr", fi.sources_uniform(g, 8, 6))]
    sig = autotune.signature(g, queries)
    json.dump({f"{sig}|another-gpu": {"params": {"partition_vertices": 8192}}}, open(autotune.CACHE, "w"))
    got = autotune.cached(g, queries)
    assert got["partition_vertices"] == 8192 and got["slice_slots"] == autotune.DEFAULTS["slice_slots"]
    other = [("sssp", fi.sources_uniform(g, 8, 6))]
    assert autotune.cached(g, other) is None  # a different query mix is a different key
    # a batch of 9 takes the entry tuned on its subset of 8
    assert autotune.cached(g, [("ppr", fi.sources_uniform(g, 9, 6))])["partition_vertices"] == 8192


def test_autotune_cache_takes_a_subset_entry_for_a_larger_batch(autotune):
    """A batch too large to tune in full takes the knobs tuned on the largest
    seeded subset of the same graph with the same query types."""
    g = fi.rmat(9, seed=5)
    small = [("sssp", np.arange(8)), ("ppr", np.arange(8))]
    mid = [("sssp", np.arange(16)), ("ppr", np.arange(16))]
    full = [("sssp", np.arange(64)), ("ppr", np.arange(64))]
    cache = {f"{autotune.signature(g, small)}|d": {"params": {"partition_vertices": 1024}},
             f"{autotune.signature(g, mid)}|d": {"params": {"partition_vertices": 2048}}}
    json.dump(cache, open(autotune.CACHE, "w"))
    assert autotune.cached(g, full)["partition_vertices"] == 2048      # the largest subset
    assert autotune.cached(g, [("sssp", np.arange(12)), ("ppr", np.arange(12))])["partition_vertices"] == 1024
    assert autotune.cached(g, [("sssp", np.arange(64))]) is None       # other query types
    assert autotune.cached(g, [("sssp", np.arange(4)), ("ppr", np.arange(4))]) is None  # no smaller subset
    assert autotune.cached(fi.rmat(9, seed=6), full) is None           # another graph


def test_autotune_keys_absolute_ppr_apart(autotune):
    """PPR with the absolute threshold tunes apart from the degree-scaled one
    on the same graph and sources."""
    g = fi.rmat(9, seed=5)
    q = [("ppr", np.arange(16))]
    deg, ab = autotune.signature(g, q, {"eps_mode": 1}), autotune.signature(g, q, {"eps_mode": 0})
    assert deg == autotune.signature(g, q) and ab != deg and "ppr@abs:16" in ab
    json.dump({f"{deg}|d": {"params": {"partition_vertices": 4096}}}, open(autotune.CACHE, "w"))
    assert autotune.cached(g, q, {"eps_mode": 1})["partition_vertices"] == 4096
    assert autotune.cached(g, q, {"eps_mode": 0}) is None
    assert autotune.signature(g, [("sssp", np.arange(16))], {"eps_mode": 0}) == \
        autotune.signature(g, [("sssp", np.arange(16))])


def test_autotune_sample_keeps_the_mix(autotune):
    g = fi.rmat(9, seed=7)
    q = [("sssp", np.arange(300)), ("bfs", np.arange(100)), ("ppr", np.arange(100))]
    s = autotune._sample(q, 100)
    assert [qt for qt, _ in s] == ["sssp", "bfs", "ppr"]
    assert [len(x) for _, x in s] == [60, 20, 20]
    assert all(np.all(np.diff(x) > 0) for _, x in s)  # subsets in submit order, no repeats


def _write_csv(path, header, rows):
    with open(path, "w") as f:
        f.write(",".join(header) + "\n")
        for r in rows:
            f.write(",".join(str(x) for x in r) + "\n")


def test_profile_summary_scales_counters_by_copy_calibration(tmp_path):
    from paper_2103_14915_amd import profile_summary as ps
    stats = tmp_path / "stats.csv"
    _write_csv(stats, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
               [["void fk::k_process<0>(x)", 4, 8e6, 2e6, 90.0], ["fk::k_select(x)", 4, 1e5, 2.5e4, 1.0]])
    pmc_hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_csv(fetch, pmc_hdr, [["fk::k_process<0>(x)", "FETCH_SIZE", 1000.0]] * 4)
    _write_csv(write, pmc_hdr, [["fk::k_process<0>(x)", "WRITE_SIZE", 500.0]] * 4)
    cf, cw = tmp_path / "cf.csv", tmp_path / "cw.csv"
    copy_bytes = 1 << 20  # the copy moved 1 MiB; its counters read half (fetch) and all (write) of it
    _write_csv(cf, pmc_hdr, [["__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0]] * 2)
    _write_csv(cw, pmc_hdr, [["__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0]] * 2)
    tcc, sq, clog = tmp_path / "tcc.csv", tmp_path / "sq.csv", tmp_path / "copy.log"
    _write_csv(tcc, pmc_hdr, [["fk::k_process<0>(x)", "TCC_HIT_sum", 300.0], ["fk::k_process<0>(x)", "TCC_MISS_sum", 100.0],
                              ["fk::k_select(x)", "TCC_HIT_sum", 1.0], ["fk::k_select(x)", "TCC_MISS_sum", 99.0]] * 2)
    _write_csv(sq, pmc_hdr, [["fk::k_process<0>(x)", "SQ_WAIT_ANY", 60.0], ["fk::k_process<0>(x)", "SQ_WAVE_CYCLES", 80.0]])
    clog.write_text("noise\n" + json.dumps({"copy_calibration_bytes": 1, "copy_gbs": 4321.0}) + "\n")
    # the counter runs' bench lines: their steps' algorithmic bytes
    flog, wlog = tmp_path / "f.out", tmp_path / "w.out"
    flog.write_text(json.dumps({"roofline": {"algorithmic_bytes_per_step": 4 * 1000.0 * 1024 * 2.0}}) + "\n")
    wlog.write_text("x\n" + json.dumps({"roofline": {"algorithmic_bytes_per_step": 8 * 500.0 * 1024}}) + "\n")
    out = tmp_path / "k.md"
    ps.main(["--stats", str(stats), "--fetch", str(fetch), "--write", str(write), "--copy-fetch", str(cf),
             "--copy-write", str(cw), "--copy-bytes", str(copy_bytes), "--kernel", "k_process",
             "--tcc", str(tcc), "--sq", str(sq), "--copy-log", str(clog), "--fetch-log", str(flog),
             "--write-log", str(wlog), "--command", "cmd", "--out", str(out)])
    blob = json.loads(out.read_text().split("```json", 1)[1].split("```", 1)[0])
    # 4 launches of 2 MiB fetched against 8 MiB algorithmic; 4 x 0.5 MiB written against 4 MiB
    assert blob["fetch_over_algorithmic"] == pytest.approx(1.0) and blob["write_over_algorithmic"] == pytest.approx(0.5)
    assert blob["traffic_over_algorithmic"] == pytest.approx(1.5) and blob["kernel_ms_total"] == pytest.approx(8.0)
    assert blob["l2_hit_rate"] == pytest.approx(0.75)  # the kernel's own counters, not k_select's
    assert blob["wave_wait_share"] == pytest.approx(0.75) and blob["copy_gbs"] == 4321.0
    assert blob["fetch_scale"] == pytest.approx(2.0) and blob["write_scale"] == pytest.approx(1.0)
    assert blob["fetch_bytes_per_launch"] == pytest.approx(1000.0 * 1024 * 2.0)
    assert blob["write_bytes_per_launch"] == pytest.approx(500.0 * 1024)
    assert blob["avg_launch_ms"] == pytest.approx(2.0) and blob["calls"] == 4
    assert blob["source_hash"] == ps.kernel_source_hash()


def test_bench_traffic_lookup_requires_matching_source(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    from paper_2103_14915_amd import profile_summary as ps
    prof = tmp_path / "profiles"
    prof.mkdir()
    blob = {"kernel": "k_process", "source_hash": ps.kernel_source_hash(), "traffic_bytes_per_launch": 123.0}
    (prof / "k_process_w.md").write_text("x\n```json\n" + json.dumps(blob) + "\n```\n")
    assert bench.measured_traffic("w", "k_process", str(tmp_path))["traffic_bytes_per_launch"] == 123.0
    # the grouped engine's kernel has its own summary and source hash
    assert bench.measured_traffic("w", "k_gprocess", str(tmp_path)) is None
    gblob = dict(blob, kernel="k_gprocess", source_hash=ps.kernel_source_hash("k_gprocess"))
    (prof / "k_gprocess_w.md").write_text("x\n```json\n" + json.dumps(gblob) + "\n```\n")
    assert bench.measured_traffic("w", "k_gprocess", str(tmp_path))["traffic_bytes_per_launch"] == 123.0
    assert ps.kernel_source_hash("k_gprocess") != ps.kernel_source_hash("k_process")
    blob["source_hash"] = "0" * 16
    (prof / "k_process_w.md").write_text("x\n```json\n" + json.dumps(blob) + "\n```\n")
    assert bench.measured_traffic("w", "k_process", str(tmp_path)) is None  # profile of another kernel version
    assert bench.measured_traffic("missing", "k_process", str(tmp_path)) is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_ablation_configs_cover_the_study():
    """The study's tables: four schedules; heuristic 1 at 0.25-4 mu with
    heuristic 2 off; heuristic 2 at 0.25-4 Delta with heuristic 1 off; a run
    without yielding; the cumulative ladder.  The priority run comes first."""
    from paper_2103_14915_amd import ablation as ab
    c = ab.configs({"sssp", "bfs"}, 1000)
    assert c[0] == ("A", "Shortest (priority functor)", {"scheduler": "priority"})
    assert [o["scheduler"] for g, _, o in c if g == "A"] == ["priority", "fifo", "random", "maxops"]
    b = [o for g, _, o in c if g == "B"]
    assert [o["edge_budget_mu"] for o in b] == [0.25, 0.5, 1.0, 2.0, 4.0, 0.0]
    assert all(o["window_mode"] == 1 and o["delta"] >= 2 ** 30 for o in b)  # heuristic 2 off
    cc = [o for g, _, o in c if g == "C"]
    assert [o["delta"] for o in cc[:5]] == [250, 500, 1000, 2000, 4000]
    assert "edge_budget_mu" not in cc[0] and cc[5] == b[5]  # heuristic 1 off; the same no-yield run
    acc = [o for g, _, o in c if g == "acc"]
    assert acc[0]["scheduler"] == "fifo" and acc[1]["scheduler"] == "priority" and acc[0]["edge_budget_mu"] == 0
    assert acc[2] == {"scheduler": "priority"}
    p = ab.configs({"ppr"}, 1)
    assert not [1 for g, _, _ in p if g == "C"]
    assert [o.get("edge_budget_mu") for g, _, o in p if g == "acc"] == [0.0, 0.0, 2.0]


def test_ablation_markdown_marks_differences():
    from paper_2103_14915_amd import ablation as ab
    rows = [{"group": "A", "config": "x", "queries_per_s": 10.0, "ms_per_run": 1.0, "passes": 3, "edges": 5,
             "sssp_bfs_identical": True, "ppr_mean_residual": None},
            {"group": "B", "config": "y", "queries_per_s": 5.0, "ms_per_run": 2.0, "passes": 4, "edges": 6,
             "sssp_bfs_identical": False, "ppr_mean_residual": 0.25}]
    md = ab.markdown(rows).splitlines()
    assert "| 1.00× |" in md[2] and "identical" in md[2]
    assert "0.50×" in md[3] and "DIFFERENT" in md[3] and "0.25" in md[3]
