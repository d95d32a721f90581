"""ctypes harness for the CPU build of the library (tests/simt/libfork_simt.so).

It drives the same C ABI as the GPU binding, reusing its structure layouts,
and reads the pool ownership checker's results.  Test infrastructure only.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import build as simt_build  # noqa: E402

import paper_2103_14915_amd as fork  # noqa: E402  (structure layouts and constants only)

_libs = {}


def load(asan: bool = False):
    if asan not in _libs:
        path = simt_build.build(asan=asan)
        lib = ctypes.CDLL(path)
        P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        lib.fork_graph_load.argtypes = [ctypes.POINTER(ctypes.c_void_p), U32, U64, P, P, P,
                                        ctypes.POINTER(fork.fork_config)]
        lib.fork_submit.argtypes = [P, I, P, U32, P, ctypes.POINTER(U32)]
        lib.fork_run.argtypes = [P, ctypes.POINTER(fork.fork_run_opts)]
        lib.fork_fetch.argtypes = [P, U32, I, P, U64, I]
        lib.fork_stats.argtypes = [P, P, U64]
        lib.fork_destroy.argtypes = [P]
        lib.fork_destroy.restype = None
        lib.fork_last_error.restype = ctypes.c_char_p
        lib.simt_check_message.restype = ctypes.c_char_p
        lib.simt_check_count.restype = U64
        lib.simt_check_failures.restype = U64
        for n in ("fork_graph_load", "fork_submit", "fork_run", "fork_fetch", "fork_stats"):
            getattr(lib, n).restype = I
        _libs[asan] = lib
    return _libs[asan]


class SimtGraph:
    """One context of the CPU build: load, submit, run, fetch."""

    def __init__(self, lib, g, partition_vertices=0, pool_bytes=0, max_queries=0):
        self.lib = lib
        self.g = g
        rp = np.ascontiguousarray(g.row_ptr, np.uint64)
        col = np.ascontiguousarray(g.col, np.uint32)
        w = None if g.weight is None else np.ascontiguousarray(g.weight, np.uint32)
        cfg = fork.fork_config(partition_vertices=partition_vertices, pool_bytes=pool_bytes, max_queries=max_queries)
        self.ctx = ctypes.c_void_p()
        self._check(lib.fork_graph_load(ctypes.byref(self.ctx), g.num_vertices, int(col.size), rp.ctypes.data,
                                        col.ctypes.data, None if w is None else w.ctypes.data, ctypes.byref(cfg)))

    def _check(self, rc):
        if rc != 0:
            raise fork.ForkError(rc, self.lib.fork_last_error().decode())

    def submit(self, qtype, sources, alpha=0.15, epsilon=1e-6, eps_mode=0, l1_target=0.0):
        s = np.ascontiguousarray(sources, np.uint32)
        prm = None
        if qtype == "ppr":
            prm = fork.fork_ppr_params(alpha=alpha, epsilon=epsilon, eps_mode=eps_mode, l1_target=l1_target)
        first = ctypes.c_uint32()
        self._check(self.lib.fork_submit(self.ctx, fork.QTYPES[qtype], s.ctypes.data, s.size,
                                         None if prm is None else ctypes.byref(prm), ctypes.byref(first)))
        return first.value

    def run(self, **kw):
        o = fork.fork_run_opts(scheduler=fork.SCHEDS[kw.pop("scheduler", "priority")])
        if isinstance(kw.get("engine"), str):
            kw["engine"] = fork.ENGINES[kw["engine"]]
        for k, v in kw.items():
            setattr(o, k, v)
        self._check(self.lib.fork_run(self.ctx, ctypes.byref(o)))

    def fetch(self, qid, field=fork.FIELD_VALUE):
        n = self.g.num_vertices
        out = np.empty(n, np.int32 if field == fork.FIELD_VALUE else np.float32)
        self._check(self.lib.fork_fetch(self.ctx, qid, field, out.ctypes.data, out.nbytes, 0))
        return out

    def digest(self, qid):
        d = fork.fork_digest()
        self._check(self.lib.fork_fetch(self.ctx, qid, fork.FIELD_DIGEST, ctypes.byref(d), ctypes.sizeof(d), 0))
        return {n: getattr(d, n) for n, _ in d._fields_}

    def stats(self):
        st = fork.fork_stats_t()
        self._check(self.lib.fork_stats(self.ctx, ctypes.byref(st), ctypes.sizeof(st)))
        return st.as_dict()

    def close(self):
        if self.ctx:
            self.lib.fork_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()


def checker(lib):
    return {"checks": int(lib.simt_check_count()), "failures": int(lib.simt_check_failures()),
            "message": lib.simt_check_message().decode()}


def reset_checker(lib):
    lib.simt_check_reset()


def run_case(name: str) -> dict:
    """Small fixed runs used by the tests (also from a subprocess, for the
    planted-mistake cases, which leave the pool damaged)."""
    import fpp_inputs as fi
    lib = load()
    reset_checker(lib)
    out = {"case": name}
    if name == "sssp_small_pool":
        g = fi.rmat(10, seed=21, weights=(1, 255), weight_seed=22)
        srcs = fi.sources_uniform(g, 8, 1)
        fg = SimtGraph(lib, g, partition_vertices=128, pool_bytes=2 << 20)
        fg.submit("sssp", srcs)
        try:
            fg.run(max_passes=100000)
            out["error"] = ""
        except fork.ForkError as e:  # a damaged pool may also trip the kernels' own checks
            out["error"] = str(e)
        fg.close()
    out["check"] = checker(lib)
    return out


if __name__ == "__main__":
    import json
    r = run_case(sys.argv[1])
    print(json.dumps({"case": r["case"], "check": r["check"], "error": r.get("error", "")}), flush=True)
