"""Python binding of the MI355X fork-processing library (``libfork.so``).

Thin ctypes marshalling over the C ABI declared in ``include/fork.h``: every
step of the fork-processing pass runs in the library's HIP kernels.  Inputs
may be numpy arrays (host) or torch tensors (host or device); results come
back as numpy arrays or are written into caller-provided torch tensors.

The library must have been built (``python -m paper_2103_14915_amd.build``);
importing this package without it raises ImportError, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfork.so")

FORK_OK, FORK_E_INVALID, FORK_E_NOMEM, FORK_E_DEVICE, FORK_E_STATE, FORK_E_CAPACITY, FORK_E_NOT_CONVERGED = (
    0, -1, -2, -3, -4, -5, -6)
SSSP, BFS, PPR = 1, 2, 3
SCHED_FIFO, SCHED_PRIORITY, SCHED_LEARNED, SCHED_RANDOM, SCHED_MAXOPS = 0, 1, 2, 3, 4
FIELD_VALUE, FIELD_P, FIELD_R, FIELD_DIGEST = 0, 1, 2, 3
QTYPES = {"sssp": SSSP, "bfs": BFS, "ppr": PPR}
SCHEDS = {"fifo": SCHED_FIFO, "priority": SCHED_PRIORITY, "learned": SCHED_LEARNED, "random": SCHED_RANDOM,
          "maxops": SCHED_MAXOPS}
ENGINE_BUFFERED, ENGINE_GROUPED = 0, 1
ENGINES = {"buffered": ENGINE_BUFFERED, "grouped": ENGINE_GROUPED}
MLP_NPARAM = 5313
INF = 0x7FFFFFFF


class ForkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fork error {code}: {msg}")
        self.code = code


class fork_config(ctypes.Structure):
    _fields_ = [("partition_vertices", ctypes.c_uint32), ("partition_edges", ctypes.c_uint32),
                ("max_queries", ctypes.c_uint32), ("pool_bytes", ctypes.c_uint64),
                ("inputs_on_device", ctypes.c_int), ("device", ctypes.c_int),
                ("vertex_order", ctypes.c_void_p)]


class fork_ppr_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("epsilon", ctypes.c_float), ("eps_mode", ctypes.c_int),
                ("l1_target", ctypes.c_float)]


class fork_run_opts(ctypes.Structure):
    _fields_ = [("scheduler", ctypes.c_int), ("parts_per_pass", ctypes.c_uint32), ("delta", ctypes.c_uint32),
                ("edge_budget_mu", ctypes.c_float), ("max_passes", ctypes.c_uint64),
                ("stream", ctypes.c_void_p), ("mlp_weights", ctypes.c_void_p), ("persistent", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("profile", ctypes.c_int), ("items_per_pass", ctypes.c_uint32),
                ("trace", ctypes.c_int), ("window_mode", ctypes.c_int), ("window", ctypes.c_uint32),
                ("slice_slots", ctypes.c_uint32), ("engine", ctypes.c_int), ("group_threads", ctypes.c_uint32)]


class fork_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("passes", "work_items", "edges", "improved", "ops_emitted",
                                                "ops_consumed", "vertex_pushes", "yields", "chunks", "waves")] + \
               [("init_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("digest_ms", ctypes.c_double),
                ("process_ms", ctypes.c_double), ("process_launches", ctypes.c_uint64),
                ("intra_edges", ctypes.c_uint64), ("pruned", ctypes.c_uint64), ("num_partitions", ctypes.c_uint32),
                ("weight_bytes", ctypes.c_uint32), ("refine_rounds", ctypes.c_uint64),
                ("selected_edges", ctypes.c_uint64), ("ppr_edges", ctypes.c_uint64),
                ("ppr_vertex_pushes", ctypes.c_uint64), ("spilled", ctypes.c_uint64),
                ("activations", ctypes.c_uint64), ("expansions", ctypes.c_uint64), ("spill_max", ctypes.c_uint64),
                ("rounds", ctypes.c_uint64), ("edge_tasks", ctypes.c_uint64), ("visit_ns", ctypes.c_uint64 * 5),
                ("wall_ms", ctypes.c_double), ("setup_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: (list(getattr(self, n)) if isinstance(getattr(self, n), ctypes.Array) else getattr(self, n))
                for n, _ in self._fields_}


class fork_sweep_t(ctypes.Structure):
    _fields_ = [("support", ctypes.c_uint32), ("swept", ctypes.c_uint32), ("best_size", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("best_conductance", ctypes.c_double), ("best_cut", ctypes.c_uint64),
                ("best_volume", ctypes.c_uint64), ("size_min", ctypes.c_double * 11)]


class fork_digest(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("sum", ctypes.c_uint64), ("hash", ctypes.c_uint64),
                ("fsum", ctypes.c_double), ("fres", ctypes.c_double), ("fmax", ctypes.c_double)]


EXPORTS = ["fork_graph_load", "fork_submit", "fork_run", "fork_prepare", "fork_fetch", "fork_stats", "fork_partitions",
           "fork_trace", "fork_destroy", "fork_last_error", "fork_mlp_forward", "fork_mlp_grad", "fork_mlp_train",
           "fork_sweep", "fork_bc", "fork_mlp_train_noalloc"]
SWEEP_MAX, SWEEP_BUCKETS = 1024, 11
TRACE_WIDTH = 20


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2103_14915_amd.build`")
    # torch (device memory and streams for callers) ships its own HIP runtime;
    # load it first so that the library binds to the same runtime and both
    # share one device context and stream namespace.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.fork_graph_load.argtypes = [ctypes.POINTER(ctypes.c_void_p), U32, U64, P, P, P,
                                    ctypes.POINTER(fork_config)]
    lib.fork_submit.argtypes = [P, I, P, U32, P, ctypes.POINTER(U32)]
    lib.fork_run.argtypes = [P, ctypes.POINTER(fork_run_opts)]
    lib.fork_prepare.argtypes = [P, ctypes.POINTER(fork_run_opts)]
    lib.fork_fetch.argtypes = [P, U32, I, P, U64, I]
    lib.fork_stats.argtypes = [P, P, U64]
    lib.fork_partitions.argtypes = [P, P, U32, ctypes.POINTER(U32)]
    lib.fork_trace.argtypes = [P, P, U64, ctypes.POINTER(U64)]
    lib.fork_mlp_forward.argtypes = [P, P, U64, P]
    lib.fork_mlp_grad.argtypes = [P, P, P, U64, P, P]
    lib.fork_mlp_train.argtypes = [P, P, P, U64, U32, U32, ctypes.c_float, U64, P]
    lib.fork_mlp_train_noalloc.argtypes = [P, P, P, U64, U32, U32, ctypes.c_float, U64, P, P]
    lib.fork_sweep.argtypes = [P, U32, U32, U32, P]
    lib.fork_bc.argtypes = [P, U32, U32, P]
    lib.fork_destroy.argtypes = [P]
    lib.fork_destroy.restype = None
    lib.fork_last_error.restype = ctypes.c_char_p
    for n in ("fork_graph_load", "fork_submit", "fork_run", "fork_prepare", "fork_fetch", "fork_stats", "fork_partitions",
              "fork_trace", "fork_mlp_forward", "fork_mlp_grad", "fork_mlp_train", "fork_sweep", "fork_bc",
              "fork_mlp_train_noalloc"):
        getattr(lib, n).restype = I
    return lib


lib = _load()


def _check(rc):
    if rc != FORK_OK:
        raise ForkError(rc, lib.fork_last_error().decode())


def _ptr(x):
    """(pointer, on_device, keepalive) for a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None, False, None
    if isinstance(x, np.ndarray):
        x = np.ascontiguousarray(x)
        return ctypes.c_void_p(x.ctypes.data), False, x
    # torch tensor
    if not x.is_contiguous():
        x = x.contiguous()
    return ctypes.c_void_p(x.data_ptr()), x.is_cuda, x


class ForkGraph:
    """A graph loaded on the GPU plus the queries submitted against it."""

    def __init__(self, num_vertices, row_ptr, col, weight=None, partition_vertices=0, partition_edges=0,
                 max_queries=0, pool_bytes=0, device=0, vertex_order=None):
        """vertex_order: None, or each vertex's position in the library's internal
        numbering (a permutation; see ``paper_2103_14915_amd.order``).  Sources,
        results and digests stay in the caller's ids."""
        rp, dev_rp, k1 = _ptr(row_ptr if not isinstance(row_ptr, np.ndarray) else row_ptr.astype(np.uint64))
        cp, dev_c, k2 = _ptr(col if not isinstance(col, np.ndarray) else col.astype(np.uint32))
        wp, dev_w, k3 = _ptr(weight if (weight is None or not isinstance(weight, np.ndarray))
                             else weight.astype(np.uint32))
        on_dev = dev_rp or dev_c or dev_w
        if on_dev and not (dev_rp and dev_c and (weight is None or dev_w)):
            raise ValueError("row_ptr, col and weight must all be on the host or all on the device")
        if vertex_order is not None and not hasattr(vertex_order, "data_ptr"):
            vertex_order = np.ascontiguousarray(vertex_order, np.uint32)
        op, dev_o, k4 = _ptr(vertex_order)
        if vertex_order is not None and bool(dev_o) != bool(on_dev):
            raise ValueError("vertex_order must be where row_ptr and col are (host or device)")
        cfg = fork_config(partition_vertices, partition_edges, max_queries, pool_bytes, int(on_dev), device, op)
        ne = int(k2.shape[0]) if k2 is not None else 0
        self._ctx = ctypes.c_void_p()
        self.num_vertices = int(num_vertices)
        self.num_edges = ne
        _check(lib.fork_graph_load(ctypes.byref(self._ctx), self.num_vertices, ne, rp, cp, wp, ctypes.byref(cfg)))
        self.types = []

    @classmethod
    def from_graph(cls, g, **kw):
        return cls(g.num_vertices, g.row_ptr, g.col, g.weight, **kw)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib.fork_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def partitions(self) -> np.ndarray:
        n = ctypes.c_uint32()
        _check(lib.fork_partitions(self._ctx, None, 0, ctypes.byref(n)))
        out = np.empty(n.value + 1, np.uint32)
        _check(lib.fork_partitions(self._ctx, ctypes.c_void_p(out.ctypes.data), n.value, ctypes.byref(n)))
        return out

    def submit(self, qtype, sources, alpha=0.15, epsilon=1e-6, eps_mode=0, l1_target=0.0) -> int:
        t = QTYPES[qtype] if isinstance(qtype, str) else int(qtype)
        src = np.ascontiguousarray(np.asarray(sources), np.uint32)
        params = None
        if t == PPR:
            params = ctypes.byref(fork_ppr_params(alpha, epsilon, eps_mode, l1_target))
        first = ctypes.c_uint32()
        _check(lib.fork_submit(self._ctx, t, ctypes.c_void_p(src.ctypes.data), src.size, params,
                               ctypes.byref(first)))
        if self.types and first.value == 0:
            self.types = []
        self.types.extend([t] * src.size)
        return first.value

    def run(self, scheduler="priority", parts_per_pass=0, delta=0, edge_budget_mu=0.0, max_passes=0,
            stream=None, mlp_weights=None, persistent=0, seed=0, profile=0, items_per_pass=0, trace=0,
            window_mode=0, window=0, slice_slots=0, engine="buffered", group_threads=0, prepare_only=False):
        """fork_run; with prepare_only, fork_prepare (allocate the run's device buffers, run nothing)."""
        s = SCHEDS[scheduler] if isinstance(scheduler, str) else int(scheduler)
        eng = ENGINES[engine] if isinstance(engine, str) else int(engine)
        w = None
        if mlp_weights is not None:
            w = np.ascontiguousarray(np.asarray(mlp_weights, np.float32))
            if w.size != MLP_NPARAM:
                raise ValueError(f"mlp_weights must have {MLP_NPARAM} values")
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        o = fork_run_opts(s, parts_per_pass, delta, edge_budget_mu, max_passes, sp,
                          None if w is None else w.ctypes.data, persistent, seed, profile, items_per_pass, trace,
                          window_mode, window, slice_slots, eng, group_threads)
        _check((lib.fork_prepare if prepare_only else lib.fork_run)(self._ctx, ctypes.byref(o)))

    def prepare(self, **kw):
        """fork_prepare with fork_run's keyword arguments."""
        self.run(prepare_only=True, **kw)

    def fetch(self, qid, field=None, out=None):
        """Result vector of query qid (numpy), or written into a device tensor `out`."""
        t = self.types[qid] if 0 <= qid < len(self.types) else SSSP  # out of range: the C ABI rejects it
        if field is None:
            field = FIELD_VALUE if t != PPR else FIELD_P
        dtype = np.int32 if field == FIELD_VALUE else np.float32
        if out is not None:
            p, on_dev, keep = _ptr(out)
            _check(lib.fork_fetch(self._ctx, qid, field, p, out.numel() * out.element_size(), int(on_dev)))
            return out
        arr = np.empty(self.num_vertices, dtype)
        _check(lib.fork_fetch(self._ctx, qid, field, ctypes.c_void_p(arr.ctypes.data), arr.nbytes, 0))
        return arr

    def sweep(self, first, n, max_size=SWEEP_MAX) -> list:
        """Sweep cuts of resident PPR queries first .. first + n - 1 (see fork_sweep):
        one dict per query with the best prefix and the least conductance per
        size range [2^j, 2^(j+1))."""
        arr = (fork_sweep_t * max(1, n))()
        _check(lib.fork_sweep(self._ctx, first, n, max_size, ctypes.cast(arr, ctypes.c_void_p)))
        out = []
        for i in range(n):
            r = arr[i]
            out.append({"support": r.support, "swept": r.swept, "best_size": r.best_size, "flags": r.flags,
                        "best_conductance": r.best_conductance, "best_cut": r.best_cut,
                        "best_volume": r.best_volume, "size_min": list(r.size_min)})
        return out

    def bc(self, first, n) -> np.ndarray:
        """Betweenness centrality from resident BFS or SSSP queries first .. first + n - 1
        (see fork_bc): float64 [V], the sum of the sources' dependencies."""
        out = np.empty(self.num_vertices, np.float64)
        _check(lib.fork_bc(self._ctx, first, n, ctypes.c_void_p(out.ctypes.data)))
        return out

    def digest(self, qid) -> dict:
        d = fork_digest()
        _check(lib.fork_fetch(self._ctx, qid, FIELD_DIGEST, ctypes.byref(d), ctypes.sizeof(d), 0))
        return {n: getattr(d, n) for n, _ in d._fields_}

    def trace(self) -> np.ndarray:
        """Scheduler trace of the last run(trace=1): [records, 20] float32."""
        n = ctypes.c_uint64()
        _check(lib.fork_trace(self._ctx, None, 0, ctypes.byref(n)))
        out = np.empty((n.value, TRACE_WIDTH), np.float32)
        if n.value:
            _check(lib.fork_trace(self._ctx, ctypes.c_void_p(out.ctypes.data), n.value, ctypes.byref(n)))
        return out

    def stats(self) -> dict:
        s = fork_stats_t()
        _check(lib.fork_stats(self._ctx, ctypes.byref(s), ctypes.sizeof(s)))
        return s.as_dict()


def last_error() -> str:
    return lib.fork_last_error().decode()


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32))


def mlp_forward(theta, x) -> np.ndarray:
    """Scores of the partition-scoring MLP, computed on the GPU."""
    th, xx = _f32(theta), _f32(x).reshape(-1, 16)
    y = np.empty(xx.shape[0], np.float32)
    _check(lib.fork_mlp_forward(th.ctypes.data, xx.ctypes.data, xx.shape[0], y.ctypes.data))
    return y


def mlp_grad(theta, x, t):
    """(loss, grad) of the mean squared error, forward and backward on the GPU."""
    th, xx, tt = _f32(theta), _f32(x).reshape(-1, 16), _f32(t)
    g = np.empty(MLP_NPARAM, np.float32)
    loss = np.zeros(1, np.float32)
    _check(lib.fork_mlp_grad(th.ctypes.data, xx.ctypes.data, tt.ctypes.data, xx.shape[0], g.ctypes.data,
                             loss.ctypes.data))
    return float(loss[0]), g


def mlp_train(theta, x, t, steps, batch=256, lr=1e-3, seed=0):
    """Adam training on the GPU; returns (theta, per-step losses)."""
    th, xx, tt = _f32(theta).copy(), _f32(x).reshape(-1, 16), _f32(t)
    losses = np.empty(max(steps, 1), np.float32)
    _check(lib.fork_mlp_train(th.ctypes.data, xx.ctypes.data, tt.ctypes.data, xx.shape[0], steps, batch, lr, seed,
                              losses.ctypes.data))
    return th, losses[:steps]


def mlp_train_noalloc(theta, x, t, steps, batch=256, lr=1e-3, seed=0, losses=None, stream=None):
    """fork_mlp_train_noalloc on device tensors (no allocation inside the library).

    theta: float32 CUDA tensor [5313], updated in place; x [n, 16] and t [n]
    float32 CUDA tensors; losses: None or a float32 CUDA tensor [steps].  The
    work is queued on `stream` (default: torch's current stream)."""
    import torch
    for name, a in (("theta", theta), ("x", x), ("t", t)) + ((("losses", losses),) if losses is not None else ()):
        if not (a.is_cuda and a.dtype == torch.float32 and a.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    n = t.numel()
    if theta.numel() != MLP_NPARAM or x.numel() != 16 * n:
        raise ValueError("shapes: theta [5313], x [n, 16], t [n]")
    if losses is not None and losses.numel() < steps:
        raise ValueError("losses needs `steps` entries")
    s = stream if stream is not None else torch.cuda.current_stream()
    sp = s if isinstance(s, int) else s.cuda_stream
    _check(lib.fork_mlp_train_noalloc(theta.data_ptr(), x.data_ptr(), t.data_ptr(), n, steps, batch, lr, seed,
                                      None if losses is None else losses.data_ptr(), sp))
