"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module generates graphs and query sources only; it contains none of the
fork-processing arithmetic.  Heavy loops live in ``gen.c`` (built with gcc into
``libfpp_gen.so`` next to this file).

Workloads (the paper measures real graphs that are not available here; these
synthetic graphs stand in for them):

* R-MAT (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), edge factor 16, directed,
  duplicates and self-loops kept -- stands in for the paper's social and web
  graphs (power-law, average degree about 16).
* 4-neighbour 2D grid, both directions of every edge -- stands in for the
  paper's high-diameter road networks.
* Integer weights uniform on an inclusive range; the two directions of a grid
  edge share one weight.
* Sources: uniform without replacement over vertices with out-degree >= 1,
  or uniform over the top 1% of vertices by out-degree (ties: lower id).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfpp_gen.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile gen.c into libfpp_gen.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _get_lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            lib.fi_rmat_edges.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_uint64, P, P]
            lib.fi_uniform_weights.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                               ctypes.c_uint64, P, P]
            lib.fi_grid_csr.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P, P, P]
            lib.fi_build_csr.argtypes = [ctypes.c_uint32, ctypes.c_uint64, P, P, P, P, P]
            _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class Graph:
    """Directed multigraph in CSR form (row_ptr: uint64[V+1], col: uint32[E])."""
    num_vertices: int
    row_ptr: np.ndarray
    col: np.ndarray
    weight: Optional[np.ndarray]  # uint32[E] or None (unweighted)
    name: str = ""

    @property
    def num_edges(self) -> int:
        return int(self.row_ptr[-1])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def stats(self) -> dict:
        src = np.repeat(np.arange(self.num_vertices, dtype=np.int64), self.out_degree())
        key = src * self.num_vertices + self.col.astype(np.int64)
        dup = int(key.size - np.unique(key).size)
        deg = self.out_degree()
        indeg = np.bincount(self.col, minlength=self.num_vertices)
        return {
            "V": self.num_vertices, "E": self.num_edges, "duplicates": dup,
            "self_loops": int(np.count_nonzero(src == self.col)),
            "outdeg0": int(np.count_nonzero(deg == 0)),
            "isolated": int(np.count_nonzero((deg == 0) & (indeg == 0))),
            "max_outdeg": int(deg.max()) if deg.size else 0,
        }


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, weights: Optional[tuple] = None, weight_seed: int = 101) -> Graph:
    """R-MAT graph with 2**scale vertices and edge_factor * 2**scale edges."""
    lib = _get_lib()
    nv = 1 << scale
    ne = edge_factor * nv
    src = np.empty(ne, np.uint32)
    dst = np.empty(ne, np.uint32)
    lib.fi_rmat_edges(scale, ne, a, b, c, seed, _ptr(src), _ptr(dst))
    row_ptr = np.empty(nv + 1, np.uint64)
    col = np.empty(ne, np.uint32)
    perm = np.empty(ne, np.uint64) if weights is not None else None
    lib.fi_build_csr(nv, ne, _ptr(src), _ptr(dst), _ptr(row_ptr), _ptr(col), _ptr(perm))
    del src, dst
    w = None
    if weights is not None:
        w = np.empty(ne, np.uint32)
        lib.fi_uniform_weights(ne, int(weights[0]), int(weights[1]), weight_seed, _ptr(perm), _ptr(w))
    return Graph(nv, row_ptr, col, w, name=f"rmat{scale}")


def grid(rows: int, cols: int, weights: Optional[tuple] = (1, 1000), weight_seed: int = 103) -> Graph:
    """4-neighbour grid, both directions; a grid edge's two directions share one weight."""
    lib = _get_lib()
    nv = rows * cols
    ne = 4 * rows * cols - 2 * rows - 2 * cols
    row_ptr = np.empty(nv + 1, np.uint64)
    col = np.empty(ne, np.uint32)
    und = np.empty(ne, np.uint64)
    lib.fi_grid_csr(rows, cols, _ptr(row_ptr), _ptr(col), _ptr(und))
    w = None
    if weights is not None:
        w = np.empty(ne, np.uint32)
        lib.fi_uniform_weights(ne, int(weights[0]), int(weights[1]), weight_seed, _ptr(und), _ptr(w))
    return Graph(nv, row_ptr, col, w, name=f"grid{rows}x{cols}")


def from_edges(num_vertices: int, src, dst, weight=None, name: str = "edges") -> Graph:
    """CSR from an explicit edge list (stable by input order); for small test graphs."""
    lib = _get_lib()
    src = np.ascontiguousarray(src, np.uint32)
    dst = np.ascontiguousarray(dst, np.uint32)
    ne = src.size
    row_ptr = np.empty(num_vertices + 1, np.uint64)
    col = np.empty(max(ne, 1), np.uint32)[:ne]
    perm = np.empty(max(ne, 1), np.uint64)[:ne]
    lib.fi_build_csr(num_vertices, ne, _ptr(src), _ptr(dst), _ptr(row_ptr), _ptr(col), _ptr(perm))
    w = None
    if weight is not None:
        w = np.ascontiguousarray(np.asarray(weight, np.uint32)[perm.astype(np.int64)])
    return Graph(num_vertices, row_ptr, col, w, name=name)


def random_small(n: int, m: int, seed: int, wmax: int = 9, weighted: bool = True) -> Graph:
    """Small random multigraph (duplicates, self-loops, dangling vertices possible)."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    w = rng.integers(1, wmax + 1, m) if weighted else None
    return from_edges(n, src, dst, w, name=f"small{n}_{m}_{seed}")


def sources_uniform(g: Graph, n: int, seed: int) -> np.ndarray:
    """n distinct sources, uniform over vertices with out-degree >= 1."""
    cand = np.flatnonzero(g.out_degree() > 0).astype(np.uint32)
    rng = np.random.Generator(np.random.PCG64(seed))
    if n > cand.size:
        return rng.choice(cand, n, replace=True).astype(np.uint32)
    return rng.choice(cand, n, replace=False).astype(np.uint32)


def top_degree_set(g: Graph, frac: float = 0.01) -> np.ndarray:
    """The ceil(frac*V) vertices of largest out-degree, ties broken by lower id."""
    k = int(np.ceil(frac * g.num_vertices))
    deg = g.out_degree()
    order = np.lexsort((np.arange(g.num_vertices), -deg))
    return order[:k].astype(np.uint32)


def sources_top(g: Graph, n: int, seed: int, frac: float = 0.01) -> np.ndarray:
    """n sources uniform over the top-frac out-degree set (without replacement if possible)."""
    cand = top_degree_set(g, frac)
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.choice(cand, n, replace=n > cand.size).astype(np.uint32)


def sources_mixed(g: Graph, n: int, seed: int) -> np.ndarray:
    """Half uniform (out-degree >= 1), half from the top 1% by out-degree, interleaved."""
    nu = n - n // 2
    u = sources_uniform(g, nu, seed)
    t = sources_top(g, n // 2, seed + 7919)
    out = np.empty(n, np.uint32)
    out[0::2] = u
    out[1::2] = t
    return out


# The workloads.  Seeds are fixed per workload: (graph, weights, sources).
WORKLOADS = {
    "rmat12_sssp64": dict(kind="rmat", scale=12, weights=(1, 255), seeds=(1, 101, 201),
                          queries=[("sssp", 64, "uniform")]),
    # PPR forward push at scale 20: the threshold epsilon scaled by the vertex's
    # degree (the variant the degree-normalised push of the paper's PPR uses) ...
    "rmat20_ppr4096": dict(kind="rmat", scale=20, weights=None, seeds=(2, 102, 202),
                           queries=[("ppr", 4096, "uniform")], alpha=0.15, epsilon=1e-6, eps_mode=1),
    # ... and with the absolute threshold r(u) >= epsilon, the same graph and sources
    "rmat20_ppr4096_abs": dict(kind="rmat", scale=20, weights=None, seeds=(2, 102, 202),
                               queries=[("ppr", 4096, "uniform")], alpha=0.15, epsilon=1e-6, eps_mode=0),
    "grid2048_sssp1024_bfs1024": dict(kind="grid", rows=2048, cols=2048, weights=(1, 1000),
                                      seeds=(3, 103, 203),
                                      queries=[("sssp", 1024, "uniform"), ("bfs", 1024, "uniform")]),
    "rmat22_mixed16384": dict(kind="rmat", scale=22, weights=(1, 255), seeds=(4, 104, 204),
                              queries=[("sssp", 8192, "mixed"), ("bfs", 4096, "mixed"),
                                       ("ppr", 4096, "mixed")], alpha=0.15, epsilon=1e-6, eps_mode=1),
    # scaled-down stand-in of the scale-23 SSSP+PPR mix (same generator, same mix, fewer vertices/queries)
    "rmat20_sssp_ppr2048": dict(kind="rmat", scale=20, weights=(1, 255), seeds=(6, 106, 206),
                                queries=[("sssp", 1024, "mixed"), ("ppr", 1024, "mixed")],
                                alpha=0.15, epsilon=1e-6, eps_mode=1),
    "rmat23_sssp_ppr65536": dict(kind="rmat", scale=23, weights=(1, 255), seeds=(5, 105, 205),
                                 queries=[("sssp", 32768, "mixed"), ("ppr", 32768, "mixed")],
                                 alpha=0.15, epsilon=1e-6, eps_mode=1),
}


def make_graph(spec: dict, scale_override: Optional[int] = None) -> Graph:
    gs, ws, _ = spec["seeds"]
    if spec["kind"] == "rmat":
        return rmat(scale_override or spec["scale"], seed=gs, weights=spec["weights"], weight_seed=ws)
    return grid(spec["rows"], spec["cols"], weights=spec["weights"], weight_seed=ws)


def make_sources(g: Graph, spec: dict) -> list:
    """[(query_type, sources)] in submit order."""
    _, _, ss = spec["seeds"]
    out = []
    for k, (qt, n, how) in enumerate(spec["queries"]):
        seed = ss * 1000 + k
        if how == "uniform":
            s = sources_uniform(g, n, seed)
        elif how == "mixed":
            s = sources_mixed(g, n, seed)
        else:
            raise ValueError(how)
        out.append((qt, s))
    return out
