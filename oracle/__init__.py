"""CPU oracle for the fork-processing pattern.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The product library never links, imports or executes it, and it
shares no code, header or table with the GPU path.

What it computes (every function is the plain definition, or the paper's
sequential algorithm, with no blocking or reordering):

* ``sssp``        -- Dijkstra per source (Section 4.1 reuses sequential
                     Dijkstra; Definition 2.3 defines the SSSP operation).
* ``bfs``         -- BFS levels per source (Section 3, supported queries).
* ``forward_push``-- sequential fp64 forward push for PPR (Section 4.1 reuses
                     a sequential PPR; Section 4.2 orders pushes by residual,
                     but any order gives a valid push result).
* ``ppr_power``   -- fp64 power iteration of the PPR linear system, the exact
                     vector that forward push approximates.
* ``sp_certificate`` -- optimality certificate for shortest distances.
* ``mlp``         -- fp64 forward/backward of the partition-scoring MLP.
* ``ncp``         -- sweep-cut conductance profiles of PPR vectors and the
                     network community profile (numpy).
* ``bc``          -- Brandes' dependencies and betweenness centrality over
                     a batch of sources (numpy, distances from ``sssp``/``bfs``).

Readings where the paper is silent (no PPR formula, alpha, epsilon or
dangling-vertex rule is printed): the walk is substochastic (a vertex without
out-edges drops its (1-alpha) share), the push threshold is absolute
(``r[u] >= eps``) in mode 0 and degree-scaled (``r[u] >= eps*outdeg(u)``) in
mode 1.  Unreachable distances and levels are INT32_MAX.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import mlp  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None
INF = np.int32(0x7FFFFFFF)


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _get_lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P, U32, U64, I, D = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_double)
            lib.or_sssp_many.argtypes = [U32, P, P, P, U32, P, P, P, I]
            lib.or_bfs_many.argtypes = [U32, P, P, U32, P, P, P, I]
            lib.or_push_many.argtypes = [U32, P, P, U32, P, D, D, I, P, P, P, I]
            lib.or_ppr_power_many.argtypes = [U32, P, P, D, U32, P, D, I, P, I]
            lib.or_sp_certificate.argtypes = [U32, P, P, P, U32, P]
            for f in (lib.or_sssp_many, lib.or_bfs_many, lib.or_push_many, lib.or_ppr_power_many,
                      lib.or_sp_certificate):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _threads(n):
    return int(n) if n else (os.cpu_count() or 1)


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, np.uint64)
    col = np.ascontiguousarray(g.col, np.uint32)
    w = None if g.weight is None else np.ascontiguousarray(g.weight, np.uint32)
    return rp, col, w


def sssp(g, sources, threads=None, return_work=False):
    """int32 [n_sources, V] shortest distances; INT32_MAX if unreachable."""
    rp, col, w = _csr(g)
    srcs = np.ascontiguousarray(sources, np.uint32)
    out = np.empty((srcs.size, g.num_vertices), np.int32)
    work = np.zeros(srcs.size, np.uint64)
    rc = _get_lib().or_sssp_many(g.num_vertices, _p(rp), _p(col), _p(w), srcs.size, _p(srcs), _p(out),
                                 _p(work), _threads(threads))
    if rc:
        raise OverflowError("a finite distance does not fit in int32")
    return (out, work) if return_work else out


def bfs(g, sources, threads=None, return_work=False):
    """int32 [n_sources, V] hop levels; INT32_MAX if unreachable."""
    rp, col, _ = _csr(g)
    srcs = np.ascontiguousarray(sources, np.uint32)
    out = np.empty((srcs.size, g.num_vertices), np.int32)
    work = np.zeros(srcs.size, np.uint64)
    _get_lib().or_bfs_many(g.num_vertices, _p(rp), _p(col), srcs.size, _p(srcs), _p(out), _p(work),
                           _threads(threads))
    return (out, work) if return_work else out


def forward_push(g, sources, alpha, eps, mode=0, threads=None, return_work=False):
    """fp64 (p, r), each [n_sources, V], from sequential forward push."""
    rp, col, _ = _csr(g)
    srcs = np.ascontiguousarray(sources, np.uint32)
    p = np.empty((srcs.size, g.num_vertices), np.float64)
    r = np.empty_like(p)
    work = np.zeros(srcs.size, np.uint64)
    _get_lib().or_push_many(g.num_vertices, _p(rp), _p(col), srcs.size, _p(srcs), float(alpha),
                            float(eps), int(mode), _p(p), _p(r), _p(work), _threads(threads))
    return (p, r, work) if return_work else (p, r)


def ppr_power(g, x0, alpha, tol=1e-14, max_iter=100000, threads=None):
    """fp64 alpha * sum_k ((1-alpha) P^T)^k x0 for each row of x0 [n, V]."""
    rp, col, _ = _csr(g)
    x0 = np.ascontiguousarray(np.atleast_2d(x0), np.float64)
    pi = np.empty_like(x0)
    _get_lib().or_ppr_power_many(g.num_vertices, _p(rp), _p(col), float(alpha), x0.shape[0], _p(x0),
                                 float(tol), int(max_iter), _p(pi), _threads(threads))
    return pi


def ppr_exact(g, sources, alpha, threads=None):
    """PPR vectors of the given sources, [n_sources, V], fp64."""
    srcs = np.asarray(sources, np.int64)
    x0 = np.zeros((srcs.size, g.num_vertices), np.float64)
    x0[np.arange(srcs.size), srcs] = 1.0
    return ppr_power(g, x0, alpha, threads=threads)


def sp_certificate(g, source, dist, unit_weights=False) -> int:
    """0 if ``dist`` is exactly the shortest-distance vector from ``source``."""
    rp, col, w = _csr(g)
    if unit_weights:
        w = None
    d = np.ascontiguousarray(dist, np.int32)
    return _get_lib().or_sp_certificate(g.num_vertices, _p(rp), _p(col), _p(w), int(source), _p(d))


def ppr_invariant_l1(g, source, p, r, alpha, threads=None) -> float:
    """|| p - PPR(e_s - r) ||_1 in fp64: zero in exact arithmetic for any push result.

    Forward push keeps p + PPR(r) = PPR(e_s) (push invariant), so by
    linearity p must equal PPR(e_s - r)."""
    x0 = -np.asarray(r, np.float64).copy()
    x0[int(source)] += 1.0
    ref = ppr_power(g, x0[None, :], alpha, threads=threads)[0]
    return float(np.abs(np.asarray(p, np.float64) - ref).sum())


def push_terminal(g, r, eps, mode=0, dtype=np.float64) -> bool:
    """True if no vertex is active: r[u] <= 0 or r[u] < thr(u) for all u.

    ``dtype`` is the precision in which the threshold decision is taken: the
    fp64 oracle decides in fp64; an fp32 push decides with
    thr = fp32(eps) * fp32(outdeg) in fp32, so its result is checked that way."""
    r = np.asarray(r, dtype)
    e = dtype(eps)
    thr = e * g.out_degree().astype(dtype) if mode else np.full(r.shape, e, dtype)
    return bool(np.all((r <= 0) | (r < thr)))
