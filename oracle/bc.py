"""Betweenness centrality from a batch of single-source queries.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/`` may
import it; the product library never does.

The paper's BC (Section 2; 100 sampled sources in Section 6.1) runs one BFS
per sampled source and gathers the results with Brandes' accumulation.  On a
weighted graph the same holds with SSSP.  Definitions used here:

* sigma_st = number of shortest s-t paths, counted as edge sequences of the
  multigraph (parallel edges of equal weight are distinct paths; with
  weights >= 1 a self-loop never lies on a shortest path);
* sigma_st(v) = the shortest s-t paths through v (v != s, t);
* dependency delta_s(v) = sum over t != s, v of sigma_st(v) / sigma_st;
  delta_s(s) = 0;
* centrality over a source set S: BC(v) = sum over s in S of delta_s(v).

``dependencies`` follows Brandes' two sweeps over the shortest-path DAG of
each source:

1. sigma in order of increasing distance: sigma(w) = the sum of sigma(v)
   over DAG edges (v, w).
2. delta in order of decreasing distance: delta(v) = the sum of
   sigma(v) / sigma(w) * (1 + delta(w)) over DAG edges (v, w).

The distances come from the oracle's Dijkstra/BFS. ``brute_force``
enumerates every simple path from each source instead (tiny graphs only),
and pins the two sweeps.
"""
from __future__ import annotations

import numpy as np

from . import bfs as _bfs
from . import sssp as _sssp

INF = 0x7FFFFFFF


def _edges(g, unit):
    rp = np.asarray(g.row_ptr, np.int64)
    col = np.asarray(g.col, np.int64)
    w = np.ones(col.size, np.int64) if (unit or g.weight is None) else np.asarray(g.weight, np.int64)
    return rp, col, w


def dependencies(g, sources, unit: bool = True) -> np.ndarray:
    """delta_s(v) for each source, [n_sources, V], float64."""
    rp, col, w = _edges(g, unit)
    n = g.num_vertices
    srcs = np.asarray(sources, np.int64)
    dist = (_bfs(g, srcs) if (unit or g.weight is None) else _sssp(g, srcs)).astype(np.int64)
    out = np.zeros((srcs.size, n), np.float64)
    for i, s in enumerate(srcs):
        d = dist[i]
        reach = np.flatnonzero(d != INF)
        order = reach[np.argsort(d[reach], kind="stable")]  # non-decreasing distance
        sigma = np.zeros(n, np.float64)
        sigma[s] = 1.0
        for v in order:
            for e in range(rp[v], rp[v + 1]):
                t = col[e]
                if d[t] != INF and d[v] + w[e] == d[t]:
                    sigma[t] += sigma[v]
        delta = np.zeros(n, np.float64)
        for v in order[::-1]:
            acc = 0.0
            for e in range(rp[v], rp[v + 1]):
                t = col[e]
                if d[t] != INF and d[v] + w[e] == d[t]:
                    acc += sigma[v] / sigma[t] * (1.0 + delta[t])
            delta[v] = acc
        delta[s] = 0.0
        out[i] = delta
    return out


def centrality(g, sources, unit: bool = True) -> np.ndarray:
    """BC(v) over the given sources, float64."""
    return dependencies(g, sources, unit).sum(axis=0)


def brute_force(g, sources, unit: bool = True) -> np.ndarray:
    """delta_s(v) from every simple path out of each source, [n_sources, V] (tiny graphs)."""
    rp, col, w = _edges(g, unit)
    n = g.num_vertices
    out = np.zeros((len(sources), n), np.float64)
    for i, s in enumerate(sources):
        best = {}   # t -> shortest length found
        paths = {}  # t -> list of vertex tuples of the paths of that length
        stack = [(int(s), 0, (int(s),))]
        while stack:
            v, length, path = stack.pop()
            if v != s:
                if v not in best or length < best[v]:
                    best[v], paths[v] = length, [path]
                elif length == best[v]:
                    paths[v].append(path)
            for e in range(rp[v], rp[v + 1]):
                t = int(col[e])
                if t not in path:  # simple paths; each parallel edge is its own path
                    stack.append((t, length + int(w[e]), path + (t,)))
        for t, ps in paths.items():
            for p in ps:
                for v in p[1:-1]:
                    out[i, v] += 1.0 / len(ps)
    return out
