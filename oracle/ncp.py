"""Sweep cuts and the network community profile (NCP) from PPR vectors.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/`` may
import it; the product library never does.

The paper runs NCP as one PPR per seed vertex (Sections 2 and 6.1: seeds are
0.01% of the vertices, after Shun et al.), and defines the profile as the
best conductance of a cluster of each size.  It does not print the sweep
itself.  The reading used here is the standard local-clustering sweep:

* The graph is read as undirected.  Every directed edge (u, v) of the
  multigraph is one undirected edge.  d(v) = out-degree + in-degree, so a
  self-loop adds 2.  vol(S) = sum of d over S; the total volume is 2|E|.
* cut(S) = number of directed edges with exactly one endpoint in S.
* conductance(S) = cut(S) / min(vol(S), 2|E| - vol(S)); undefined when that
  minimum is 0.
* Sweep of a vector p: the vertices with p[v] > 0 and d(v) > 0, in
  decreasing p[v] / d(v).  The key is computed in fp32, the precision of
  the GPU's p, as fp32(p[v]) / fp32(d(v)).  Equal keys go in increasing
  ``pos[v]`` (the library's internal position; the vertex id when no order
  is given).  Prefix S_k holds the first k vertices, k = 1..K with
  K = min(max_size, support).
* Best cut of a sweep: the k with the least conductance (the smallest k on
  ties).
* NCP: for each size range [2^j, 2^(j+1)), the least conductance of any
  prefix of any seed's sweep whose size falls in the range.

Two implementations of the prefix profile are kept on purpose.
``sweep_profile_direct`` evaluates the definition for every prefix from a
membership mask (O(K |E|), small graphs).  ``sweep_profile`` adds one
vertex at a time: when v joins S, each edge between v and a vertex already
in S stops being cut and every other edge at v starts being cut.  The tests
pin the second to the first.
"""
from __future__ import annotations

import numpy as np


def _endpoints(g):
    rp = np.asarray(g.row_ptr, np.int64)
    src = np.repeat(np.arange(g.num_vertices, dtype=np.int64), np.diff(rp))
    dst = np.asarray(g.col, np.int64)
    return src, dst


def degrees(g) -> np.ndarray:
    """d(v) = out-degree + in-degree (each directed edge is one undirected edge)."""
    src, dst = _endpoints(g)
    n = g.num_vertices
    return np.bincount(src, minlength=n).astype(np.int64) + np.bincount(dst, minlength=n).astype(np.int64)


def sweep_order(g, p, max_size=None, pos=None) -> np.ndarray:
    """Vertex ids of the sweep, in order, truncated to max_size."""
    p = np.asarray(p, np.float32)
    d = degrees(g)
    pos = np.arange(g.num_vertices, dtype=np.int64) if pos is None else np.asarray(pos, np.int64)
    sup = np.flatnonzero((p > 0) & (d > 0))
    key = p[sup] / d[sup].astype(np.float32)  # fp32 division, as on the GPU
    order = sup[np.lexsort((pos[sup], -key.astype(np.float64)))]  # key descending, then position ascending
    return order if max_size is None else order[:max_size]


def sweep_profile_direct(g, p, max_size=None, pos=None):
    """(order, cut[k], vol[k], phi[k]) for k = 1..K, each prefix evaluated from the definition."""
    order = sweep_order(g, p, max_size, pos)
    src, dst = _endpoints(g)
    d = degrees(g)
    total = 2 * src.size
    inside = np.zeros(g.num_vertices, bool)
    cut = np.zeros(order.size, np.int64)
    vol = np.zeros(order.size, np.int64)
    for k, v in enumerate(order):
        inside[v] = True
        cut[k] = np.count_nonzero(inside[src] != inside[dst])
        vol[k] = d[inside].sum()
    return order, cut, vol, _phi(cut, vol, total)


def sweep_profile(g, p, max_size=None, pos=None):
    """The same profile, one vertex at a time (adjacency in both directions)."""
    order = sweep_order(g, p, max_size, pos)
    src, dst = _endpoints(g)
    d = degrees(g)
    total = 2 * src.size
    n = g.num_vertices
    # undirected incidence lists: every directed edge is listed at both endpoints
    ends = np.concatenate([src, dst])
    other = np.concatenate([dst, src])
    srt = np.argsort(ends, kind="stable")
    start = np.searchsorted(ends[srt], np.arange(n + 1))
    nbr = other[srt]
    rank = np.full(n, -1, np.int64)
    cut = np.zeros(order.size, np.int64)
    vol = np.zeros(order.size, np.int64)
    c = 0
    s = 0
    for k, v in enumerate(order):
        rank[v] = k
        inc = nbr[start[v]:start[v + 1]]
        # a self-loop is listed twice at v and stays uncut; an edge to S is no longer cut
        # (it was counted when its other end joined); every other incident edge is now cut
        joined = np.count_nonzero((rank[inc] >= 0) & (inc != v))
        c += inc.size - np.count_nonzero(inc == v) - 2 * joined
        s += d[v]
        cut[k] = c
        vol[k] = s
    return order, cut, vol, _phi(cut, vol, total)


def _phi(cut, vol, total):
    den = np.minimum(vol, total - vol).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(den > 0, cut / den, np.inf)


def best_cut(phi):
    """(k, conductance) of the least-conductance prefix (1-based k; smallest k on ties), or (0, inf)."""
    if phi.size == 0 or not np.isfinite(phi).any():
        return 0, float("inf")
    k = int(np.argmin(phi))
    return k + 1, float(phi[k])


def ncp(profiles, max_size):
    """Least conductance per size range [2^j, 2^(j+1)) over all given phi arrays."""
    nb = int(max_size).bit_length()
    best = np.full(nb, np.inf)
    for phi in profiles:
        sizes = np.arange(1, phi.size + 1)
        b = np.floor(np.log2(sizes)).astype(np.int64)
        np.minimum.at(best, b, phi)
    return best
