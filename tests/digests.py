"""The per-query SSSP/BFS digest that fork_fetch(FIELD_DIGEST) returns,
computed on the CPU from a distance vector: the count of reached vertices,
the sum of their values, and the sum over reached vertices v of
mix64((v << 32) | value(v)) mod 2^64, where mix64 is the SplitMix64
finaliser (Steele, Lea and Flood 2014).  Test infrastructure."""
import numpy as np

INF = np.int32(0x7FFFFFFF)


def mix64(z):
    """SplitMix64 finaliser, vectorised over uint64."""
    with np.errstate(over="ignore"):
        z = (z + np.uint64(0x9E3779B97F4A7C15)).astype(np.uint64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def sp_digest(vec):
    """(count, sum, hash) of an int32 distance or level vector."""
    v = np.flatnonzero(vec != INF)
    x = vec[v].astype(np.uint64)
    with np.errstate(over="ignore"):
        h = np.sum(mix64((v.astype(np.uint64) << np.uint64(32)) | x), dtype=np.uint64)
    return int(v.size), int(x.sum()), int(h)
