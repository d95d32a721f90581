"""Pins of the CPU digest that the GPU tests compare fork_fetch(FIELD_DIGEST)
against: its mixing function reproduces the published SplitMix64 outputs
(Steele, Lea and Flood 2014: the generator seeded with 0 yields
0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, each the
finaliser of the state advanced by the golden gamma), and the digest of a
small vector worked by hand."""
import numpy as np

from digests import INF, mix64, sp_digest

GAMMA = 0x9E3779B97F4A7C15


def test_mix64_reproduces_splitmix64_seeded_with_zero():
    # output k of SplitMix64(seed 0) is the finaliser of k * gamma, which mix64 takes as (z + gamma)
    states = np.array([0, GAMMA, (2 * GAMMA) % (1 << 64)], dtype=np.uint64)
    assert [int(x) for x in mix64(states)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_sp_digest_of_a_small_vector():
    vec = np.array([0, INF, 7, INF], dtype=np.int32)
    count, total, h = sp_digest(vec)
    assert (count, total) == (2, 7)  # vertices 0 and 2 reached, values 0 and 7
    # vertex 0 with value 0 contributes mix64(0) = the first SplitMix64 output
    rest = int(mix64(np.array([(2 << 32) | 7], dtype=np.uint64))[0])
    assert h == (0xE220A8397B1DCDAF + rest) % (1 << 64)
    assert sp_digest(np.full(5, INF, dtype=np.int32)) == (0, 0, 0)
