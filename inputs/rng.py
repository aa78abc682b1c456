"""Counter-based random numbers (splitmix64, Steele, Lea and Flood 2014).

Value i of stream `seed` is mix(seed + (i + 1) * 0x9E3779B97F4A7C15), where mix is
the splitmix64 finaliser.  Being counter-based, any element can be regenerated
without replaying the stream.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n, offset=0):
    """Return n uint64 values of stream `seed`, starting at counter `offset`."""
    with np.errstate(over="ignore"):
        ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed) + ctr * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed, n, offset=0):
    """n doubles in [0, 1) from the top 53 bits of splitmix64."""
    return (splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def permutation(seed, n, offset=0):
    """A seeded random permutation of range(n): argsort of splitmix64 keys.

    Sorting i.i.d. 64-bit keys gives a uniformly random permutation (ties have
    probability ~n^2 / 2^64), equivalent in distribution to Fisher-Yates.
    """
    keys = splitmix64(seed, n, offset)
    return np.argsort(keys, kind="stable").astype(np.int64)
