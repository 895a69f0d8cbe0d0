"""SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) as a counter-based generator.

``splitmix64(c)`` returns the output of the SplitMix64 finaliser applied to
``c * GOLDEN`` (mod 2^64), i.e. the c-th output of a SplitMix64 stream started
from state 0.  Streams are addressed by adding a 64-bit key to the counter.
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(counter):
    """Vectorised SplitMix64 output for uint64 counters (wraps mod 2^64)."""
    z = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, n, stream=0):
    """n doubles in [0, 1): (k >> 11) * 2^-53 for k = splitmix64(key + i)."""
    key = np.uint64((int(seed) * 0x100000001B3 + int(stream) * 0x9E3779B1) % (1 << 64))
    with np.errstate(over="ignore"):
        k = splitmix64(key + np.arange(n, dtype=np.uint64))
    return (k >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def integers(seed, n, stream, modulus):
    key = np.uint64((int(seed) * 0x100000001B3 + int(stream) * 0x9E3779B1) % (1 << 64))
    with np.errstate(over="ignore"):
        k = splitmix64(key + np.arange(n, dtype=np.uint64))
    return (k % np.uint64(modulus)).astype(np.int64)
