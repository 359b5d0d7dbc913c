"""Counter-based SplitMix64 streams (Steele, Lea & Flood, OOPSLA 2014).

Output i of the stream keyed by (seed, tag) is mix64(s0 + (i + 1) * GAMMA)
with s0 = seed XOR tag, all arithmetic modulo 2**64.  That is exactly the
sequential SplitMix64 generator started from state s0, evaluated by counter so
a whole stream is one vectorised numpy expression.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# One independent stream per kind of draw.  The values are arbitrary
# distinct 64-bit constants.
STREAM_TAGS = {
    "jitter": 0x6A69747465720001,
    "state": 0x7374617465000002,
    "perm_cell": 0x7065726D63000003,
    "perm_edge": 0x7065726D65000004,
    "perm_node": 0x7065726D6E000005,
    "perm_bedge": 0x7065726D62000006,
    "hex_jitter": 0x68656A6974000007,
    "hex_vel": 0x68657676656C0008,
    "perm_elem": 0x7065726D6C000009,
    "mesh_size": 0x6D73697A6500000A,
}


def splitmix64(seed: int, tag: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+n-1 of the SplitMix64 stream keyed by (seed, tag)."""
    s0 = np.uint64((int(seed) ^ int(tag)) & 0xFFFFFFFFFFFFFFFF)
    i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = s0 + i * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(bits: np.ndarray) -> np.ndarray:
    """Top 53 bits as a double in [0, 1): (x >> 11) * 2**-53 (exact)."""
    return (bits >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform(bits: np.ndarray, lo: float, hi: float) -> np.ndarray:
    return lo + (hi - lo) * uniform01(bits)


def random_permutation(seed: int, tag: int, n: int) -> np.ndarray:
    """A uniform random permutation of 0..n-1 from one stream.

    perm[r] is the element whose key ranks r-th; keys are the stream's
    64-bit outputs and ties (probability ~ n^2 / 2^65) are broken by index
    through a stable sort, so the result is fully specified.
    """
    keys = splitmix64(seed, tag, n)
    return np.argsort(keys, kind="stable").astype(np.int64)
