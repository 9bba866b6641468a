"""Counter-based SplitMix64 stream and Box-Muller normals.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the k-th output of a stream with seed s is the
64-bit finaliser applied to s + (k+1) * 0x9E3779B97F4A7C15 (mod 2^64).
Being counter based, element k can be produced without producing 0..k-1,
which keeps every draw reproducible independently of numpy's generators.
"""

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset..offset+count-1 of the SplitMix64 stream for `seed` (uint64)."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in (0, 1]: the top 53 bits of each output, plus one, times 2^-53."""
    z = splitmix64(seed, count, offset)
    return ((z >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def gaussian(seed: int, count: int) -> np.ndarray:
    """Standard normal draws by the Box-Muller transform on consecutive uniform pairs."""
    npairs = (count + 1) // 2
    u = uniform01(seed, 2 * npairs)
    u1, u2 = u[0::2], u[1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * npairs)
    out[0::2] = rad * np.cos(2.0 * np.pi * u2)
    out[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return out[:count]
