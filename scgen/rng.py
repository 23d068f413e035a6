"""SplitMix64 (S. Vigna, public domain generator used to seed xoshiro), in a
counter-based, vectorised form.

The k-th output (k = 0, 1, ...) of the stream with initial state s is
mix(s + (k+1) * GOLDEN) with the published finaliser constants; computing it
from the counter lets numpy produce any slice of a stream in one shot.
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream seeded with `seed`."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + k * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_uniform(seed: int, count: int, lo: float = -1.0, hi: float = 1.0,
                       start: int = 0) -> np.ndarray:
    """Uniform doubles in [lo, hi) from the top 53 bits of each output."""
    z = splitmix64(seed, count, start)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u


def stream_seed(base_seed: int, index: int) -> int:
    """Seed of the per-subdomain stream number `index` of a configuration."""
    return (base_seed + index * 0x9E3779B97F4A7C15) & MASK64


def signs_from_seed(seed: int, m: int) -> np.ndarray:
    """+1/-1 per multiplier: -1 when the top bit of the output is set."""
    z = splitmix64(seed, m)
    return np.where((z >> np.uint64(63)) != 0, -1, 1).astype(np.int8)
