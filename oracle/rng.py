"""Counter-based stratified jitter for training samples (test infrastructure).

TEST INFRASTRUCTURE ONLY (see oracle/render.py).  The random offsets xi of
stratified sampling (Sec. 2.1, Sec. 4.4) are drawn from SplitMix64 (Steele,
Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA
2014), used as a counter-based generator: output n of a SplitMix64 stream
with seed k is mix(k + (n + 1) * 0x9E3779B97F4A7C15), where
  mix(z): z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
          z = (z ^ (z >> 27)) * 0x94D049BB133111EB
          return z ^ (z >> 31)            (all mod 2^64).
For ray b of a batch and sample i of S, n = b * S + i and
xi = (mix(...) >> 40) * 2^-24, a value in [0, 1) with 24 random bits.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n) -> np.ndarray:
    """Output n (0-based, array) of the SplitMix64 stream seeded with `seed`."""
    n = np.asarray(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (n + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def stratified_xi(seed: int, n_rays: int, S: int) -> np.ndarray:
    """[n_rays, S] float64 jitter in [0, 1)."""
    n = np.arange(n_rays, dtype=np.uint64)[:, None] * np.uint64(S) + np.arange(S, dtype=np.uint64)[None, :]
    return (splitmix64(seed, n) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)
