"""Random draws taken by the fit (Algorithm 5 and Appendix A), oracle side.

The fit draws two kinds of random numbers: the uniform sample of at most 1e5
normalised learn vectors on which spherical k-means runs (Appendix A), and the
k-means++ seeding draws.  Both sides of the parity check (this oracle and the
device library) generate them from one counter-based generator, SplitMix64,
implemented here from its published definition (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014; the 64-bit
finaliser constants of Vigna's public reference code):

    state += 0x9E3779B97F4A7C15
    z = state
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    return z ^ (z >> 31)

A uniform double in [0, 1) is ``(r >> 11) * 2^-53``.

Order of draws for one fit with seed ``s`` (one generator, state = s):
1. if the learn set has n > 1e5 rows: a partial Fisher-Yates shuffle of
   0..n-1, step i swapping position i with ``i + r_i mod (n - i)``, for
   i < 1e5; the sample is the first 1e5 positions, sorted ascending;
2. k-means++: first centre ``r mod n_s``; then one uniform per further centre.

Test infrastructure: shares no code with the HIP path.
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & MASK

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next() >> 11) * 2.0 ** -53


def sample_without_replacement(gen: SplitMix64, n: int, s: int) -> np.ndarray:
    """Sorted ids of a uniform sample of ``min(n, s)`` rows out of ``n``."""
    if s >= n:
        return np.arange(n, dtype=np.int64)
    perm = list(range(n))
    for i in range(s):
        j = i + gen.next() % (n - i)
        perm[i], perm[j] = perm[j], perm[i]
    return np.array(sorted(perm[:s]), dtype=np.int64)
