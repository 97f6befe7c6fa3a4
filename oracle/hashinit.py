"""Counter-based initial guess of a new mode -- oracle, test infrastructure only.

The paper initialises each new mode without saying how (Sec. 3.3, step 1).
A constant guess fails for zero-mean cosine data (the right-hand side of the
first directional solve vanishes), so the reading used here is a
deterministic pseudo-random guess in [-1, 1] drawn from splitmix64 (Steele,
Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
keyed by (seed, time step, mode, direction, node).  The HIP library carries
its own implementation of the same published generator.
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(x: int) -> int:
    """One splitmix64 output for counter x (state advanced by the golden gamma)."""
    z = (x + GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def mode_key(seed: int, step: int, mode: int, direction: int) -> int:
    k = (seed * 1000003 + step) & MASK
    k = (k * 1000003 + mode) & MASK
    k = (k * 8 + direction) & MASK
    return (k << 32) & MASK


def init_vector(seed: int, step: int, mode: int, direction: int, n: int) -> np.ndarray:
    """u[i] = 2 * U53(splitmix64(key + i)) - 1, U53(z) = (z >> 11) * 2^-53."""
    base = mode_key(seed, step, mode, direction)
    out = np.empty(n)
    for i in range(n):
        z = splitmix64((base + i) & MASK)
        out[i] = 2.0 * ((z >> 11) * 2.0 ** -53) - 1.0
    return out
