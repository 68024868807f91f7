"""Counter-based SplitMix64 stream (Steele, Lea & Flood 2014, "Fast splittable
pseudorandom number generators"; the finaliser constants are the published
"Mix13" variant used by Java's SplittableRandom).

The k-th output of a stream seeded with ``s`` is ``mix(s + (k + 1) * GAMMA)``,
so any slice of the stream can be drawn without drawing what precedes it.
Everything here is plain integer bit-mixing; it holds none of the N-body
arithmetic and is shared by the oracle tests and the GPU tests as the single
source of seeded inputs.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class Stream:
    """A SplitMix64 stream with a running counter."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.k = 0

    def u64(self, n: int) -> np.ndarray:
        idx = np.arange(self.k + 1, self.k + 1 + n, dtype=np.uint64)
        self.k += n
        with np.errstate(over="ignore"):
            return _mix(self.seed + idx * GAMMA)

    def uniform(self, n: int) -> np.ndarray:
        """Doubles strictly inside (0, 1): ((z >> 11) + 0.5) * 2^-53."""
        z = self.u64(n) >> np.uint64(11)
        return (z.astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)

    def normal(self, n: int) -> np.ndarray:
        """Standard normals by the Box-Muller transform of two uniforms."""
        u1 = self.uniform(n)
        u2 = self.uniform(n)
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def splitmix64_reference(seed: int, count: int) -> list[int]:
    """Scalar, pure-Python form of the same stream (for self-checks)."""
    out = []
    s = seed & 0xFFFFFFFFFFFFFFFF
    mask = 0xFFFFFFFFFFFFFFFF
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & mask
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        out.append(z ^ (z >> 31))
    return out
