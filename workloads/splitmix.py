"""SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), written from its published definition.

Every seeded workload in this repository draws from this one generator so
that a seed names the same input everywhere.
"""

import math

_MASK = (1 << 64) - 1


class SplitMix64:
    """64-bit SplitMix generator with the published constants."""

    __slots__ = ("state",)

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def below(self, m: int) -> int:
        """Integer in [0, m) as ``next() % m`` (the bias is < 2^-50 here)."""
        if m <= 0:
            raise ValueError("m must be positive")
        return self.next() % m

    def uniform_int(self, lo: int, hi: int) -> int:
        """Integer uniform on the closed range [lo, hi]."""
        return lo + self.below(hi - lo + 1)

    def coin(self) -> int:
        """Fair bit: the top bit of the next output."""
        return self.next() >> 63

    def unit(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next() >> 11) * (1.0 / (1 << 53))

    def exponential(self, rate: float) -> float:
        """Exponential variate with the given rate (inverse CDF)."""
        return -math.log1p(-self.unit()) / rate
