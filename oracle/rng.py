"""Counter-based pseudo-random numbers used by the method itself (test
infrastructure only): splitmix64 as published by Steele, Lea and Flood, one
output of the generator whose state is the argument."""
from __future__ import annotations

_MASK = (1 << 64) - 1


def splitmix64(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)
