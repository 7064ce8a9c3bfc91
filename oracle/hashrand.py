"""Counter-based generator used where the method draws random numbers.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then two
xor-shift-multiply rounds and a final xor-shift.  A key is hashed by chaining
the mixer over its integer fields, and a double in [0, 1) is the top 53 bits.

The GPU library implements the same published definition on its own; the
two share no code.  Test infrastructure only.
"""
M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def hkey(*vals: int) -> int:
    h = 0
    for v in vals:
        h = splitmix64(h ^ (int(v) & M64))
    return h


def u01(h: int) -> float:
    return (h >> 11) * (1.0 / (1 << 53))
