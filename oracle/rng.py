"""Counter-based SplitMix64 Rademacher probes.

TEST INFRASTRUCTURE ONLY (see the package header).

The stochastic trace estimate of Section 2.1 uses Rademacher probe vectors.
The library takes them from the caller; its optional device generator follows
the published SplitMix64 generator (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014, with the 64-bit finaliser of
Vigna's reference implementation splitmix64.c), and this module implements
the same definition on its own, so that the two can be compared bit for bit.

Definition.  Seeded with s, the generator's state after t steps is
s_t = s + t * GAMMA (mod 2^64), GAMMA = 0x9E3779B97F4A7C15, and its t-th output
(t = 1, 2, ...) is mix(s_t), where mix xors in the value shifted right by 30,
multiplies by 0xBF58476D1CE4E5B9, xors in the value shifted right by 27,
multiplies by 0x94D049BB133111EB and xors in the value shifted right by 31
(all modulo 2^64).  Element (i, c) of an n x ncols probe block takes output
t = i * ncols + c + 1 and is -1 if that output's top bit is set, else +1.

Parity status: pinned (tests/test_oracle_rng.py) by the reference
implementation's published outputs for two seeds, by the closed counter form
agreeing with the sequential state update, and by the signs' balance.
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1


def mix(z):
    """SplitMix64's finaliser on a Python int (modulo 2^64)."""
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


def splitmix64_stream(seed, count):
    """The first `count` outputs, by stepping the state one GAMMA at a time
    (pure Python, for small counts)."""
    s = seed & MASK
    out = []
    for _ in range(count):
        s = (s + GAMMA) & MASK
        out.append(mix(s))
    return out


def splitmix64_at(seed, t):
    """Outputs number t (an integer array, t >= 1) in closed counter form,
    uint64 arithmetic wrapping modulo 2^64."""
    t = np.asarray(t, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK) + t * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        return z ^ (z >> np.uint64(31))


def rademacher(n, ncols, seed):
    """n x ncols block of +-1 (float64): element (i, c) from output
    i * ncols + c + 1."""
    t = np.arange(1, n * ncols + 1, dtype=np.uint64)
    z = splitmix64_at(seed, t)
    return np.where((z >> np.uint64(63)) == 1, -1.0, 1.0).reshape(n, ncols)
