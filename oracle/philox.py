"""Philox4x64-10 counter-based generator (oracle side).

Test infrastructure: this module is part of the CPU oracle. Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may use it.

Written from the published definition of the Philox family (Salmon, Moraes,
Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4-word
counter is passed through 10 rounds, each of which multiplies words 0 and 2
by two fixed odd constants, swaps the high/low halves around and XORs in the
round key; the 2-word key is bumped by two Weyl constants between rounds.
The paper being reproduced draws its Bernoulli picks (Algorithm 2) without
naming a generator; this one is used because both the CPU oracle and the GPU
library can evaluate it at any (key, counter) independently, so the same seed
yields the same picks on both sides.

Pure Python integers: slow, exact, and independent of numpy's own Philox
(which the tests use as the pin).
"""

MASK64 = (1 << 64) - 1

# Multipliers and Weyl key increments of Philox4x64 (SC'11, Table 2 / text).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B


def _mulhilo(a, b):
    p = a * b
    return (p >> 64) & MASK64, p & MASK64


def philox4x64_10(counter, key):
    """Return the 4 output words for a 4-word counter and a 2-word key."""
    x0, x1, x2, x3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        hi0, lo0 = _mulhilo(PHILOX_M0, x0)
        hi1, lo1 = _mulhilo(PHILOX_M1, x2)
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def uniform_u64(seed, stream, index):
    """The draw used by the samplers: word 0 of the block at counter
    (index, 0, 0, 0) under key (seed, stream)."""
    return philox4x64_10((index, 0, 0, 0), (seed, stream))[0]
