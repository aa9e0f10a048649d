"""Philox4x64-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11), in plain Python integers.

TEST INFRASTRUCTURE: part of the CPU oracle. Only tests, the smoke check and
the bench's CPU-baseline leg may import it; the product path never does.

The paper leaves the random source of the pivot draws unspecified. The draw
convention used on both sides of the parity tests is:

  key     = (seed, 0)
  counter = (t, stream, 0, 0)       t = 0-based step, stream = instance id
  w0..w3  = Philox4x64-10(counter, key)
  u1 = (w0 >> 11) * 2^-53           row draw, in [0, 1)
  u2 = (w1 >> 11) * 2^-53           column draw, in [0, 1)

With row-norm bounds and rejection sampling (Cauchy-like form), trial q of
step t uses counter (t, stream, q, 0): w0 draws the row, w2 gives the
acceptance uniform v = (w2 >> 11) * 2^-53; the column draw uses u2 of trial 0.
w3 is unused. numpy.random.Philox implements the same generator but
increments its 256-bit counter before each block; the pin test accounts for
that offset.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1

# Round multipliers and Weyl key increments of Philox4x64 (SC'11, Table 2
# and Sec. 3.3): the multipliers were chosen by the authors for avalanche;
# the key bumps are the golden ratio and sqrt(3) - 1 in 64-bit fixed point.
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B


def philox4x64_10(counter, key):
    """One 4x64-bit output block for a 4x64 counter and a 2x64 key."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c0          # exact 128-bit products
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def word_to_unit(w: int) -> float:
    """Top 53 bits of a 64-bit word as a double in [0, 1) (exact)."""
    return float(w >> 11) * (2.0 ** -53)


def step_uniforms(seed: int, stream: int, t: int):
    """(u1, u2) for step t of the run keyed by (seed, stream)."""
    w = philox4x64_10((t, stream, 0, 0), (seed, 0))
    return word_to_unit(w[0]), word_to_unit(w[1])


def trial_uniforms(seed: int, stream: int, t: int, q: int):
    """(row uniform, acceptance uniform) of trial q of step t (words w0, w2
    of counter (t, stream, q, 0))."""
    w = philox4x64_10((t, stream, q, 0), (seed, 0))
    return word_to_unit(w[0]), word_to_unit(w[2])
