"""Counter-based noise for the Hutchinson samples and the setup start vectors (oracle; test only).

The paper draws Z2 noise (Sec. 2, eq. 2: entries +-1, E[x_i] = 0, E[x_i x_j] = delta_ij)
but names no generator.  Both sides of the parity tests implement the same published
counter-based generator, SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), so that every
sample value is a function of (seed, level, sample index) alone and is bit-identical
whatever the RHS block size or the order in which blocks are processed.

SM(z) is one SplitMix64 step from state z: add the golden gamma 0x9E3779B97F4A7C15,
then the variant-13 finaliser (xor-shift 30, multiply 0xBF58476D1CE4E5B9, xor-shift 27,
multiply 0x94D049BB133111EB, xor-shift 31), all modulo 2^64.

Z2 entry j of sample i at level l (1-based l, 0-based i and j):
    w = SM(SM(SM(SM(seed) + l) + i) + floor(j / 64)),  x_j = 1 - 2 * ((w >> (j % 64)) & 1)
Z4 entry j of setup start vector v at level l:
    w = SM(SM(SM(SM(seed) + l + 32) + v) + floor(j / 32)),  c = (w >> (2 (j % 32))) & 3,
    value i^c in {1, i, -1, -i}.
"""
from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def sm(z: int) -> int:
    """One SplitMix64 step from state z (pure Python integers, exact)."""
    z = (z + GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64_stream(seed: int, count: int):
    """The generator's published output sequence from `seed`: state += gamma, output mix(state)."""
    out = []
    state = seed & MASK
    for _ in range(count):
        out.append(sm(state))
        state = (state + GOLDEN) & MASK
    return out


def _sm_array(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64) + np.uint64(GOLDEN)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def z2_noise(seed: int, level: int, sample: int, n: int) -> np.ndarray:
    """Real Z2 vector (+1/-1, float64) of length n for (seed, level, sample)."""
    base = sm((sm((sm(seed) + level) & MASK) + sample) & MASK)
    j = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        w = _sm_array(np.uint64(base) + (j >> np.uint64(6)))
    bits = (w >> (j & np.uint64(63))) & np.uint64(1)
    return 1.0 - 2.0 * bits.astype(np.float64)


def z4_start(seed: int, level: int, vec: int, n: int) -> np.ndarray:
    """Complex Z4 start vector (entries in {1, i, -1, -i}) for the setup of level `level`."""
    base = sm((sm((sm(seed) + level + 32) & MASK) + vec) & MASK)
    j = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        w = _sm_array(np.uint64(base) + (j >> np.uint64(5)))
    c = ((w >> (np.uint64(2) * (j & np.uint64(31)))) & np.uint64(3)).astype(np.int64)
    return np.array([1.0, 1.0j, -1.0, -1.0j], dtype=np.complex128)[c]
