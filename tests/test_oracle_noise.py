"""Pins of the checker's counter-based noise (CPU).

* SplitMix64 reproduces the generator's published output streams (tests/golden/
  splitmix64_published.txt, cited there).
* The vectorised Z2/Z4 expansion agrees with the scalar definition entry by entry.
* Z2 entries are +-1 with E[x_j] = 0 and E[x_j x_k] = delta_jk (Sec. 2, eq. 2's
  assumptions) to within sampling error; Z4 entries are the four roots of unity.
* Frozen values (tests/golden/noise_golden.json, written by make_golden.py) guard against
  drift; the HIP generator is checked bit-exactly against the same function.
"""
import json
import os

import numpy as np

from oracle import noise

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _published():
    rows = []
    with open(os.path.join(GOLDEN, "splitmix64_published.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                vals = [int(v) for v in line.split()]
                rows.append((vals[0], vals[1:]))
    return rows


def test_splitmix64_published_streams():
    rows = _published()
    assert len(rows) == 2
    for seed, outs in rows:
        assert noise.splitmix64_stream(seed, len(outs)) == outs


def test_z2_matches_scalar_definition():
    seed, level, sample, n = 12345, 3, 17, 400
    x = noise.z2_noise(seed, level, sample, n)
    base = noise.sm((noise.sm((noise.sm(seed) + level) & noise.MASK) + sample) & noise.MASK)
    for j in range(n):
        w = noise.sm((base + j // 64) & noise.MASK)
        assert x[j] == 1 - 2 * ((w >> (j % 64)) & 1)


def test_z4_matches_scalar_definition():
    seed, level, vec, n = 7, 2, 5, 150
    z = noise.z4_start(seed, level, vec, n)
    base = noise.sm((noise.sm((noise.sm(seed) + level + 32) & noise.MASK) + vec) & noise.MASK)
    roots = [1, 1j, -1, -1j]
    for j in range(n):
        w = noise.sm((base + j // 32) & noise.MASK)
        assert z[j] == roots[(w >> (2 * (j % 32))) & 3]


def test_z2_moments():
    n, m = 4096, 64
    X = np.column_stack([noise.z2_noise(3, 1, i, n) for i in range(m)])
    assert set(np.unique(X)) == {-1.0, 1.0}
    assert abs(X.mean()) < 5.0 / np.sqrt(X.size)
    C = X @ X.T / m                      # E[x_j x_k] estimate over samples
    off = C[~np.eye(n, dtype=bool)]
    assert np.allclose(np.diag(C), 1.0)
    assert abs(off.mean()) < 5.0 / np.sqrt(off.size * m) + 1e-3
    assert off.std() < 1.2 / np.sqrt(m)
    # different levels and samples give different streams
    assert not np.array_equal(noise.z2_noise(3, 1, 0, n), noise.z2_noise(3, 2, 0, n))


def test_z4_values_uniform():
    z = noise.z4_start(1, 1, 0, 40000)
    c = np.rint(np.angle(z) / (np.pi / 2)).astype(int) % 4
    counts = np.bincount(c, minlength=4)
    assert np.all(np.abs(counts - 10000) < 500)
    assert np.allclose(np.abs(z), 1.0)


def test_noise_frozen_values():
    with open(os.path.join(GOLDEN, "noise_golden.json")) as f:
        g = json.load(f)
    for r in g["z2"]:
        x = noise.z2_noise(r["seed"], r["level"], r["sample"], len(r["bits"]))
        assert "".join("1" if v < 0 else "0" for v in x) == r["bits"]
    for r in g["z4"]:
        z = noise.z4_start(r["seed"], r["level"], r["vec"], len(r["c"]))
        c = np.rint(np.angle(z) / (np.pi / 2)).astype(int) % 4
        assert "".join(str(v) for v in c) == r["c"]
