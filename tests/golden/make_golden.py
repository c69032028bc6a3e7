"""Writes the frozen noise values in tests/golden/noise_golden.json.

Calls only the CPU checker (oracle.noise).  Each Z2 record stores the +-1 entries of
one sample vector as a bit string (bit = 1 for -1), Z4 records store c with value i^c.
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import noise  # noqa: E402

CASES_Z2 = [(11, 1, 0, 300), (11, 1, 1, 300), (11, 2, 0, 300), (15, 4, 12345, 300),
            (0, 1, 0, 130), (2**63 + 5, 3, 2**40, 200)]
CASES_Z4 = [(7, 1, 0, 100), (7, 2, 3, 100), (99, 1, 7, 70)]


def main():
    out = {"z2": [], "z4": []}
    for seed, level, sample, n in CASES_Z2:
        x = noise.z2_noise(seed, level, sample, n)
        out["z2"].append({"seed": seed, "level": level, "sample": sample,
                          "bits": "".join("1" if v < 0 else "0" for v in x)})
    for seed, level, vec, n in CASES_Z4:
        z = noise.z4_start(seed, level, vec, n)
        c = np.rint(np.angle(z) / (np.pi / 2)).astype(int) % 4
        out["z4"].append({"seed": seed, "level": level, "vec": vec,
                          "c": "".join(str(v) for v in c)})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "noise_golden.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
