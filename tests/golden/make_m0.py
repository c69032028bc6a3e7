"""Fixes the bare mass m0 of each workload by the sigma_min ~ 1e-2 rule and writes
tests/golden/m0.json.  Calls only the CPU checker (oracle.mass) and the seeded link
generator.  Run from the repository root:

    python tests/golden/make_m0.py [workload ...]

Entries already in the file are kept unless named on the command line.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mass  # noqa: E402
from paper_2211_15383_amd.inputs import M0_FILE, WORKLOADS, batched_fields  # noqa: E402

# scan start per workload (default +0.1); the 1024^2 scan starts closer to the crossing
# to keep the number of 2M-unknown factorisations small.
M_START = {"schwinger1024": -0.04}


def main(names):
    table = {}
    if os.path.exists(M0_FILE):
        with open(M0_FILE) as f:
            table = json.load(f)
    all_w = dict(WORKLOADS)
    all_w.update({w.name: w for w in batched_fields()})
    if not names:
        names = [n for n in all_w if n not in table]
    for name in names:
        w = all_w[name]
        t = time.time()
        m0, s, kind = mass.m0_rule(w.theta(), m_start=M_START.get(name, 0.1))
        table[name] = {"m0": m0, "sigma_min": s, "kind": kind, "Lx": w.Lx, "Lt": w.Lt,
                       "sigma": w.sigma, "link_seed": w.link_seed}
        print(f"{name}: m0={m0:.8f} sigma_min={s:.6g} ({kind}, {time.time() - t:.1f} s)", flush=True)
        with open(M0_FILE, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
