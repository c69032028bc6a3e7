"""Fixes the bare mass m0 of each workload by the sigma_min ~ 1e-2 rule and writes
tests/golden/m0.json.  Calls only the CPU checker (oracle.mass) and the seeded link
generator.  Run from the repository root:

    python tests/golden/make_m0.py [--jobs J] [--scan-points K] [workload ...]

Entries already in the file are kept unless named on the command line.  Every scan
starts at +0.1.  With --scan-points K the first K masses of the scan are evaluated
beforehand in J parallel processes (each one sparse factorisation; at 1024^2 about
3 minutes and 9 GB apiece); the rule itself then runs unchanged on those values.  The
(m, sigma_min) pairs the rule asked for are kept in the record ("evaluations"), so that
the rule can be replayed from them.
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mass  # noqa: E402
from paper_2211_15383_amd.inputs import M0_FILE, WORKLOADS, batched_fields  # noqa: E402

M_START = 0.1
STEP = 0.005


def _all_workloads():
    all_w = dict(WORKLOADS)
    all_w.update({w.name: w for w in batched_fields()})
    return all_w


def _sigma_at(args):
    name, m = args
    t = time.time()
    s = mass.sigma_min(_all_workloads()[name].theta(), m)
    print(f"  {name}: sigma_min({m:+.6f}) = {s:.9g} ({time.time() - t:.0f} s)", flush=True)
    return m, s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--jobs", type=int, default=1)
    ap.add_argument("--scan-points", type=int, default=0)
    a = ap.parse_args()
    table = {}
    if os.path.exists(M0_FILE):
        with open(M0_FILE) as f:
            table = json.load(f)
    all_w = _all_workloads()
    names = a.names or [n for n in all_w if n not in table]
    for name in names:
        w = all_w[name]
        t = time.time()
        known = {}
        if a.scan_points > 0:
            pts = mass.scan_points(M_START, STEP, a.scan_points)
            with ProcessPoolExecutor(max_workers=a.jobs) as ex:
                known = dict(ex.map(_sigma_at, [(name, m) for m in pts]))
        theta = w.theta()
        used = []

        def sigma_fn(m):
            if m not in known:
                known[m] = _sigma_at((name, m))[1]
            used.append([m, known[m]])
            return known[m]

        m0, s, kind = mass.m0_rule(theta, m_start=M_START, step=STEP, sigma_fn=sigma_fn)
        rec = {"m0": m0, "sigma_min": s, "kind": kind, "Lx": w.Lx, "Lt": w.Lt,
               "sigma": w.sigma, "link_seed": w.link_seed, "m_start": M_START,
               # every (m, sigma_min) the rule asked for, in its order
               "evaluations": used}
        table[name] = rec
        print(f"{name}: m0={m0:.12f} sigma_min={s:.9g} ({kind}, {time.time() - t:.1f} s)", flush=True)
        with open(M0_FILE, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
