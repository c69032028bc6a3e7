"""Pins of the bare-mass rule (CPU).

* The shift-invert path (nested-dissection LU + Lanczos) gives the same sigma_min as a
  dense eigensolve of Gamma5 D.
* Stored masses satisfy the rule they were fixed by: a local minimum of sigma_min(m), or
  sigma_min within 1e-3 of 1e-2.
"""
import json

import numpy as np
import pytest
from oracle import mass
from paper_2211_15383_amd.inputs import M0_FILE, WORKLOADS, link_angles


def test_shift_invert_matches_dense():
    theta = link_angles(24, 20, 0.3, 4)
    m = -0.07
    dense = mass.sigma_min(theta, m, method="dense")
    assert abs(mass.sigma_min(theta, m, method="shift_invert") - dense) < 1e-12


def test_nested_dissection_is_permutation():
    s = mass.nested_dissection_sites(40, 24)
    assert np.array_equal(np.sort(s), np.arange(40 * 24))


@pytest.mark.parametrize("name", ["schwinger16", "tiny8x16", "rect24x16"])
def test_stored_m0_satisfies_rule(name):
    with open(M0_FILE) as f:
        rec = json.load(f)[name]
    theta = WORKLOADS[name].theta()
    s0 = mass.sigma_min(theta, rec["m0"])
    assert abs(s0 - rec["sigma_min"]) < 1e-12
    if rec["kind"] == "crossing":
        assert abs(s0 / mass.TARGET - 1) < 1e-3
    else:
        assert s0 > mass.TARGET
        for dm in (-1e-3, 1e-3):
            assert mass.sigma_min(theta, rec["m0"] + dm) >= s0 - 1e-9
