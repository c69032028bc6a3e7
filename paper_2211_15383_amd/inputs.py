"""Seeded synthetic inputs shared by the HIP path's tests, the benchmark and the CPU checker.

This module holds no arithmetic of the method.  It only

* draws the U(1) gauge-link angles theta_mu(x) i.i.d. from N(0, sigma^2) with numpy's
  PCG64 generator (the paper's own 128^2 gauge configuration, Section 4.3, is not
  public; i.i.d. angles at the same lattice shapes stand in for it), and
* lists the workloads (lattice sizes, aggregates, test vectors, deflation size, seeds,
  tolerances) the library is exercised and measured on.

The bare mass m0 of each workload is not drawn here: it is fixed once by the rule
"sigma_min(D) ~ 1e-2" and stored in ``tests/golden/m0.json`` (see ``load_m0``).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

_REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
M0_FILE = os.path.join(_REPO, "tests", "golden", "m0.json")


def link_angles(Lx: int, Lt: int, sigma: float, seed: int) -> np.ndarray:
    """Gauge-link angles theta[mu, t, x] (mu = 0: x direction, mu = 1: t direction).

    U_mu(x, t) = exp(i * theta[mu, t, x]).  Values are i.i.d. N(0, sigma^2) from
    ``numpy.random.default_rng(seed)``; sigma = 0 gives the free field U = 1.
    """
    if sigma == 0.0:
        return np.zeros((2, Lt, Lx), dtype=np.float64)
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, sigma, size=(2, Lt, Lx)).astype(np.float64)


@dataclass(frozen=True)
class Workload:
    name: str
    Lx: int
    Lt: int
    sigma: float
    link_seed: int
    aggs: Tuple[Tuple[int, int], ...]   # aggregate extents (ax, at) per coarsening step
    ntv: Tuple[int, ...]                # test vectors per chirality per coarsening step
    k_defl: int                         # deflation vectors at the coarsest level
    noise_seed: int
    mg_seed: int = 7                    # seed of the Z4 start vectors of the setup
    n_inv: int = 3                      # inverse-iteration steps of the setup
    eps: float = 1e-2                   # relative trace tolerance of the stopping rule
    rtol: float = 1e-10                 # relative residual of each solve
    n0: int = 32                        # initial samples per level
    rhs_block: int = 32
    notes: str = ""

    @property
    def nlevels(self) -> int:
        return len(self.aggs) + 1

    @property
    def n_fine(self) -> int:
        return 2 * self.Lx * self.Lt

    def level_dims(self) -> List[Tuple[int, int, int]]:
        """(Lx_l, Lt_l, dofs per site) for l = 1..L."""
        dims = [(self.Lx, self.Lt, 2)]
        for (ax, at), N in zip(self.aggs, self.ntv):
            Lx, Lt, _ = dims[-1]
            dims.append((Lx // ax, Lt // at, 2 * N))
        return dims

    def theta(self) -> np.ndarray:
        return link_angles(self.Lx, self.Lt, self.sigma, self.link_seed)


WORKLOADS = {
    # 16^2, two levels, dense-LU exact trace available.
    "schwinger16": Workload("schwinger16", 16, 16, 0.3, 1, ((4, 4),), (4,), 16,
                            noise_seed=11, n0=200, rhs_block=40),
    # 128^2, three levels, FP64 and mixed precision.
    "schwinger128": Workload("schwinger128", 128, 128, 0.3, 2, ((4, 4), (4, 4)), (8, 8), 32,
                             noise_seed=12, n0=32),
    # 1024^2, four levels; the measured workload.
    "schwinger1024": Workload("schwinger1024", 1024, 1024, 0.3, 5,
                              ((4, 4), (4, 4), (2, 2)), (8, 8, 8), 128,
                              noise_seed=15, n0=32),
    # small shapes for parity tests (odd aggregate counts, non-square lattices)
    "tiny8x16": Workload("tiny8x16", 8, 16, 0.3, 3, ((2, 4),), (2,), 4, noise_seed=13, n0=8),
    "rect24x16": Workload("rect24x16", 24, 16, 0.3, 4, ((4, 4), (3, 2)), (4, 3), 6,
                          noise_seed=14, n0=8),
    "schwinger64": Workload("schwinger64", 64, 64, 0.3, 6, ((4, 4), (4, 4)), (8, 8), 32,
                            noise_seed=16, n0=32),
}


def batched_fields() -> List[Workload]:
    """The multi-field batch: 4 fields each at 64^2, 128^2, 256^2.

    Field j at size index s uses sigma = (0.2, 0.3, 0.4, 0.3)[j] and link seed
    1000 + 10 * s + j; three levels with 4x4 aggregates and 8 test vectors per chirality,
    k = 32, 512 samples per level.
    """
    out = []
    for s, L in enumerate((64, 128, 256)):
        for j, sig in enumerate((0.2, 0.3, 0.4, 0.3)):
            out.append(Workload(f"field{L}_{j}", L, L, sig, 1000 + 10 * s + j,
                                ((4, 4), (4, 4)), (8, 8), 32, noise_seed=14, n0=512))
    return out


def load_m0(name: str) -> float:
    """The bare mass of a workload, fixed once by the sigma_min ~ 1e-2 rule."""
    with open(M0_FILE) as f:
        table = json.load(f)
    if name not in table:
        raise KeyError(f"no m0 stored for workload {name!r} in {M0_FILE}")
    return float(table[name]["m0"])
