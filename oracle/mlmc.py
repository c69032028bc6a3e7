"""Multigrid multilevel Monte Carlo with exact deflation of the coarsest term (oracle; test only).

Hutchinson (eq. 1) on every term of the telescoping sum (eq. 11):

    tr(D^-1) = sum_{l<L} tr(D_l^-1 - P_l D_{l+1}^-1 P_l^H) + tr(D_L^-1 (I - Pi)) + tr(D_L^-1 Pi)

with the coarsest term split by exact deflation (eq. 5, small term eq. 6-7).  Sample i of
level l uses its own real Z2 vector x = z2_noise(seed, l, i, n_l):

    difference level l < L:  s = x^H D_l^-1 x - y^H D_{l+1}^-1 y,   y = P_l^H x
    coarsest level L:        s = x^H D_L^-1 (x - W W^H x)

All solves are direct (sparse LU).  The estimate is Re(sum_l mean_l) + tr(D_L^-1 Pi) and
its relative error sqrt(sum_l var_l / N_l) / |estimate| (var: sample variance of the
complex samples, E|s - mean|^2, ddof = 1).

Sample allocation (the paper cites Giles' multilevel Monte Carlo for it and gives only
the relative tolerance eps): N_l* = ceil(eps^-2 T^-2 sqrt(V_l / C_l) sum_j sqrt(V_j C_j)),
rounded up to a whole number of sample blocks, repeated until the error estimate is at
most eps.  C_l is a fixed work proxy: the stencil entries touched by one application of
every operator the level's sample solves with (fine level: 18 per site; coarse level with
d dofs per site: 5 d^2 per site), so that runs in different precisions draw the same
samples.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.sparse.linalg as spla

from . import noise
from .deflation import Deflation
from .multigrid import Level


def level_work(levels: Sequence[Level], l: int) -> float:
    """Work proxy of one operator application at level l (1-based)."""
    lv = levels[l - 1]
    sites = lv.Lx * lv.Lt
    return 18.0 * sites if l == 1 else 5.0 * lv.dofs * lv.dofs * sites


def sample_cost(levels: Sequence[Level], l: int) -> float:
    L = len(levels)
    return level_work(levels, l) + (level_work(levels, l + 1) if l < L else 0.0)


class DirectSolver:
    """Sparse LU of every level operator, computed on first use."""

    def __init__(self, levels: Sequence[Level]):
        self.levels = levels
        self._lu = {}

    def solve(self, l: int, b: np.ndarray) -> np.ndarray:
        if l not in self._lu:
            self._lu[l] = spla.splu(self.levels[l - 1].D.tocsc())
        return self._lu[l].solve(np.asarray(b, dtype=np.complex128))


def difference_terms(levels, solver: DirectSolver, l: int, x: np.ndarray):
    """(x^H D_l^-1 x, y^H D_{l+1}^-1 y) with y = P_l^H x; x may hold one noise vector per column."""
    z = solver.solve(l, x)
    y = levels[l - 1].P.conj().T @ x
    zc = solver.solve(l + 1, y)
    return np.sum(x.conj() * z, axis=0), np.sum(y.conj() * zc, axis=0)


def coarsest_term(levels, solver: DirectSolver, defl: Optional[Deflation], x: np.ndarray):
    """x^H D_L^-1 (x - W W^H x); x may hold one noise vector per column."""
    L = len(levels)
    xt = x if defl is None else x - defl.W @ (defl.W.conj().T @ x)
    return np.sum(x.conj() * solver.solve(L, xt), axis=0)


def difference_sample(levels, solver: DirectSolver, seed: int, l: int, i: int):
    """(s, x^H D_l^-1 x, y^H D_{l+1}^-1 y) for sample i of difference level l < L."""
    x = noise.z2_noise(seed, l, i, levels[l - 1].n)
    t1, t2 = difference_terms(levels, solver, l, x)
    return complex(t1 - t2), complex(t1), complex(t2)


def coarsest_sample(levels, solver: DirectSolver, defl: Optional[Deflation], seed: int, i: int):
    L = len(levels)
    x = noise.z2_noise(seed, L, i, levels[L - 1].n)
    return complex(coarsest_term(levels, solver, defl, x))


def hutchinson_term(levels, solver: DirectSolver, defl: Optional[Deflation], x: np.ndarray):
    """Plain Hutchinson at the fine level with exact deflation (eq. 1 with the split of
    eq. 5 applied to D_1): x^H D_1^-1 (x - W W^H x), W from a deflation of level 1; x may
    hold one noise vector per column."""
    xt = x if defl is None else x - defl.W @ (defl.W.conj().T @ x)
    return np.sum(x.conj() * solver.solve(1, xt), axis=0)


def hutchinson_sample(levels, solver: DirectSolver, defl: Optional[Deflation], seed: int, i: int):
    """Sample i of the deflated fine-level Hutchinson estimator; its noise is that of level 1."""
    x = noise.z2_noise(seed, 1, i, levels[0].n)
    return complex(hutchinson_term(levels, solver, defl, x))


def sample_values(levels, solver: DirectSolver, defl: Optional[Deflation], seed: int, l: int,
                  ids) -> np.ndarray:
    L = len(levels)
    if l < L:
        return np.array([difference_sample(levels, solver, seed, l, i)[0] for i in ids])
    return np.array([coarsest_sample(levels, solver, defl, seed, i) for i in ids])


def sample_var(s: np.ndarray) -> float:
    s = np.asarray(s)
    if s.size < 2:
        return 0.0
    return float(np.sum(np.abs(s - s.mean()) ** 2) / (s.size - 1))


def estimate(samples: List[np.ndarray], tr_defl: float):
    """(T, Im part, relative error) from per-level complex samples."""
    means = [np.mean(s) for s in samples]
    T = float(np.real(np.sum(means))) + tr_defl
    var_over_n = sum(sample_var(s) / s.size for s in samples)
    err = math.sqrt(var_over_n) / abs(T) if T != 0 else math.inf
    return T, float(np.imag(np.sum(means))), err


def allocation(var: Sequence[float], cost: Sequence[float], T: float, eps: float) -> List[int]:
    s = sum(math.sqrt(v * c) for v, c in zip(var, cost))
    return [int(math.ceil(math.sqrt(v / c) * s / (eps * eps * T * T))) for v, c in zip(var, cost)]


@dataclass
class MLMCResult:
    trace: float
    trace_imag: float
    rel_err: float
    N: List[int]
    samples: List[np.ndarray] = field(repr=False)
    tr_defl: float = 0.0


def run(sample_fn: Callable[[int, range], np.ndarray], L: int, cost: Sequence[float], eps: float,
        n0: int, block: int, tr_defl: float, fixed: bool = False,
        max_samples: int = 1 << 20) -> MLMCResult:
    """Adaptive MLMC loop; sample_fn(l, ids) returns the sample values of level l."""
    def roundup(m):
        return ((m + block - 1) // block) * block

    samples = [np.zeros(0, dtype=np.complex128) for _ in range(L)]
    targets = [roundup(n0)] * L
    while True:
        for l in range(1, L + 1):
            have = samples[l - 1].size
            if targets[l - 1] > have:
                new = sample_fn(l, range(have, targets[l - 1]))
                samples[l - 1] = np.concatenate([samples[l - 1], new])
        T, Ti, err = estimate(samples, tr_defl)
        if fixed or err <= eps:
            break
        var = [sample_var(s) for s in samples]
        want = allocation(var, cost, T, eps)
        grew = False
        for l in range(L):
            t = min(roundup(max(want[l], samples[l].size)), max_samples)
            if t > samples[l].size:
                targets[l] = t
                grew = True
        if not grew:
            break
    return MLMCResult(T, Ti, err, [s.size for s in samples], samples, tr_defl)


# ---------------------------------------------------------------- dense references (tiny lattices)

def dense_inverse(levels, l: int) -> np.ndarray:
    return np.linalg.inv(levels[l - 1].D.toarray())


def difference_operator(levels, l: int) -> np.ndarray:
    """M_l = D_l^-1 - P_l D_{l+1}^-1 P_l^H (eq. 13), dense."""
    P = levels[l - 1].P.toarray()
    return dense_inverse(levels, l) - P @ dense_inverse(levels, l + 1) @ P.conj().T


def z2_variance(A: np.ndarray) -> float:
    """Variance of x^H A x for real Z2 noise: 1/2 ||offdiag(A + A^T)||_F^2 (eq. 2)."""
    B = A + A.T
    B = B - np.diag(np.diag(B))
    return 0.5 * float(np.sum(np.abs(B) ** 2))
