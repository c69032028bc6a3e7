"""Pins of the checker's large-operator solvers (CPU).

* NDLU (nested-dissection LU + refinement) reproduces a plain sparse LU solve and reaches
  a relative residual near machine precision.
* Block-Jacobi: one undamped sweep solves a block-diagonal operator exactly.
* Two-level iteration of eq. (8): for b = D P c (b in the range of D P) the coarse-grid
  correction alone returns x = P c exactly (this fails for P and P^H swapped, a wrong
  coarse operator or a sign error in the residual); the V-cycle is a linear map.
* FGMRES: with the identity preconditioner on a small dense system it returns the numpy
  solve; with the V-cycle it reaches 1e-13 and matches the sparse LU solution.
* HybridSolver with every large level forced onto FGMRES gives the same sample values as
  the direct solver of oracle.mlmc on a three-level hierarchy.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import mlmc as omlmc, multigrid as omg, noise as onoise, solvers, wilson
from paper_2211_15383_amd.inputs import WORKLOADS, link_angles


def _hier(name, m0=-0.06, n_inv=1):
    W = WORKLOADS[name]
    return W, omg.build_hierarchy(W.theta(), m0, W.aggs, W.ntv, n_inv, W.mg_seed)


def test_ndlu_matches_splu():
    theta = link_angles(24, 20, 0.3, 4)
    lv = omg.Level(24, 20, 2, wilson.dirac_operator(theta, -0.07))
    rng = np.random.default_rng(0)
    b = rng.normal(size=(lv.n, 3)) + 1j * rng.normal(size=(lv.n, 3))
    x = solvers.NDLU(lv).solve(b)
    ref = spla.splu(lv.D.tocsc()).solve(b)
    assert np.abs(x - ref).max() < 1e-11 * np.abs(ref).max()
    assert solvers.relres(lv.D, x, b).max() < 1e-14


def test_block_jacobi_solves_block_diagonal_operator():
    rng = np.random.default_rng(1)
    ns, d = 12, 4
    blocks = rng.normal(size=(ns, d, d)) + 1j * rng.normal(size=(ns, d, d)) + 4 * np.eye(d)
    D = sp.block_diag(list(blocks)).tocsr()
    lv = omg.Level(4, 3, d, D)
    b = rng.normal(size=ns * d) + 1j * rng.normal(size=ns * d)
    x = solvers.BlockJacobi(lv, 1.0).sweeps(b, np.zeros_like(b), 1)
    assert np.abs(D @ x - b).max() < 1e-13


def test_coarse_grid_correction_is_exact_on_range_of_DP():
    W, lv = _hier("schwinger16")
    mg = solvers.VCycle(lv, 1, 2, nu_pre=0, nu_post=0)
    c = onoise.z2_noise(3, 2, 0, lv[1].n).astype(np.complex128) * (1 + 0.5j)
    b = lv[0].D @ (lv[0].P @ c)
    x = mg.apply(b)
    assert np.abs(x - lv[0].P @ c).max() < 1e-12 * np.abs(c).max()


def test_vcycle_is_linear():
    W, lv = _hier("rect24x16")
    mg = solvers.VCycle(lv, 1, 3)
    rng = np.random.default_rng(2)
    u = rng.normal(size=lv[0].n) + 1j * rng.normal(size=lv[0].n)
    v = rng.normal(size=lv[0].n) + 1j * rng.normal(size=lv[0].n)
    a = 0.3 - 1.7j
    lhs = mg.apply(a * u + v)
    rhs = a * mg.apply(u) + mg.apply(v)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_fgmres_identity_preconditioner_dense():
    rng = np.random.default_rng(3)
    n = 60
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) + 12 * np.eye(n)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    x, res, it = solvers.fgmres(lambda v: A @ v, b, lambda v: v, 1e-13, restart=25)
    assert res <= 1e-13
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-11 * np.abs(x).max()


@pytest.mark.parametrize("level", [1, 2])
def test_fgmres_vcycle_matches_lu(level):
    W, lv = _hier("schwinger64")
    bottom = 3
    mg = solvers.VCycle(lv, level, bottom)
    D = lv[level - 1].D
    b = onoise.z2_noise(5, level, 0, lv[level - 1].n).astype(np.complex128)
    x, res, it = solvers.fgmres(lambda v: D @ v, b, mg.apply, 1e-13)
    assert res <= 1e-13
    ref = spla.splu(D.tocsc()).solve(b)
    assert np.abs(x - ref).max() < 1e-10 * np.abs(ref).max()


def test_hybrid_solver_matches_direct_samples():
    W, lv = _hier("schwinger64")
    direct = omlmc.DirectSolver(lv)
    # lu_max below the level-2 size: level 1 -> ND LU, level 2 -> FGMRES + V-cycle, level 3 -> LU
    hybrid = solvers.HybridSolver(lv, rtol=1e-13, lu_max=lv[2].n)
    assert hybrid.uses_lu(1) and not hybrid.uses_lu(2) and hybrid.uses_lu(3)
    for l in (1, 2):
        for i in range(2):
            s_d, t1_d, t2_d = omlmc.difference_sample(lv, direct, 9, l, i)
            s_h, t1_h, t2_h = omlmc.difference_sample(lv, hybrid, 9, l, i)
            assert abs(s_h - s_d) <= 1e-11 * (abs(t1_d) + abs(t2_d)), (l, i)
