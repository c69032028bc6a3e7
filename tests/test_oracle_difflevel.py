"""Pins of the checker's difference-level deflation (Sec. 4.2) and skipped-level split
(Sec. 4.1, eq. 12) (CPU).

Through routes independent of the checker's formulas:
* numpy's SVD of the dense difference operator M_ab: the singular values equal |lambda(J_ab)|
  for the k largest, and M_ab v_i = s_i u_i with v_i = Gamma5 x_i, u_i = x_i sign(lambda_i)
  (eq. 16); J_ab is Hermitian (eq. 15) although M_ab is not;
* the trace split tr(M_ab) = tr(M_ab (I - Pi)) + sum_i lambda_i x_i^H Gamma5 x_i with Pi
  built from numpy's right singular vectors;
* brute force over all 2^16 Z2 vectors: the deflated samples average to tr(M_ab (I - Pi))
  and their variance is eq. (2) on M_ab (I - Pi), which is below that of M_ab;
* ARPACK on J as an operator agrees with dense eigh;
* inexact deflation: for any orthonormal X the split holds with the evaluated small term
  Re tr(M_ab V V^H) (dense trace) and reduces to the eigenpair formula for exact vectors;
* skipping a level: the composite P_13 = P_1 P_2 maps level 3 to level 1, the split of
  eq. 12 telescopes to tr(D^-1) and the per-sample sum with coupled noise reproduces
  x^H D^-1 x.
"""
import functools

import numpy as np

from oracle import difflevel as dl, mlmc, multigrid as mg, noise
from paper_2211_15383_amd.inputs import WORKLOADS, link_angles


@functools.lru_cache(maxsize=None)
def _tiny_hier():
    """8 x 4 lattice (n = 64), 2 x 2 then 2 x 1 aggregates, one test vector per chirality:
    levels of 64, 16 and 8 unknowns."""
    theta = link_angles(8, 4, 0.6, 23)
    return mg.build_hierarchy(theta, 0.1, ((2, 2), (2, 1)), (1, 1), 2, 3)


@functools.lru_cache(maxsize=None)
def _rect():
    W = WORKLOADS["rect24x16"]
    return mg.build_hierarchy(W.theta(), -0.05, W.aggs, W.ntv, W.n_inv, W.mg_seed)


def test_difference_deflation_against_svd():
    lv = _rect()
    for a, b in ((1, 2), (2, 3), (1, 3)):
        k = 6
        M = dl.M_dense(lv, a, b)
        J = dl.J_dense(lv, a, b)
        assert np.abs(J - J.conj().T).max() < 1e-10 * np.abs(J).max()
        assert np.abs(M - M.conj().T).max() > 1e-3 * np.abs(M).max()  # M itself is not Hermitian
        d = dl.deflate_difference(lv, a, b, k)
        U, S, Vh = np.linalg.svd(M)
        assert S[k - 1] - S[k] > 1e-8 * S[0]
        assert np.abs(np.abs(d.lam) - S[:k]).max() < 1e-10 * S[0]
        for i in range(k):
            u = d.X[:, i] * np.sign(d.lam[i])
            assert np.linalg.norm(M @ d.V[:, i] - abs(d.lam[i]) * u) < 1e-9 * S[0]
        # trace split with Pi from numpy's right singular vectors
        Vk = Vh[:k].conj().T
        Pi = Vk @ Vk.conj().T
        lhs = np.trace(M @ (np.eye(M.shape[0]) - Pi)) + d.corr
        assert abs(lhs - np.trace(M)) < 1e-10 * np.abs(M).sum()
        assert abs(np.trace(M @ Pi) - d.corr) < 1e-10 * abs(d.corr)


def test_brute_force_deflated_difference_samples():
    lv = _tiny_hier()
    n = lv[0].n
    assert n == 64
    d = dl.deflate_difference(lv, 1, 2, 3)
    solver = mlmc.DirectSolver(lv)
    # all 2^16 Z2 vectors of the 16 unknowns of level 2, deflated term (2, 3)
    a, b = 2, 3
    d2 = dl.deflate_difference(lv, a, b, 2)
    n2 = lv[a - 1].n
    assert n2 == 16
    bits = (np.arange(1 << n2)[None, :] >> np.arange(n2)[:, None]) & 1
    X = (1 - 2 * bits).astype(np.complex128)
    t1, t2 = dl.pair_terms(lv, solver, a, b, X, d2)
    s = t1 - t2
    M = dl.M_dense(lv, a, b)
    A = M @ (np.eye(n2) - d2.V @ d2.V.conj().T)
    assert abs(s.mean() - np.trace(A)) < 1e-12 * max(1.0, np.abs(A).sum())
    var = np.mean(np.abs(s - s.mean()) ** 2)
    assert abs(var - mlmc.z2_variance(A)) < 1e-10 * mlmc.z2_variance(A)
    assert mlmc.z2_variance(A) < mlmc.z2_variance(M)
    # undeflated pair terms are the ordinary difference-level sample
    u1, u2 = dl.pair_terms(lv, solver, a, b, X[:, :64])
    v1, v2 = mlmc.difference_terms(lv, solver, a, X[:, :64])
    assert np.abs((u1 - u2) - (v1 - v2)).max() < 1e-12 * np.abs(v1).max()
    # the same deflated sample at the fine level against the dense formula
    x = noise.z2_noise(4, 1, 7, n).astype(np.complex128)
    sd, _, _ = dl.pair_sample(lv, solver, 4, 1, 2, 7, d)
    M1 = dl.M_dense(lv, 1, 2)
    ref = np.vdot(x, M1 @ (x - d.V @ (d.V.conj().T @ x)))
    assert abs(sd - ref) < 1e-11 * abs(ref)


def test_arpack_matches_dense():
    lv = _rect()
    dd = dl.deflate_difference(lv, 1, 2, 6, method="dense")
    da = dl.deflate_difference(lv, 1, 2, 6, method="arpack")
    assert np.abs(dd.lam - da.lam).max() < 1e-9 * np.abs(dd.lam).max()
    Pd = dd.X @ dd.X.conj().T
    Pa = da.X @ da.X.conj().T
    assert np.abs(Pd - Pa).max() < 1e-7
    assert abs(dd.corr - da.corr) < 1e-9 * abs(dd.corr)


def test_skip_level_split():
    lv = _rect()
    L = len(lv)
    assert dl.terms(L, skip=(2,)) == [(1, 3)]
    assert dl.terms(4, skip=(2,)) == [(1, 3), (3, 4)]
    P13 = dl.composite_P(lv, 1, 3)
    assert P13.shape == (lv[0].n, lv[2].n)
    # eq. 14 carries over: Gamma5 P_13 = P_13 Gamma5
    assert abs(lv[0].gamma5 @ P13 - P13 @ lv[2].gamma5).max() < 1e-14
    # eq. 12: tr(D_1^-1 - P_13 D_3^-1 P_13^H) + tr(D_3^-1) = tr(D^-1)
    tr = np.trace(dl.M_dense(lv, 1, 3)) + np.trace(mlmc.dense_inverse(lv, 3))
    exact = np.trace(mlmc.dense_inverse(lv, 1))
    assert abs(tr - exact) < 1e-11 * abs(exact)
    # per sample with coupled noise (y = P_13^H x): the two terms add up to x^H D^-1 x
    solver = mlmc.DirectSolver(lv)
    x = noise.z2_noise(5, 1, 3, lv[0].n).astype(np.complex128)
    t1, t2 = dl.pair_terms(lv, solver, 1, 3, x)
    y = P13.conj().T @ x
    total = t1 - t2 + np.vdot(y, solver.solve(3, y))
    assert abs(total - np.vdot(x, solver.solve(1, x))) < 1e-11 * abs(t1)


def test_inexact_deflation_split():
    lv = _rect()
    a, b = 1, 2
    M = dl.M_dense(lv, a, b)
    n = M.shape[0]
    rng = np.random.default_rng(3)
    exact = dl.deflate_difference(lv, a, b, 4)
    # approximate vectors: exact ones perturbed, re-orthonormalised
    Xp = np.linalg.qr(exact.X + 1e-2 * (rng.normal(size=exact.X.shape) + 1j * rng.normal(size=exact.X.shape)))[0]
    for X in (Xp, np.linalg.qr(rng.normal(size=(n, 3)) + 1j * rng.normal(size=(n, 3)))[0]):
        d = dl.inexact_deflation(lv, a, b, X, dense=True)
        Pi = d.V @ d.V.conj().T
        small = np.trace(M @ Pi)
        assert abs(d.corr - small.real) < 1e-10 * np.abs(M).sum()
        assert abs(np.trace(M @ (np.eye(n) - Pi)) + small - np.trace(M)) < 1e-10 * np.abs(M).sum()
        solver = mlmc.DirectSolver(lv)
        ds = dl.inexact_deflation(lv, a, b, X, solver=solver)
        assert abs(ds.corr - d.corr) < 1e-10 * abs(d.corr)
    de = dl.inexact_deflation(lv, a, b, exact.X, dense=True)
    assert abs(de.corr - exact.corr) < 1e-10 * abs(exact.corr)
    assert np.abs(de.lam - exact.lam).max() < 1e-10 * np.abs(exact.lam).max()
