"""Exact deflation of the difference levels and the skipped-level split on the GPU,
against the CPU checker (Sec. 4.1-4.2).

* the device block-Davidson eigensolver of J_ab = Q_a^-1 - P_ab Q_b^-1 P_ab^H against
  dense eigh (3-level 24 x 16 lattice, terms (1, 2), (2, 3) and the skipped term (1, 3))
  and against ARPACK on the 128^2 hierarchy;
* every sample value of fixed-count runs with a deflated difference term and with level 2
  skipped, against the checker's direct-solve samples for the same noise indices (the
  deflation vectors imported, so the comparison isolates the projected solves), error per
  sample |s_gpu - s_ref| / (|t1| + |t2|).
"""
import numpy as np
import pytest

from oracle import difflevel as dl, mlmc as omlmc

from _helpers import oracle_deflation, oracle_hierarchy

pytestmark = pytest.mark.gpu


def _gpu_hier(gpu, name):
    torch, dm, ctx = gpu
    W, m0, lv = oracle_hierarchy(name)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                     import_tv=[l.V for l in lv[:-1]])
    return W, lv, H


@pytest.mark.parametrize("a,b", [(1, 2), (2, 3), (1, 3)])
@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_difference_eigensolver_dense(gpu, a, b, prec_name):
    torch, dm, ctx = gpu
    prec = dm.FP64 if prec_name == "fp64" else dm.MIXED
    W, lv, H = _gpu_hier(gpu, "rect24x16")
    k = 6
    ref = dl.deflate_difference(lv, a, b, k)
    d = dm.Deflation(H, a, k, eig_rtol=1e-9, level_b=b, solve_rtol=1e-13 if prec == dm.FP64 else 1e-12, prec=prec)
    assert d.status == dm.OK, d.info()
    X, lam = d.export()
    scale = np.abs(ref.lam).max()
    assert np.abs(np.sort(lam) - np.sort(ref.lam)).max() < 1e-8 * scale, (lam, ref.lam)
    Pg = X.T @ X.conj()
    Pr = ref.X @ ref.X.conj().T
    assert np.abs(Pg - Pr).max() < 1e-6
    assert abs(d.tr_defl - ref.corr) < 1e-8 * abs(ref.corr)


def test_difference_eigensolver_arpack_128(gpu):
    torch, dm, ctx = gpu
    W, lv, H = _gpu_hier(gpu, "schwinger128")
    k = 4
    ref = dl.deflate_difference(lv, 1, 2, k, method="arpack", tol=1e-12)
    d = dm.Deflation(H, 1, k, eig_rtol=1e-9, level_b=2, solve_rtol=1e-12, prec=dm.MIXED)
    assert d.status == dm.OK, d.info()
    X, lam = d.export()
    assert np.abs(np.sort(lam) - np.sort(ref.lam)).max() < 1e-8 * np.abs(ref.lam).max(), (lam, ref.lam)
    assert abs(d.tr_defl - ref.corr) < 1e-7 * abs(ref.corr)


@pytest.mark.parametrize("prec_name,rtol,tol", [("fp64", 1e-13, 1e-10), ("mixed", 1e-10, 1e-6)])
@pytest.mark.parametrize("skip", [(), (2,)])
def test_deflated_and_skipped_samples(gpu, prec_name, rtol, tol, skip):
    torch, dm, ctx = gpu
    prec = dm.FP64 if prec_name == "fp64" else dm.MIXED
    name = "rect24x16"
    W, lv, H = _gpu_hier(gpu, name)
    L = len(lv)
    cref = oracle_deflation(name, W.k_defl)
    dc = dm.Deflation(H, L, W.k_defl, import_X=cref.X, import_lambda=cref.lam)
    pairs = dl.terms(L, skip)
    a0, b0 = pairs[0]
    dref = dl.deflate_difference(lv, a0, b0, 4)
    dd = dm.Deflation(H, a0, 4, level_b=b0, import_X=dref.X, import_lambda=dref.lam)
    assert abs(dd.tr_defl - dref.corr) < 1e-10 * abs(dref.corr)
    term_defl = [None] * L
    term_defl[a0 - 1] = dd
    nsamp = 10
    res = dm.mlmc_trace(H, dc, 1e-2, W.noise_seed, [nsamp] * L, 5, prec=prec, rtol=rtol, fixed_counts=True,
                        max_samples=[nsamp] * L, keep_samples=True, skip=skip, term_defl=term_defl)
    for l in skip:
        assert res.N[l - 1] == 0
    assert abs(res.tr_defl - (cref.tr_defl + dref.corr)) < 1e-9 * abs(res.tr_defl)
    solver = omlmc.DirectSolver(lv)
    for a, b in pairs:
        got = res.samples[a - 1][:nsamp]
        for i in range(nsamp):
            s, t1, t2 = dl.pair_sample(lv, solver, W.noise_seed, a, b, i, dref if a == a0 else None)
            assert abs(got[i] - s) / (abs(t1) + abs(t2)) < tol, (a, b, i, got[i], s)
    got = res.samples[L - 1][:nsamp]
    for i in range(nsamp):
        s = omlmc.coarsest_sample(lv, solver, cref, W.noise_seed, i)
        assert abs(got[i] - s) / abs(s) < tol, (L, i)


@pytest.mark.parametrize("prec_name,srtol,tol", [("fp64", 1e-13, 1e-10), ("mixed", 1e-12, 1e-6)])
def test_inexact_difference_deflation(gpu, prec_name, srtol, tol):
    """Approximate vectors with the evaluated small term Re sum x^H Gamma5 J x (inexact
    deflation): imported perturbed vectors, and a loose device eigensolve (1e-1, solves to
    1e-3) followed by the accurate small term; samples against the checker."""
    torch, dm, ctx = gpu
    prec = dm.FP64 if prec_name == "fp64" else dm.MIXED
    W, lv, H = _gpu_hier(gpu, "rect24x16")
    exact = dl.deflate_difference(lv, 1, 2, 4)
    rng = np.random.default_rng(3)
    Xp = np.linalg.qr(exact.X + 1e-2 * (rng.normal(size=exact.X.shape) + 1j * rng.normal(size=exact.X.shape)))[0]
    ref = dl.inexact_deflation(lv, 1, 2, Xp, dense=True)
    d = dm.Deflation(H, 1, 4, level_b=2, import_X=Xp, import_lambda=ref.lam, prec=prec, corr_rtol=srtol)
    assert abs(d.tr_defl - ref.corr) < 10 * tol * abs(ref.corr), (d.tr_defl, ref.corr)
    loose = dm.Deflation(H, 1, 4, eig_rtol=1e-1, level_b=2, solve_rtol=1e-3, prec=dm.MIXED, corr_rtol=1e-12)
    X2, _ = loose.export()
    ref2 = dl.inexact_deflation(lv, 1, 2, X2.T, dense=True)
    assert abs(loose.tr_defl - ref2.corr) < 1e-7 * abs(ref2.corr)
    L = len(lv)
    nsamp = 8
    res = dm.mlmc_trace(H, None, 1e-2, W.noise_seed, [nsamp] * L, 4, prec=prec, rtol=srtol if prec == dm.FP64 else 1e-10,
                        fixed_counts=True, max_samples=[nsamp] * L, keep_samples=True, term_defl=[d] + [None] * (L - 1))
    solver = omlmc.DirectSolver(lv)
    for i in range(nsamp):
        s, t1, t2 = dl.pair_sample(lv, solver, W.noise_seed, 1, 2, i, ref)
        assert abs(res.samples[0][i] - s) / (abs(t1) + abs(t2)) < tol, (i, res.samples[0][i], s)
