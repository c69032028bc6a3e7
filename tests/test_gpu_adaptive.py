"""The adaptive sample allocation and stopping rule of the MLMC loop on the GPU against
the checker's loop on the same sample stream (GPU).

The paper stops on a relative tolerance eps (Sec. 3.2; allocation as in the multilevel
Monte Carlo method it cites): start with n0 samples per level, then repeatedly set
N_l = ceil(eps^-2 T^-2 sqrt(V_l / C_l) sum_j sqrt(V_j C_j)) rounded up to the RHS block
until sqrt(sum_l V_l / N_l) <= eps |T|.  The device loop (mixed precision and FP64) and
oracle.mlmc.run (direct-solve samples of the checker's hierarchy, imported by the
device) must draw the same number of samples on every level, over at least two rounds,
and give the same estimate and error estimate.
"""
import numpy as np
import pytest

from oracle import mlmc as omlmc

from _helpers import oracle_deflation, oracle_hierarchy

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,eps", [("schwinger128", 1e-3), ("rect24x16", 2e-3)])
@pytest.mark.parametrize("prec_name,rtol,tol", [("mixed", 1e-10, 1e-6), ("fp64", 1e-13, 1e-10)])
def test_adaptive_counts_match_checker(gpu, name, eps, prec_name, rtol, tol):
    torch, dm, ctx = gpu
    prec = dm.FP64 if prec_name == "fp64" else dm.MIXED
    W, m0, lv = oracle_hierarchy(name)
    L = len(lv)
    ref_defl = oracle_deflation(name, W.k_defl)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                     import_tv=[l.V for l in lv[:-1]])
    D = dm.Deflation(H, L, W.k_defl, import_X=ref_defl.X, import_lambda=ref_defl.lam)
    n0, blk, cap = 16, 16, 8192
    print(f"[adaptive] {name} {prec_name} eps {eps}", flush=True)
    r = dm.mlmc_trace(H, D, eps, W.noise_seed, [n0] * L, blk, prec=prec, rtol=rtol, fixed_counts=False,
                      max_samples=[cap] * L, keep_samples=True)
    solver = omlmc.DirectSolver(lv)
    cost = [omlmc.sample_cost(lv, l) for l in range(1, L + 1)]
    ro = omlmc.run(lambda l, ids: omlmc.sample_values(lv, solver, ref_defl, W.noise_seed, l, ids),
                   L, cost, eps, n0, blk, ref_defl.tr_defl, max_samples=cap)
    print(f"[adaptive] device N {r.N} rel_err {r.rel_err:.4e}; checker N {ro.N} rel_err {ro.rel_err:.4e}", flush=True)
    assert max(ro.N) > n0, "the allocation never ran"
    assert max(ro.N) < cap
    assert r.N == ro.N
    assert ro.rel_err <= eps and r.rel_err <= eps
    assert abs(r.trace - ro.trace) <= tol * abs(ro.trace)
    assert abs(r.rel_err - ro.rel_err) <= 10 * tol * ro.rel_err
    for l in range(L):
        assert np.abs(r.samples[l] - ro.samples[l]).max() <= tol * np.abs(ro.samples[l]).max() * 10
