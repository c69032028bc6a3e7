"""The RHS-block autotuner (GPU): it measures every candidate, records the fastest in the
hierarchy, and an estimate with rhs_block = 0 then draws exactly the samples of an
estimate with that block size given explicitly (sample values are independent of the
block size, so both agree with the checker's samples as well)."""
import numpy as np
import pytest

from oracle import mlmc as omlmc

from _helpers import oracle_deflation, oracle_hierarchy

pytestmark = pytest.mark.gpu


def test_tuned_block_estimate(gpu):
    torch, dm, ctx = gpu
    name = "schwinger128"
    W, m0, lv = oracle_hierarchy(name)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                     import_tv=[l.V for l in lv[:-1]])
    ref = oracle_deflation(name, W.k_defl)
    d = dm.Deflation(H, len(lv), W.k_defl, import_X=ref.X, import_lambda=ref.lam)
    L = len(lv)
    with pytest.raises(dm.DmlmcError):
        dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [4] * L, 0, prec=dm.MIXED, fixed_counts=True)
    cands = (8, 16, 32)
    best, secs = H.tune_rhs_block(d, cands, prec=dm.MIXED, rtol=W.rtol, noise_seed=W.noise_seed)
    assert best in cands
    assert all(v > 0 for v in secs.values())
    assert secs[best] == min(secs.values())
    kw = dict(prec=dm.MIXED, rtol=W.rtol, fixed_counts=True, max_samples=[40] * L, keep_samples=True)
    r0 = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [20] * L, 0, **kw)
    r1 = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [20] * L, best, **kw)
    assert r0.N == r1.N and all(n % best == 0 for n in r0.N)
    for l in range(L):
        assert np.array_equal(r0.samples[l], r1.samples[l])
    solver = omlmc.DirectSolver(lv)
    for i in (0, 7):
        s, t1, t2 = omlmc.difference_sample(lv, solver, W.noise_seed, 1, i)
        assert abs(r0.samples[0][i] - s) / (abs(t1) + abs(t2)) < 1e-6


def test_recorded_iterations_match_direct_launches(gpu):
    """FGMRES iterations replayed from recorded HIP graphs give bitwise the samples of
    direct launches, over several estimates (record, then replays with eager work and
    host synchronisation in between)."""
    torch, dm, ctx = gpu
    name = "schwinger128"
    W, m0, lv = oracle_hierarchy(name)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                     import_tv=[l.V for l in lv[:-1]])
    ref = oracle_deflation(name, W.k_defl)
    d = dm.Deflation(H, len(lv), W.k_defl, import_X=ref.X, import_lambda=ref.lam)
    L = len(lv)
    kw = dict(prec=dm.MIXED, rtol=W.rtol, fixed_counts=True, max_samples=[32] * L, keep_samples=True)
    assert H.solver_params(use_graphs=0)["use_graphs"] == 0
    direct = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [32] * L, 16, **kw)
    assert H.solver_params(use_graphs=1)["use_graphs"] == 1
    for rep in range(3):
        g = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [32] * L, 16, **kw)
        for l in range(L):
            assert np.array_equal(g.samples[l], direct.samples[l]), (rep, l)
        assert g.trace == direct.trace


def test_smoothing_parameters(gpu):
    """Fine and coarse post-smoothing counts, the reduction target of the complex-FP32
    cycles and the precision of the smoother's coarse blocks are settings; a V-cycle that would leave a level unsmoothed and a target outside
    (0, 1) are rejected, and every setting still solves to tolerance with the same samples
    up to the solve tolerance."""
    torch, dm, ctx = gpu
    name = "schwinger128"
    W, m0, lv = oracle_hierarchy(name)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                     import_tv=[l.V for l in lv[:-1]])
    p0 = H.solver_params()
    assert p0["nu_pre"] == 0 and p0["nu_post"] >= 1 and p0["nu_post_coarse"] >= 1
    with pytest.raises(dm.DmlmcError):
        H.solver_params(nu_pre=0, nu_post_coarse=0)
    with pytest.raises(dm.DmlmcError):
        H.solver_params(nu_pre=0, nu_post=0)
    with pytest.raises(dm.DmlmcError):
        H.solver_params(inner_rtol=1.5)
    with pytest.raises(dm.DmlmcError):
        H.solver_params(smoother_half=2)
    assert H.solver_params() == p0  # a rejected call changes nothing
    assert 0.0 < p0["inner_rtol"] < 1.0
    L = len(lv)
    ref = oracle_deflation(name, W.k_defl)
    d = dm.Deflation(H, L, W.k_defl, import_X=ref.X, import_lambda=ref.lam)
    kw = dict(prec=dm.MIXED, rtol=W.rtol, fixed_counts=True, max_samples=[16] * L, keep_samples=True)
    base = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [16] * L, 16, **kw)
    for fine, coarse, inner, half in ((1, 3, 1e-2, 1), (3, 1, 2e-6, 0), (2, 2, 0.1, 0), (2, 2, 1e-2, 1)):
        q = H.solver_params(nu_post=fine, nu_post_coarse=coarse, inner_rtol=inner, smoother_half=half)
        assert (q["nu_post"], q["nu_post_coarse"], q["inner_rtol"], q["smoother_half"]) == (fine, coarse, inner, half)
        r = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [16] * L, 16, **kw)
        for l in range(L):
            dev = np.max(np.abs(r.samples[l] - base.samples[l]))
            assert dev <= 1e-7 * np.max(np.abs(base.samples[l])), (fine, coarse, inner, half, l, dev)
    H.solver_params(**p0)


def test_kernel_variants_leave_samples_bitwise_identical(gpu, tmp_path):
    """Launch variants (RHS per thread, wavefronts per site, tiles per wavefront) change how
    work is divided, not what is computed: estimates with every variant forced on every
    level, and with the autotuner's picks, give bitwise the samples of the built-in rule;
    the tuner reports a choice for each kernel on each level where it runs and writes
    its cache file, which a second tuning reads back without timing."""
    torch, dm, ctx = gpu
    name = "schwinger128"
    W, m0, lv = oracle_hierarchy(name)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                     import_tv=[l.V for l in lv[:-1]])
    ref = oracle_deflation(name, W.k_defl)
    d = dm.Deflation(H, len(lv), W.k_defl, import_X=ref.X, import_lambda=ref.lam)
    L = len(lv)
    kw = dict(prec=dm.MIXED, rtol=W.rtol, fixed_counts=True, max_samples=[32] * L, keep_samples=True)
    base = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [32] * L, 32, **kw)
    forced = [
        {dm.KV_WILSON_RB: 1, dm.KV_COARSE_SPLIT: 2, dm.KV_SAP_RB: 1, dm.KV_GS_SPLIT: 2, dm.KV_RESTRICT_UT: 1,
         dm.KV_PROLONG_MT: 1},
        {dm.KV_WILSON_RB: 8, dm.KV_COARSE_SPLIT: 1, dm.KV_SAP_RB: 8, dm.KV_GS_SPLIT: 1, dm.KV_RESTRICT_UT: 4,
         dm.KV_PROLONG_MT: 2},
        {dm.KV_WILSON_RB: 2, dm.KV_SAP_RB: 2, dm.KV_RESTRICT_UT: 2, dm.KV_PROLONG_MT: 4, dm.KV_GS_SPLIT: 3},
        {dm.KV_GS_SPLIT: 4, dm.KV_PROLONG_STAGED: 1, dm.KV_RESTRICT_STAGED: 1},
        {dm.KV_PROLONG_STAGED: 2, dm.KV_COARSE_SPLIT: 3, dm.KV_RESTRICT_STAGED: 2},
    ]
    for case in forced:
        for l in range(1, L + 1):
            for k, v in case.items():
                H.set_kernel_variant(l, k, v)
                assert H.kernel_variant(l, k) == v
        print(f"[variants] forced {case}", flush=True)
        r = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [32] * L, 32, **kw)
        for l in range(L):
            assert np.array_equal(r.samples[l], base.samples[l]), (case, l)
    with pytest.raises(dm.DmlmcError):
        H.set_kernel_variant(1, dm.KV_SAP_RB, 3)
    with pytest.raises(dm.DmlmcError):
        H.set_kernel_variant(L + 1, dm.KV_SAP_RB, 1)
    cache = str(tmp_path / "variants.txt")
    picks = H.tune_kernels(32, reps=3, cache_path=cache)
    print(f"[variants] tuned {picks}", flush=True)
    kinds = {k for (_, k) in picks}
    assert {"wilson_rb", "sap_rb", "coarse_split", "gs_split", "restrict_ut", "prolong_mt", "prolong_staged",
            "restrict_staged"} <= kinds
    for (l, k), (v, best, rule) in picks.items():
        assert H.kernel_variant(l, dm.KV_NAMES.index(k)) == v
        assert best > 0 and rule > 0 and best <= rule
    lines = open(cache).read().split("\n")
    assert sum(1 for s in lines if s.strip()) == len(picks)
    r = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [32] * L, 32, **kw)
    for l in range(L):
        assert np.array_equal(r.samples[l], base.samples[l])
    # a second hierarchy of the same shapes takes the cached choices without timing them
    H2 = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                      import_tv=[l.V for l in lv[:-1]])
    again = H2.tune_kernels(32, reps=3, cache_path=cache)
    assert {key: v[0] for key, v in again.items()} == {key: v[0] for key, v in picks.items()}
    assert all(v[1] == 0.0 and v[2] == 0.0 for v in again.values())
