"""Checker parity on every level of the full 1024^2 four-level workload, in the launch
configuration the benchmark times: 32 RHS per block, complex-FP32 bulk inside FP64
refinement to 1e-10, k = 128 coarsest deflation, explicit coarsest inverse applied in
complex FP16 (GPU).

The hierarchy's test vectors are each level's Z4 start vectors, computed by the checker
and imported.  They are a pure function of the counter hash, so the device and the
checker build the same P_l and D_{l+1} = P_l^H D_l P_l up to rounding (inverse-iteration
test vectors agree only to the setup solves' tolerance, ~1e-7, which the condition number
of D_{l+1} amplifies in a sample).  The checker's sample values come from
tests/golden/c5_samples.json (tests/golden/make_c5_samples.py: ND-ordered LU on level 1,
FGMRES + V-cycle to 1e-13 on level 2, LU on levels 3-4, dense eigh for the deflation).

Checks:
* P_l (prolongation of unit vectors, restriction of random vectors) and D_{l+1}
  (operator action) against the checker's P_l and P_l^H D_l P_l, every coarsening step;
* the deflation: eigenvalues and tr(D_L^-1 Pi) against dense eigh;
* 32 mixed-precision solves on every level with residuals recomputed by the checker's
  sparse operators;
* sample values of all four levels (mixed: per-sample error <= 1e-6 relative to
  |x^H D_l^-1 x| + |y^H D_{l+1}^-1 y|, coarsest relative to |s|; FP64 at rtol 1e-13:
  <= 1e-10), and the composed estimate of those samples.
"""
import json
import os

import numpy as np
import pytest

from oracle import multigrid as omg, noise as onoise
from paper_2211_15383_amd.inputs import WORKLOADS, load_m0

from _helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NAME = "schwinger1024"
B = 32
FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_samples.json")


@pytest.fixture(scope="module")
def c5(gpu):
    torch, dm, ctx = gpu
    with open(FIXTURE) as f:
        ref = json.load(f)
    W = WORKLOADS[NAME]
    m0 = load_m0(NAME)
    assert abs(ref["m0"] - m0) < 1e-14, "fixture made for another bare mass"
    print("[fullsize-samples] checker hierarchy from Z4 start vectors", flush=True)
    dims = W.level_dims()
    tv = [omg.start_vectors(W.mg_seed, l + 1, N, dims[l][0] * dims[l][1] * dims[l][2])
          for l, N in enumerate(W.ntv)]
    lv = omg.build_hierarchy(W.theta(), m0, W.aggs, W.ntv, 0, W.mg_seed, import_tv=tv)
    print("[fullsize-samples] device hierarchy with the imported vectors", flush=True)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed, import_tv=tv)
    D = dm.Deflation(H, W.nlevels, W.k_defl, eig_rtol=1e-12)
    H.coarsest_direct(D, dm.DIRECT_FP16)
    yield W, ref, lv, H, D
    H.coarsest_direct(None, dm.DIRECT_OFF)
    D.close()
    H.close()


def test_c5_interpolators_and_coarse_operators(gpu, c5):
    torch, dm, ctx = gpu
    W, ref, lv, H, D = c5
    rng = np.random.default_rng(4)
    for l in range(1, W.nlevels):
        P = lv[l - 1].P.tocsc()
        nf, nc = P.shape
        assert (H.n(l), H.n(l + 1)) == (nf, nc)
        cols = np.concatenate([np.arange(16), nc // 2 + np.arange(16), nc - 16 + np.arange(16)])
        E = np.zeros((nc, cols.size), dtype=np.complex128)
        E[cols, np.arange(cols.size)] = 1.0
        out = torch.empty((cols.size, nf), dtype=torch.complex128, device="cuda:0")
        H.apply(dm.OP_PROLONG, l, to_dev(torch, E), out, dm.FP64)
        assert np.abs(to_host(out) - P[:, cols].toarray()).max() < 1e-13, ("P columns", l)
        x = rng.normal(size=(nf, 4)) + 1j * rng.normal(size=(nf, 4))
        y = torch.empty((4, nc), dtype=torch.complex128, device="cuda:0")
        H.apply(dm.OP_RESTRICT, l, to_dev(torch, x), y, dm.FP64)
        assert rel_err(to_host(y), P.conj().T @ x) < 1e-13, ("P^H", l)
        xc = rng.normal(size=(nc, 4)) + 1j * rng.normal(size=(nc, 4))
        yc = torch.empty((4, nc), dtype=torch.complex128, device="cuda:0")
        H.apply(dm.OP_D, l + 1, to_dev(torch, xc), yc, dm.FP64)
        assert rel_err(to_host(yc), lv[l].D @ xc) < 1e-13, ("D_c", l + 1)


def test_c5_deflation_against_dense_eigh(gpu, c5):
    torch, dm, ctx = gpu
    W, ref, lv, H, D = c5
    X, lam = D.export()
    lam_ref = np.array(ref["lambda"])
    assert np.abs(lam - lam_ref).max() < 1e-10 * np.abs(lam_ref).max()
    assert abs(D.tr_defl - ref["tr_defl"]) < 1e-9 * abs(ref["tr_defl"])


def test_c5_solves_on_every_level_by_checker_matvec(gpu, c5):
    torch, dm, ctx = gpu
    W, ref, lv, H, D = c5
    H.set_deflation(D)
    try:
        for l in range(1, W.nlevels + 1):
            n = lv[l - 1].n
            print(f"[fullsize-samples] 32 mixed solves on level {l}", flush=True)
            Bm = np.column_stack([onoise.z2_noise(W.noise_seed, l, i, n) for i in range(B)]).astype(np.complex128)
            X, st = H.solve(l, to_dev(torch, Bm), prec=dm.MIXED, rtol=W.rtol, maxiter=4000)
            res = np.linalg.norm(Bm - lv[l - 1].D @ to_host(X), axis=0) / np.linalg.norm(Bm, axis=0)
            assert res.max() <= W.rtol * 1.0001, (l, res.max())
            del X
    finally:
        H.set_deflation(None)


def _check_samples(ref, samples, L, bar, ids=None):
    worst = 0.0
    for l in range(1, L + 1):
        for row in ref["levels"][str(l)]["samples"]:
            i = row["i"]
            if ids is not None and i not in ids:
                continue
            s_ref = complex(*row["s"])
            den = abs(complex(*row["t1"])) + abs(complex(*row["t2"])) if l < L else abs(s_ref)
            err = abs(samples[l - 1][i] - s_ref) / den
            worst = max(worst, err)
            assert err <= bar, (l, i, err)
    return worst


def test_c5_mixed_samples_all_levels(gpu, c5):
    torch, dm, ctx = gpu
    W, ref, lv, H, D = c5
    L = W.nlevels
    print("[fullsize-samples] mixed estimate, 32 samples per level", flush=True)
    r = dm.mlmc_trace(H, D, W.eps, W.noise_seed, [B] * L, B, prec=dm.MIXED, rtol=W.rtol, fixed_counts=True,
                      max_samples=[B] * L, keep_samples=True, maxiter=4000)
    worst = _check_samples(ref, r.samples, L, 1e-6)
    print(f"[fullsize-samples] mixed worst per-sample error {worst:.2e}, iterations {r.iters}", flush=True)
    # the estimate is Re sum of level means + tr(D_L^-1 Pi)
    T = sum(np.mean(s) for s in r.samples).real + r.tr_defl
    assert abs(T - r.trace) <= 1e-12 * abs(T)


def test_c5_fp64_samples_all_levels(gpu, c5):
    torch, dm, ctx = gpu
    W, ref, lv, H, D = c5
    L = W.nlevels
    ids = (0, 1, 2, 3)
    print("[fullsize-samples] FP64 estimate, 4 samples per level at rtol 1e-13", flush=True)
    r = dm.mlmc_trace(H, D, W.eps, W.noise_seed, [4] * L, 4, prec=dm.FP64, rtol=1e-13, fixed_counts=True,
                      max_samples=[4] * L, keep_samples=True, maxiter=6000)
    worst = _check_samples(ref, r.samples, L, 1e-10, ids)
    print(f"[fullsize-samples] FP64 worst per-sample error {worst:.2e}, iterations {r.iters}", flush=True)
