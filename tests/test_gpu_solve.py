"""Solves, deflation and sample parity against the CPU checker (GPU).

* solve_multi_rhs at every level, FP64 and mixed precision: the residual is recomputed by
  the checker's own sparse matvec and the solution compared with its sparse-LU solve;
* deflation: the device eigensolver against dense eigh (eigenvalues, projector, small
  trace term) and the deflation products (FP64 and FP32 matrix cores) against numpy;
* MLMC samples: every sample value of a fixed-count run against the checker's
  direct-solve sample values for the same noise indices (hierarchy and deflation
  imported, so the comparison isolates the solves), error per sample measured as
  |s_gpu - s_ref| / (|x^H D_l^-1 x| + |y^H D_{l+1}^-1 y|).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import mlmc as omlmc, noise as onoise

from _helpers import oracle_deflation, oracle_hierarchy, random_vectors, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def _gpu_hier(gpu, name):
    torch, dm, ctx = gpu
    W, m0, lv = oracle_hierarchy(name)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                     import_tv=[l.V for l in lv[:-1]])
    return W, lv, H


@pytest.mark.parametrize("name", ["schwinger16", "rect24x16", "schwinger128"])
@pytest.mark.parametrize("prec_name,rtol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_solve_every_level(gpu, name, prec_name, rtol):
    torch, dm, ctx = gpu
    prec = dm.FP64 if prec_name == "fp64" else dm.MIXED
    W, lv, H = _gpu_hier(gpu, name)
    for l in range(1, len(lv) + 1):
        D = lv[l - 1].D
        n = D.shape[0]
        nrhs = 5
        B = np.column_stack([onoise.z2_noise(9, l, i, n) for i in range(nrhs)]).astype(np.complex128)
        X, st = H.solve(l, to_dev(torch, B), prec=prec, rtol=rtol, maxiter=3000)
        Xh = to_host(X)
        res = np.linalg.norm(B - D @ Xh, axis=0) / np.linalg.norm(B, axis=0)
        assert res.max() <= rtol * 1.0001, (l, res.max(), st.iters)
        ref = spla.splu(D.tocsc()).solve(B)
        assert rel_err(Xh, ref) < rtol * 1e4, (l, rel_err(Xh, ref))


@pytest.mark.parametrize("prec_name,rtol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_converged_rhs_leave_the_refinement(gpu, prec_name, rtol):
    """Right-hand sides that reach the tolerance early leave the refinement loop (the
    others move to the front of the block): a zero RHS (converged before any cycle), one
    that is D applied to a smooth vector (few cycles) and noise vectors (more cycles) in
    one block each meet the tolerance, come back in the caller's order, and agree with
    the same RHS solved alone."""
    torch, dm, ctx = gpu
    prec = dm.FP64 if prec_name == "fp64" else dm.MIXED
    W, lv, H = _gpu_hier(gpu, "schwinger128")
    D = lv[0].D
    n = D.shape[0]
    smooth = np.exp(2j * np.pi * np.arange(n) / n)
    B = np.column_stack([onoise.z2_noise(5, 1, 0, n), np.zeros(n), D @ smooth, onoise.z2_noise(5, 1, 1, n),
                         1e-3 * (D @ smooth) + onoise.z2_noise(5, 1, 2, n)]).astype(np.complex128)
    X, st = H.solve(1, to_dev(torch, B), prec=prec, rtol=rtol, maxiter=3000)
    Xh = to_host(X)
    nb = np.linalg.norm(B, axis=0)
    res = np.linalg.norm(B - D @ Xh, axis=0) / np.where(nb > 0, nb, 1.0)
    assert st.converged and res.max() <= rtol * 1.0001, res
    assert np.all(Xh[:, 1] == 0)
    ref = spla.splu(D.tocsc()).solve(B)
    for j in range(B.shape[1]):
        if j == 1:
            continue
        Xj, _ = H.solve(1, to_dev(torch, B[:, j:j + 1]), prec=prec, rtol=rtol, maxiter=3000)
        assert rel_err(to_host(Xj)[:, 0], ref[:, j]) < rtol * 1e4
        assert rel_err(Xh[:, j], ref[:, j]) < rtol * 1e4, j


@pytest.mark.parametrize("name,k", [("schwinger16", 16), ("rect24x16", 6), ("schwinger128", 32)])
def test_eigensolver_against_dense(gpu, name, k):
    torch, dm, ctx = gpu
    W, lv, H = _gpu_hier(gpu, name)
    ref = oracle_deflation(name, k)
    d = dm.Deflation(H, len(lv), k, eig_rtol=1e-12)
    assert d.status == dm.OK, d.info()
    X, lam = d.export()
    assert np.abs(np.abs(lam) - np.abs(ref.lam)).max() < 1e-10
    g5 = lv[-1].gamma5.diagonal().real
    Wg = (g5[None, :] * X).T
    Pi = Wg @ Wg.conj().T
    Pr = ref.W @ ref.W.conj().T
    assert np.abs(Pi - Pr).max() < 1e-8
    assert abs(d.tr_defl - ref.tr_defl) < 1e-9 * abs(ref.tr_defl)


@pytest.mark.parametrize("name,k", [("schwinger16", 16), ("schwinger128", 32)])
def test_deflation_products(gpu, name, k):
    torch, dm, ctx = gpu
    W, lv, H = _gpu_hier(gpu, name)
    ref = oracle_deflation(name, k)
    d = dm.Deflation(H, len(lv), k, import_X=ref.X, import_lambda=ref.lam)
    assert abs(d.tr_defl - ref.tr_defl) < 1e-11 * abs(ref.tr_defl)
    H.set_deflation(d)
    n = ref.W.shape[0]
    for nrhs in (1, 17, 32):
        x = random_vectors(n, nrhs, nrhs)
        C_ref = ref.W.conj().T @ x
        Y_ref = x - ref.W @ C_ref
        xd = to_dev(torch, x)
        for prec, tol in ((dm.FP64, 1e-13), (dm.MIXED, 2e-6)):
            C = torch.empty((nrhs, k), dtype=torch.complex128, device="cuda:0")
            H.apply(dm.OP_DEFL_C, len(lv), xd, C, prec)
            assert rel_err(to_host(C), C_ref) < tol, ("C", prec, nrhs)
            Y = torch.empty_like(xd)
            H.apply(dm.OP_DEFL_P, len(lv), xd, Y, prec)
            assert rel_err(to_host(Y), Y_ref) < tol, ("Y", prec, nrhs)
    H.set_deflation(None)


@pytest.mark.parametrize("name,prec_name,rtol,tol", [("schwinger16", "fp64", 1e-13, 1e-10),
                                                     ("schwinger16", "mixed", 1e-10, 1e-6),
                                                     ("rect24x16", "fp64", 1e-13, 1e-10),
                                                     ("schwinger128", "fp64", 1e-13, 1e-10),
                                                     ("schwinger128", "mixed", 1e-10, 1e-6)])
def test_sample_parity(gpu, name, prec_name, rtol, tol):
    torch, dm, ctx = gpu
    prec = dm.FP64 if prec_name == "fp64" else dm.MIXED
    W, lv, H = _gpu_hier(gpu, name)
    k = W.k_defl
    ref = oracle_deflation(name, k)
    d = dm.Deflation(H, len(lv), k, import_X=ref.X, import_lambda=ref.lam)
    L = len(lv)
    nsamp = 12
    res = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [nsamp] * L, 5, prec=prec, rtol=rtol, fixed_counts=True,
                        max_samples=[nsamp] * L, keep_samples=True)
    assert res.N == [nsamp + (-nsamp) % 5] * L or all(n >= nsamp for n in res.N)
    solver = omlmc.DirectSolver(lv)
    for l in range(1, L + 1):
        got = res.samples[l - 1][:nsamp]
        for i in range(nsamp):
            if l < L:
                s, t1, t2 = omlmc.difference_sample(lv, solver, W.noise_seed, l, i)
                scale = abs(t1) + abs(t2)
            else:
                s = omlmc.coarsest_sample(lv, solver, ref, W.noise_seed, i)
                scale = abs(s)
            assert abs(got[i] - s) / scale < tol, (l, i, got[i], s)


@pytest.mark.parametrize("mode_name,vtol,maxit", [("fp32", 1e-4, 10), ("fp16", 5e-3, 16), ("fp8", 6e-2, 40)])
def test_direct_coarsest_solve(gpu, mode_name, vtol, maxit):
    """Explicit-inverse coarsest solve, applied in complex FP32, FP16 or the 8-bit form: the
    V-cycle of the coarsest level is D_L^-1 to that precision (FP16: 2^-11 rounding of the
    inverse and of the scaled RHS; 8-bit: 2^-4 relative rounding of each entry after its
    row scaling; FP32 accumulation), solves still reach their FP64 tolerance (in a few
    iterations at the coarsest level), and samples match the checker's."""
    torch, dm, ctx = gpu
    mode = {"fp32": dm.DIRECT_FP32, "fp16": dm.DIRECT_FP16, "fp8": dm.DIRECT_FP8}[mode_name]
    name = "schwinger128"
    W, lv, H = _gpu_hier(gpu, name)
    L = len(lv)
    ref = oracle_deflation(name, W.k_defl)
    d = dm.Deflation(H, L, W.k_defl, import_X=ref.X, import_lambda=ref.lam)
    H.coarsest_direct(d, mode)
    D = lv[-1].D
    n = D.shape[0]
    b = random_vectors(n, 5, 77)
    x = torch.empty((5, n), dtype=torch.complex64, device="cuda:0")
    H.apply(dm.OP_VCYCLE, L, to_dev(torch, b, torch.complex64), x, dm.MIXED)
    xs = spla.splu(D.tocsc()).solve(b)
    assert rel_err(to_host(x), xs) < vtol
    X, st = H.solve(L, to_dev(torch, b), prec=dm.MIXED, rtol=1e-10)
    res = np.linalg.norm(b - D @ to_host(X), axis=0) / np.linalg.norm(b, axis=0)
    assert res.max() <= 1e-10 * 1.0001 and st.iters <= maxit, (res.max(), st.iters)
    nsamp = 10
    r = dm.mlmc_trace(H, d, 1e-2, W.noise_seed, [nsamp] * L, 5, prec=dm.MIXED, rtol=1e-10, fixed_counts=True,
                      max_samples=[nsamp] * L, keep_samples=True)
    solver = omlmc.DirectSolver(lv)
    for l in range(1, L + 1):
        for i in range(nsamp):
            if l < L:
                s, t1, t2 = omlmc.difference_sample(lv, solver, W.noise_seed, l, i)
                scale = abs(t1) + abs(t2)
            else:
                s = omlmc.coarsest_sample(lv, solver, ref, W.noise_seed, i)
                scale = abs(s)
            assert abs(r.samples[l - 1][i] - s) / scale < 1e-6, (l, i)
    H.coarsest_direct(enable=False)
    X2, st2 = H.solve(L, to_dev(torch, b), prec=dm.MIXED, rtol=1e-10)
    res2 = np.linalg.norm(b - D @ to_host(X2), axis=0) / np.linalg.norm(b, axis=0)
    assert res2.max() <= 1e-10 * 1.0001


def test_direct_fp16_scaling_and_mode_switch(gpu):
    """FP16 coarsest inverse: each RHS is scaled by its own power of two, so the relative
    accuracy does not depend on its magnitude (1e-30 .. 1e30, where an unscaled FP16 copy
    would flush to zero or overflow), a zero RHS gives zero, and the result is linear
    in the RHS up to the rounding; the 8-bit form likewise, to its precision; switching
    FP32 -> FP16 -> 8-bit -> FP16 reuses the inverses (the FP32 one is built to the
    tightest column tolerance) and the V-cycles follow the current mode (recorded
    iterations are keyed by it)."""
    torch, dm, ctx = gpu
    name = "schwinger128"
    W, lv, H = _gpu_hier(gpu, name)
    L = len(lv)
    ref = oracle_deflation(name, W.k_defl)
    d = dm.Deflation(H, L, W.k_defl, import_X=ref.X, import_lambda=ref.lam)
    D = lv[-1].D
    n = D.shape[0]
    b = random_vectors(n, 4, 78)
    mags = np.array([1e-30, 1.0, 1e30, 0.0])
    bs = b * mags[None, :]
    xs = spla.splu(D.tocsc()).solve(b)
    out = {}
    tol = {dm.DIRECT_FP16: 5e-3, dm.DIRECT_FP32: 1e-4, dm.DIRECT_FP8: 6e-2}
    for mode in (dm.DIRECT_FP32, dm.DIRECT_FP16, dm.DIRECT_FP8, dm.DIRECT_FP16):
        H.coarsest_direct(d, mode)
        x = torch.empty((4, n), dtype=torch.complex64, device="cuda:0")
        H.apply(dm.OP_VCYCLE, L, to_dev(torch, bs, torch.complex64), x, dm.MIXED)
        xh = to_host(x)
        assert np.all(xh[:, 3] == 0)
        errs = [rel_err(xh[:, j] / mags[j], xs[:, j]) for j in range(3)]
        assert max(errs) < tol[mode], (mode, errs)
        out.setdefault(mode, []).append(xh)
        X, st = H.solve(L, to_dev(torch, b), prec=dm.MIXED, rtol=1e-10)
        res = np.linalg.norm(b - D @ to_host(X), axis=0) / np.linalg.norm(b, axis=0)
        assert res.max() <= 1e-10 * 1.0001
    # both FP16 passes ran the same kernels on the same inverse
    assert np.array_equal(out[dm.DIRECT_FP16][0], out[dm.DIRECT_FP16][1])
    assert not np.array_equal(out[dm.DIRECT_FP16][0], out[dm.DIRECT_FP32][0])
    H.coarsest_direct(enable=False)


@pytest.mark.parametrize("scale", [1e-30, 1e30, 2.0 ** -40])
def test_mixed_solve_badly_scaled_rhs(gpu, scale):
    """A right-hand side far from unit size (entries 1e-30, 1e30, 2^-40) is solved to the same
    relative residual as the unit-sized one, and its solution is the scaled solution: the
    complex-FP32 bulk must not underflow or overflow (checked by the checker's matvec)."""
    torch, dm, ctx = gpu
    W, lv, H = _gpu_hier(gpu, "schwinger128")
    for l in (1, 2):
        D = lv[l - 1].D
        n = D.shape[0]
        B = np.column_stack([onoise.z2_noise(21, l, i, n) for i in range(3)]).astype(np.complex128)
        X1, _ = H.solve(l, to_dev(torch, B), prec=dm.MIXED, rtol=1e-10)
        Xs, st = H.solve(l, to_dev(torch, B * scale), prec=dm.MIXED, rtol=1e-10)
        Bs = B * scale
        res = np.linalg.norm(Bs - D @ to_host(Xs), axis=0) / np.linalg.norm(Bs, axis=0)
        assert res.max() <= 1e-10 * 1.0001, (l, scale, res.max())
        assert rel_err(to_host(Xs) / scale, to_host(X1)) < 1e-8, (l, scale)
