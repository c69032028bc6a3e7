"""The hierarchy the device builds by itself (no imported test vectors) against the CPU
checker's (GPU).

The device solves D_l V = V with FGMRES to 1e-12 (preconditioned by a provisional
hierarchy) where the checker uses sparse LU, and orthonormalises with classical
Gram-Schmidt twice where the checker uses modified Gram-Schmidt; the interpolators and
coarse operators must still agree to the accuracy the solves allow (1e-7, relative), and
P^H P = I must hold to rounding.
"""
import numpy as np
import pytest

from oracle import multigrid as omg

from _helpers import oracle_hierarchy

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["schwinger16", "rect24x16", "schwinger128"])
def test_device_setup_matches_checker(gpu, name):
    torch, dm, ctx = gpu
    W, m0, lv = oracle_hierarchy(name)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed)
    for l in range(1, len(lv)):
        e = H.export(l, P=True)
        P = e["P"]
        nc = P.shape[1]
        assert np.abs(P.conj().T @ P - np.eye(nc)).max() < 1e-12, ("orthonormal", l)
        err = float(np.abs(P - lv[l - 1].P.toarray()).max())
        assert err < 1e-7, ("P", l, err)
        c = lv[l]
        ref = omg.coarse_blocks(c.D, c.Lx, c.Lt, c.dofs)
        Dc = H.export(l + 1, Dc=True)["Dc"]
        err = float(np.abs(Dc - ref).max() / np.abs(ref).max())
        assert err < 1e-7, ("Dc", l + 1, err)


def test_deflated_coarsest_solve(gpu):
    """With the coarsest deflation attached, the V-cycle's coarsest solve inverts the
    deflation space exactly; solves at the coarsest level still meet rtol."""
    import scipy.sparse.linalg as spla

    from _helpers import oracle_deflation, rel_err, to_dev, to_host
    from oracle import noise as onoise
    torch, dm, ctx = gpu
    W, m0, lv = oracle_hierarchy("schwinger128")
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                     import_tv=[x.V for x in lv[:-1]])
    ref = oracle_deflation("schwinger128", W.k_defl)
    d = dm.Deflation(H, len(lv), W.k_defl, import_X=ref.X, import_lambda=ref.lam)
    H.set_deflation(d)
    try:
        for l in (len(lv), 1):
            D = lv[l - 1].D
            n = D.shape[0]
            B = np.column_stack([onoise.z2_noise(4, l, i, n) for i in range(6)]).astype(np.complex128)
            ref_x = spla.splu(D.tocsc()).solve(B)
            for prec, rtol in ((dm.FP64, 1e-12), (dm.MIXED, 1e-10)):
                X, st = H.solve(l, to_dev(torch, B), prec=prec, rtol=rtol)
                Xh = to_host(X)
                res = np.linalg.norm(B - D @ Xh, axis=0) / np.linalg.norm(B, axis=0)
                assert res.max() <= rtol * 1.0001, (l, prec, res.max())
                assert rel_err(Xh, ref_x) < rtol * 1e4
    finally:
        H.set_deflation(None)
