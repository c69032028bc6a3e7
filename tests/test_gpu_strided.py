"""Strided single operators (GPU).

The solver keeps its internal work vectors at a padded stride between right-hand sides.
Every operator called on RHS blocks padded that way must give bit-identical results to
the unpadded call (the arithmetic is the same, only the addresses move), and must neither
read nor write the padding: NaN planted in the pads of the input does not leak into the
result, and NaN planted in the pads of the output stays where it is.

The padded inputs are made by device-side fills and copies that may still be pending on
torch's stream when the library is called, so this also checks that every library call
is ordered after torch's pending work (the binding waits for it before passing a tensor).
"""
import pytest

from _helpers import oracle_hierarchy

pytestmark = pytest.mark.gpu


def _hier(gpu, name):
    torch, dm, ctx = gpu
    W, m0, lv = oracle_hierarchy(name)
    H = dm.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed,
                     import_tv=[l.V for l in lv[:-1]])
    return W, lv, H


def _padded(torch, x, ld):
    out = torch.full((x.shape[0], ld), complex(float("nan"), float("nan")), dtype=x.dtype, device=x.device)
    out[:, :x.shape[1]] = x
    return out


def test_work_stride_rule(gpu):
    torch, dm, ctx = gpu
    W, lv, H = _hier(gpu, "schwinger128")
    L = len(lv)
    for l in range(1, L + 1):
        n = H.n(l)
        expect = n + 256 if (l < L and n >= 4096) else n
        assert H.work_stride(l) == expect, (l, n)


@pytest.mark.parametrize("nrhs", [19, 32])
def test_strided_operators_match_unpadded(gpu, nrhs):
    torch, dm, ctx = gpu
    W, lv, H = _hier(gpu, "schwinger128")
    L = len(lv)
    gen = torch.Generator().manual_seed(1234 + nrhs)
    for prec, dt in ((dm.FP64, torch.complex128), (dm.MIXED, torch.complex64)):
        for l in range(1, L):
            n, nc = H.n(l), H.n(l + 1)
            ld = H.work_stride(l)
            ldc = nc + 6  # any even stride >= nc is accepted on the coarse side
            x = torch.randn(nrhs, n, dtype=dt, generator=gen).to("cuda:0")
            y0 = torch.randn(nrhs, n, dtype=dt, generator=gen).to("cuda:0")
            xc = torch.randn(nrhs, nc, dtype=dt, generator=gen).to("cuda:0")
            cases = [("D", dm.OP_D, x, ld, n, ld, None, 0),
                     ("G5D", dm.OP_GAMMA5_D, x, ld, n, ld, None, 0),
                     ("R", dm.OP_RESTRICT, x, ld, nc, ldc, None, 0),
                     ("P", dm.OP_PROLONG, xc, ldc, n, ld, None, 0),
                     ("S", dm.OP_SMOOTH, x, ld, n, ld, y0, 2),
                     ("V", dm.OP_VCYCLE, x, ld, n, ld, None, 0)]
            for tag, op, a, lda, nout, ldo, init, arg in cases:
                ref = init.clone() if init is not None else torch.zeros(nrhs, nout, dtype=dt, device="cuda:0")
                H.apply(op, l, a, ref, prec, arg)
                ap = _padded(torch, a, lda)
                outp = _padded(torch, init if init is not None else torch.zeros(nrhs, nout, dtype=dt,
                                                                                  device="cuda:0"), ldo)
                H.apply(op, l, ap, outp, prec, arg, ld_in=lda, ld_out=ldo)
                torch.cuda.synchronize()
                got = outp[:, :nout]
                assert torch.equal(got, ref), (tag, prec, l, int(torch.isnan(got.real).sum()),
                                               int(torch.isnan(ref.real).sum()),
                                               torch.nonzero(torch.isnan(got.real).any(dim=1)).flatten().tolist()[:8],
                                               float((got - ref).abs().nan_to_num(0.0).max()))
                assert bool(torch.isnan(outp[:, nout:].real).all()), (tag, prec, l, "pad written")
                assert bool(torch.isnan(ap[:, a.shape[1]:].real).all()), (tag, prec, l, "input pad written")


def test_strided_apply_rejects_bad_strides(gpu):
    torch, dm, ctx = gpu
    W, lv, H = _hier(gpu, "schwinger128")
    L = len(lv)
    n = H.n(1)
    x = torch.zeros(2, n + 8, dtype=torch.complex64, device="cuda:0")
    y = torch.zeros(2, n + 8, dtype=torch.complex64, device="cuda:0")
    with pytest.raises(dm.DmlmcError):  # odd stride
        H.apply(dm.OP_D, 1, x, y, dm.MIXED, 0, ld_in=n + 7, ld_out=n + 8)
    with pytest.raises(dm.DmlmcError):  # stride below the level size
        H.apply(dm.OP_D, 1, x, y, dm.MIXED, 0, ld_in=n - 2, ld_out=n + 8)
    with pytest.raises(dm.DmlmcError):  # the smoother takes one stride
        H.apply(dm.OP_SMOOTH, 1, x, y, dm.MIXED, 1, ld_in=n + 8, ld_out=n + 2)
    nL = H.n(L)
    xL = torch.zeros(2, nL + 2, dtype=torch.complex64, device="cuda:0")
    yL = torch.zeros(2, nL + 2, dtype=torch.complex64, device="cuda:0")
    with pytest.raises(dm.DmlmcError):  # coarsest-level vectors are unpadded
        H.apply(dm.OP_VCYCLE, L, xL, yL, dm.MIXED, 0, ld_in=nL + 2, ld_out=nL + 2)


def test_strided_vcycle_with_presmoothing(gpu):
    """With pre-smoothing the V-cycle starts its top-level iterate from zero; on padded
    rows that zeroing covers the level's entries only, so the pads still hold their NaN and
    the result equals the unpadded call bit for bit."""
    torch, dm, ctx = gpu
    W, lv, H = _hier(gpu, "schwinger128")
    L = len(lv)
    base = H.solver_params()
    gen = torch.Generator().manual_seed(99)
    try:
        H.solver_params(nu_pre=1)
        for prec, dt in ((dm.FP64, torch.complex128), (dm.MIXED, torch.complex64)):
            for l in range(1, L):
                n, ld = H.n(l), H.work_stride(l)
                x = torch.randn(7, n, dtype=dt, generator=gen).to("cuda:0")
                ref = torch.zeros(7, n, dtype=dt, device="cuda:0")
                H.apply(dm.OP_VCYCLE, l, x, ref, prec)
                ap = _padded(torch, x, ld)
                outp = _padded(torch, torch.zeros(7, n, dtype=dt, device="cuda:0"), ld)
                H.apply(dm.OP_VCYCLE, l, ap, outp, prec, 0, ld_in=ld, ld_out=ld)
                torch.cuda.synchronize()
                assert torch.equal(outp[:, :n], ref), (prec, l)
                assert bool(torch.isnan(outp[:, n:].real).all()), (prec, l, "pad written")
    finally:
        H.solver_params(nu_pre=base["nu_pre"])
