"""The allocation-free deflation projection (dmlmc_deflate_project_noalloc) against the
allocating entry point it mirrors (dmlmc_apply with DMLMC_OP_DEFL_P in complex FP32)
(GPU).  Two calls in a row, the second with fewer RHS, on a level whose size spans many
K-chunks; the outputs must be bitwise equal (same kernels, fixed reduction order) and
within the complex-FP32 bar of the FP64 projection; no device memory is taken by the
call; a size beyond the scratch array is rejected before any device work."""
import numpy as np
import pytest

from paper_2211_15383_amd.inputs import WORKLOADS, load_m0

pytestmark = pytest.mark.gpu

NAME = "schwinger128"


@pytest.fixture(scope="module")
def level2_deflation(gpu):
    torch, dm, ctx = gpu
    W = WORKLOADS[NAME]
    H = dm.Hierarchy(ctx, W.theta(), load_m0(NAME), W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed)
    # level 2 (n = 16384: 64 K-chunks of 256) with k = 24 (ragged against the 16-row tiles)
    D = dm.Deflation(H, 2, 24, eig_rtol=1e-10)
    yield H, D
    D.close()
    H.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_projection_matches_allocating_entry_point(gpu, level2_deflation):
    torch, dm, ctx = gpu
    H, D = level2_deflation
    n = H.n(2)
    g = torch.Generator(device="cuda:0").manual_seed(11)
    for nrhs in (40, 7):
        print(f"[no_alloc] nrhs {nrhs}, n {n}, k {D.k}", flush=True)
        x = torch.randn(nrhs, n, dtype=torch.complex128, device="cuda:0", generator=g)
        ref = torch.empty_like(x)
        H.set_deflation(D)
        try:
            H.apply(dm.OP_DEFL_P, 2, x, ref, dm.MIXED)
            ref64 = torch.empty_like(x)
            H.apply(dm.OP_DEFL_P, 2, x, ref64, dm.FP64)
        finally:
            H.set_deflation(None)
        out = torch.full_like(x, float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        D.project_noalloc(x, out)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] >= free0
        assert torch.equal(out, ref), nrhs
        o, r64 = out.cpu().numpy(), ref64.cpu().numpy()
        for r in range(nrhs):
            assert _rel(o[r], r64[r]) < 1e-5, (nrhs, r)


def test_noalloc_rejects_sizes_beyond_scratch(gpu, level2_deflation):
    torch, dm, ctx = gpu
    H, D = level2_deflation
    n = H.n(2)
    # 16 * k * nrhs * (n / 256 + 1) bytes: 800 RHS at k = 24 need 19.97 MB > 16 MiB
    x = torch.zeros(800, n, dtype=torch.complex128, device="cuda:0")
    out = torch.zeros_like(x)
    with pytest.raises(dm.DmlmcError) as e:
        D.project_noalloc(x, out)
    assert e.value.status == dm.EINVAL
    with pytest.raises(dm.DmlmcError) as e:
        D.project_noalloc(x[:4], x[:4])
    assert e.value.status == dm.EINVAL
