"""The no-allocation apply (ads_apply_noalloc) against ads_apply, through the
C interface: same kernels, workspace in the library's scratch array."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2201_02250_amd import ads  # noqa: E402

DEV = "cuda:0"


def noalloc_apply(ctx, R):
    """z = M^{-1} R through ads_apply_noalloc (R: n x nrhs device tensor)."""
    L = ads.lib()
    nrhs = 1 if R.dim() == 1 else R.shape[1]
    rr = R if R.dim() == 1 else R.t().contiguous()
    zz = torch.empty_like(rr)
    st = L.ads_apply_noalloc(ctx.ctx, rr.data_ptr(), zz.data_ptr(), nrhs, None)
    torch.cuda.synchronize()
    return st, (zz if R.dim() == 1 else zz.reshape(nrhs, ctx.n).t())


def check(ctx, R, label):
    st, Z = noalloc_apply(ctx, R)
    assert st == ads.ADS_OK, (label, ads.ads_status_string(st), ads.ads_last_error())
    Zr = ctx.apply(R)
    torch.cuda.synchronize()
    Z, Zr = Z.cpu().numpy(), Zr.cpu().numpy()
    err = np.abs(Z - Zr).max() / np.abs(Zr).max()
    print(f"{label}: max rel. difference to ads_apply {err:.1e}", flush=True)
    assert err <= 1e-14, (label, err)


def test_noalloc_apply_matches_apply_twice_smaller_second():
    """Two calls in a row on the two-ended fast path (2D convection-diffusion
    96^2, 3 x 3 blocks, overlap 2, nev 6, eq. 4): four right-hand sides, then
    one (a smaller input); then the one-ended general path with the
    non-restricted eq. 2 (3D, block size beyond the fast path), three and two
    right-hand sides.  Each result equals ads_apply's."""
    rng = np.random.default_rng(31)
    A = W.convdiff2d(96, 0.01)
    ctx = ads.Context(A, W.block_partition_2d(96, 3), 9, 2, 6)
    check(ctx, torch.tensor(rng.standard_normal((A.n, 4)), device=DEV), "fast path, 4 rhs")
    check(ctx, torch.tensor(rng.standard_normal(A.n), device=DEV), "fast path, 1 rhs")
    ctx.close()
    A3 = W.convdiff3d(21, nu=0.02)
    c3 = ads.Context(A3, W.block_partition_3d(21, 3, 3, 3), 27, 2, 6,
                     variant=ads.ADS_VARIANT_ADDITIVE, precision=ads.ADS_PREC_FP32)
    check(c3, torch.tensor(rng.standard_normal((A3.n, 3)), device=DEV), "general path, 3 rhs")
    check(c3, torch.tensor(rng.standard_normal((A3.n, 2)), device=DEV), "general path, 2 rhs")
    c3.close()


def test_noalloc_apply_rejects_workspace_beyond_the_scratch_array():
    """The full-scale 3D workload needs more than the scratch array for 16
    right-hand sides (a clear ADS_ERR_ARG), and fits it for one."""
    A, part, N, o = W.config("c5_jump3d_128_boxes1024")
    Ad = ads.DeviceCSR(A, DEV)
    ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], precision=ads.ADS_PREC_FP32)
    R = torch.tensor(np.random.default_rng(5).standard_normal((A.n, 16)), device=DEV)
    st, _ = noalloc_apply(ctx, R)
    assert st == ads.ADS_ERR_ARG and "beyond the scratch array" in ads.ads_last_error()
    check(ctx, R[:, 0].contiguous(), "3D jumping coefficients, 1 rhs")
    ctx.close()
