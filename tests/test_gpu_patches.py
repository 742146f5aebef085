"""GPU parity of patches (K.3): placements of integer patches (up to 16x16,
overlapping, at the frame's edges) added by the HIP kernel to the filtered
XYB frame, against the FP64 oracle; then end to end, and an ill-formed
placement reported through the device flag."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03565_amd import workload as wl
from tests import parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1908_03565_amd import jxlr as J
    return J.Context(0)


@pytest.mark.parametrize("W,H,seed,n,iters", [(192, 136, 121, 40, 2), (131, 77, 122, 25, 1),
                                              (300, 264, 123, 200, 0)])
def test_patches_end_to_end(ctx, W, H, seed, n, iters):
    from paper_1908_03565_amd import jxlr as J
    f = wl.with_patches(wl.small(W, H, seed=seed, epf_iters=iters), n, seed)
    p = J.params(W, H, num_patches=n, **f["params"])
    df = J.DeviceFrame(f)
    gpu = P.gpu_stages(ctx, p, df)
    q = O.params(W, H, **f["params"])
    orc = O.decode_stages(q, f)
    # the patched frame before Gaborish
    mask, _ = P.affected_mask(p, [(g, s) for _, g, s in gpu["epf"]],
                              [(g, s) for _, g, s in orc["epf"]])
    err = np.abs(gpu["patches"] - orc["patches"])[:, ~mask].max()
    scale = max(1.0, float(np.abs(orc["patches"]).max()) / 8.0)
    print("patched xyb err", err, "scale", scale)
    assert err <= 4e-6 * scale
    cmp = P.compare_rgb(p, gpu, orc)
    print({k: v for k, v in cmp.items() if k != "mask"})
    assert cmp["max_err"] <= P.RGB_TOL
    assert ctx.device_status() == 0
    # jxlr_decode adds the same patches (sums of overlaps may round apart)
    out = ctx.empty_out(p)
    ctx.decode(p, df, out, ctx.workspace(p))
    # (float atomics: overlapping contributions may sum in another order)
    np.testing.assert_allclose(out.cpu().numpy(), gpu["out"], rtol=2e-6, atol=1e-5)


def test_ill_formed_patch_sets_the_flag(ctx):
    from paper_1908_03565_amd import jxlr as J
    f = wl.with_patches(wl.small(64, 48, seed=124, epf_iters=0), 3, 124)
    f["patch_place"][1] = [60, 0, 8, 8, 0]  # leaves the frame
    p = J.params(64, 48, num_patches=3, **f["params"])
    df = J.DeviceFrame(f)
    ctx.device_status()  # reads and clears the flag
    xyb = ctx.empty_xyb(p)
    xyb.zero_()
    ctx.patches(p, df, xyb)
    assert ctx.device_status() != 0
    assert ctx.device_status() == 0  # cleared by the read
