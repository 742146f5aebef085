"""GPU parity of dots (K.2): quantized dots (circles and ellipses, every
angle and sign, some overlapping, some at the frame's edges) dequantized and
added by the HIP kernels after a separate Gaborish pass, against the FP64
oracle; then end to end with the noise after them."""
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


@pytest.mark.parametrize("W,H,seed,n,gab,noise", [(192, 136, 141, 300, 1, 0), (131, 77, 142, 120, 0, 0),
                                                  (300, 264, 143, 500, 1, 1),
                                                  # centres far from the origin, where a
                                                  # binary32 centre would be off by 1e-4 px
                                                  (2056, 96, 144, 2000, 1, 0)])
def test_dots_end_to_end(ctx, W, H, seed, n, gab, noise):
    from paper_1908_03565_amd import jxlr as J
    f = wl.with_dots(wl.small(W, H, seed=seed, epf_iters=1), n, seed)
    kw = dict(f["params"], gab=gab, noise=noise, noise_lut=np.full(16, 0.05),
              dot_colour_quant=(0.004, 0.02, 0.01))
    p = J.params(W, H, num_dots=n, **kw)
    df = J.DeviceFrame(f)
    gpu = P.gpu_stages(ctx, p, df)
    orc = O.decode_stages(O.params(W, H, **kw), f)
    mask, _ = P.affected_mask(p, [(g, s) for _, g, s in gpu["epf"]],
                              [(g, s) for _, g, s in orc["epf"]])
    if gab:
        mask = P.dilate(mask, range(-1, 2), range(-1, 2))
    err = np.abs(gpu["dots"] - orc["dots"])[:, ~mask].max()
    moved = np.abs(orc["dots"] - orc["gab"]).max()
    print("dots xyb err", err, "moved", moved)
    # binary32 exp / sin / cos (a few ulp each) and float sums of up to a few
    # dozen overlapping dots per sample (measured: below 6e-7)
    assert err <= 2e-6 * max(1.0, float(np.abs(orc["dots"]).max()))
    assert moved > 0.01
    cmp = P.compare_rgb(p, gpu, orc)
    print({k: v for k, v in cmp.items() if k != "mask"})
    assert cmp["max_err"] <= P.RGB_TOL
    out = ctx.empty_out(p)
    ctx.decode(p, df, out, ctx.workspace(p))
    # (float atomics: overlapping contributions may sum in another order)
    np.testing.assert_allclose(out.cpu().numpy(), gpu["out"], rtol=2e-6, atol=1e-5)
