"""GPU parity of one edge-preserving filter pass (J.2) in isolation: the same
binary32 XYB input goes to the HIP pass and to the FP64 oracle's pass, under
several loop-filter parameter sets, so that both forms of the weight
threshold in the kernel are exercised: the SAD bound (weights that drop
below the minimum do so before the SAD reaches 507) and the clamped form
(a minimum of 0, or large sigmas, keep weights up to the clamp).

The guide bytes and sigmas are compared directly (they may differ where the
binary32 and binary64 evaluations of J.2.2 / J.2.4 straddle an integer);
outside the pixels such a difference can reach, the filtered samples must
agree to binary32 rounding of a 56-term weighted average.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03565_amd import workload as wl
from tests import parity as P

pytestmark = pytest.mark.gpu

# 56 binary32 products and the division: a few ulp of the largest sample.
EPF_TOL = 4e-6


@pytest.fixture(scope="module")
def ctx():
    from paper_1908_03565_amd import jxlr as J
    return J.Context(0)


CASES = {
    "defaults": {},
    "no_minimum": dict(epf_weight_min=0.0),
    "low_minimum_wide_sigma": dict(epf_weight_min=0.05, epf_sigma_max=672),
    "minimum_one": dict(epf_weight_min=1.0),
    "sigma_shift": dict(epf_sigma_shift=3, epf_sigma_max=400, epf_quant_mul=60.0),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("W,H,seed", [(192, 136, 41), (131, 77, 42)])
def test_epf_pass_against_oracle(ctx, case, W, H, seed):
    import torch
    from paper_1908_03565_amd import jxlr as J
    f = wl.small(W, H, seed=seed)
    kw = dict(f["params"])
    kw.update(CASES[case])
    kw["epf_iters"] = 1
    p = J.params(W, H, **kw)
    assert J.validate_maps_host(p, f) == 0
    df = J.DeviceFrame(f)
    info = ctx.empty_info(p)
    ctx.block_info(p, df, info)
    xyb = ctx.empty_xyb(p)
    ctx.reconstruct(p, df, info, xyb)
    out = ctx.empty_xyb(p)
    guide = torch.empty((3, H, W), dtype=torch.uint8, device=xyb.device)
    sigma = torch.empty(((H + 7) // 8, (W + 7) // 8), dtype=torch.int32, device=xyb.device)
    ctx.epf_pass(p, df, info, xyb, out, guide, sigma)
    torch.cuda.synchronize()
    x32 = xyb.cpu().numpy()
    got, gg, gs = out.cpu().numpy(), guide.cpu().numpy(), sigma.cpu().numpy()

    q = O.params(W, H, **kw)
    ref, og, osig = O.epf_pass(q, f, x32.astype(np.float64), want_debug=True)
    mask, stats = P.affected_mask(p, [(gg, gs)], [(og, osig)])
    print(case, stats, "filtered blocks", int((osig >= 16).sum()), "of", osig.size)
    assert stats[0]["guide_flips"] <= 0.01 * W * H and stats[0]["sigma_flips"] <= 2
    scale = max(1.0, float(np.abs(ref).max()) / 8.0)
    err = np.abs(got.astype(np.float64) - ref)[:, ~mask]
    assert err.max() <= EPF_TOL * scale, (case, float(err.max()))
    if case == "defaults":
        assert (osig >= 16).any()  # the filter is active somewhere
