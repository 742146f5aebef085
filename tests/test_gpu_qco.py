"""GPU parity of the quantization constraint (J.3).

The isolated pass: the same binary32 reconstruction and filtered frame go to
the HIP pass (through the C-ABI) and to the FP64 oracle's, over frames that
hold every transform type and ragged edges, at two interval multipliers (one
that clamps most coefficients, the default that clamps some).  End to end:
the whole decode with the constraint on against the oracle's, with the
flip-affected pixels of the filter spread over their varblocks (the
constraint mixes a varblock's samples).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03565_amd import workload as wl
from tests import parity as P

pytestmark = pytest.mark.gpu

# binary32 forward and inverse transforms of up to 32 points per axis around
# a clamp: a few tens of ulp of the largest sample of the frame
QCO_TOL = 4e-6


@pytest.fixture(scope="module")
def ctx():
    from paper_1908_03565_amd import jxlr as J
    return J.Context(0)


def _frames():
    types = [t for t in wl.ALL_TYPES if t not in (wl.DCT32X8, wl.DCT8X32)]
    return [("mixed", wl.small(192, 136, seed=61)),
            ("all_types", wl.frame(200, 104, seed=62, choices=types, name="all")),
            ("ragged", wl.frame(131, 77, seed=63, choices=wl.ALL_TYPES[:8] + [12, 13, 14],
                                name="ragged")),
            ("wide", wl.frame(104, 72, seed=64, choices=[wl.DCT32X8, wl.DCT8X32, wl.DCT16X32],
                              name="wide"))]


def _filtered(ctx, p, f):
    """GPU reconstruction and one GPU EPF pass (the constraint's two inputs)."""
    import torch
    from paper_1908_03565_amd import jxlr as J
    df = J.DeviceFrame(f)
    info = ctx.empty_info(p)
    ctx.block_info(p, df, info)
    xyb = ctx.empty_xyb(p)
    ctx.reconstruct(p, df, info, xyb)
    filt = ctx.empty_xyb(p)
    ctx.epf_pass(p, df, info, xyb, filt)
    torch.cuda.synchronize()
    return df, info, xyb, filt


@pytest.mark.parametrize("mul", [0.05, 0.5])
@pytest.mark.parametrize("name,f", _frames(), ids=lambda v: v if isinstance(v, str) else "")
def test_qco_pass_against_oracle(ctx, name, f, mul):
    import torch
    from paper_1908_03565_amd import jxlr as J
    W, H = f["xsize"], f["ysize"]
    kw = dict(f["params"], epf_iters=1, qco=1, qco_interval_mul=mul)
    p = J.params(W, H, **kw)
    assert J.validate_maps_host(p, f) == 0
    df, info, xyb, filt = _filtered(ctx, p, f)
    orig32, filt32 = xyb.cpu().numpy(), filt.cpu().numpy()
    print(f"[qco] {name} {W}x{H} mul {mul}", flush=True)
    ctx.qco_pass(p, df, info, xyb, filt)
    torch.cuda.synchronize()
    got = filt.cpu().numpy().astype(np.float64)
    q = O.params(W, H, **kw)
    ref = O.qco(q, f, orig32.astype(np.float64), filt32.astype(np.float64))
    scale = np.maximum(1.0, np.abs(ref).max(axis=(1, 2)) / 8.0)
    err = np.abs(got - ref).max(axis=(1, 2))
    moved = np.abs(ref - filt32).max()
    print(name, mul, "err", err, "moved", moved)
    assert np.all(err <= QCO_TOL * scale), err
    assert moved > 100 * QCO_TOL  # the constraint is active on these frames
    # the reconstruction is left as it was
    np.testing.assert_array_equal(xyb.cpu().numpy(), orig32)


@pytest.mark.parametrize("name,f", _frames()[1:3], ids=lambda v: v if isinstance(v, str) else "")
def test_qco_small_residual_passes_through(ctx, name, f):
    # a residual far inside every interval comes back as it went in: the
    # forward passes invert the reconstruction's inverse ones for every type
    import torch
    from paper_1908_03565_amd import jxlr as J
    W, H = f["xsize"], f["ysize"]
    p = J.params(W, H, **dict(f["params"], epf_iters=1, qco=1))
    df, info, xyb, _ = _filtered(ctx, p, f)
    noise = torch.from_numpy(
        (np.random.default_rng(5).standard_normal((3, H, W)) * 1e-6).astype(np.float32))
    filt = xyb + noise.to(xyb.device)
    want = filt.cpu().numpy()
    ctx.qco_pass(p, df, info, xyb, filt)
    torch.cuda.synchronize()
    err = np.abs(filt.cpu().numpy() - want).max()
    print(name, "pass-through err", err)
    assert err <= 2e-7 * max(1.0, float(np.abs(want).max()))


@pytest.mark.parametrize("W,H,seed,iters", [(192, 136, 71, 2), (131, 77, 72, 1)])
def test_qco_end_to_end(ctx, W, H, seed, iters):
    from paper_1908_03565_amd import jxlr as J
    f = wl.small(W, H, seed=seed, epf_iters=iters)
    kw = dict(f["params"], qco=1)
    p = J.params(W, H, **kw)
    assert J.validate_maps_host(p, f) == 0
    df = J.DeviceFrame(f)
    gpu = P.gpu_stages(ctx, p, df)
    q = O.params(W, H, **kw)
    orc = O.decode_stages(q, f)
    cmp = P.compare_rgb(p, gpu, orc, f["strategy"])
    print({k: v for k, v in cmp.items() if k != "mask"})
    assert cmp["max_err"] <= P.RGB_TOL
    assert cmp["affected"] <= 0.25 * cmp["pixels"]
    # jxlr_decode runs the same stages (the constraint after the last pass,
    # against the reconstruction kept in its own buffer)
    out = ctx.empty_out(p)
    ctx.decode(p, df, out, ctx.workspace(p))
    np.testing.assert_array_equal(out.cpu().numpy(), gpu["out"])
    # the flag is honoured
    p0 = J.params(W, H, **f["params"])
    out0 = ctx.empty_out(p0)
    ctx.decode(p0, df, out0, ctx.workspace(p0))
    assert np.abs(out0.cpu().numpy() - gpu["out"]).max() > 1e-4

