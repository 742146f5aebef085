"""The two batch workloads at full size, in the launch configuration the
benchmark times (the tuned schedule, captured in a HIP graph and replayed):

- 64 frames with sides log-uniform in [256, 3072] (89.7 MP), EPF x1, 8-bit
  sRGB out: every frame equals its single-frame decode byte for byte, and
  the three smallest frames are checked against the FP64 oracle (codes equal
  the oracle's rounding of the same linear values; against the all-binary64
  oracle at most one code apart, and equal wherever no EPF decision flipped
  and the value is not within the binary32 error of a code boundary);
- 1024 frames of 256x256, DCT8 only, no EPF, f32 out (67 MP): every frame
  equals the single-frame decode, which matches the oracle within the
  binary32 tolerance.
"""
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


def _run_batch(ctx, frames, cache):
    """Uploads the frames, tunes the schedule, replays the captured graph
    twice into outputs filled with a marker; returns (ps, dfs, outs)."""
    import torch
    from paper_1908_03565_amd import jxlr as J, tuning
    ps, dfs, outs = [], [], []
    for i, fr in enumerate(frames):
        p = J.params(fr["xsize"], fr["ysize"], out_format=fr["out_format"], **fr["params"])
        if i > 0 and fr is frames[0]:
            df = dfs[0].clone()  # a repeated frame still gets its own device memory
        else:
            assert J.validate_maps_host(p, fr) == 0
            df = J.DeviceFrame(fr)
        ps.append(p)
        dfs.append(df)
        outs.append(ctx.empty_out(p))
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    stream = torch.cuda.current_stream()
    plan = ctx.batch_prepare(ps, ios, ctx.batch_workspace(ps))
    cfg, _ = tuning.tuned_config(ctx, plan, stream=stream, path=str(cache))
    for o in outs:
        o.fill_(7 if o.dtype.is_floating_point else 0x5A)
    graph = ctx.graph(plan, cfg)
    graph.launch(stream)
    graph.launch(stream)
    torch.cuda.synchronize()
    assert ctx.device_status() == 0
    return ps, dfs, outs


def _equals_single_frames(ctx, ps, dfs, outs):
    import torch
    for i, (p, df) in enumerate(zip(ps, dfs)):
        o = ctx.empty_out(p)
        ctx.decode(p, df, o, ctx.workspace(p))
        assert torch.equal(o, outs[i]), f"frame {i} differs from its single-frame decode"


def test_batch64_full_size_in_bench_configuration(ctx, tmp_path):
    from paper_1908_03565_amd import jxlr as J
    frames = wl.c4()
    ps, dfs, outs = _run_batch(ctx, frames, tmp_path / "schedules.json")
    assert sum(p.xsize * p.ysize for p in ps) == 89708608
    _equals_single_frames(ctx, ps, dfs, outs)
    for i in sorted(range(len(ps)), key=lambda k: ps[k].xsize * ps[k].ysize)[:3]:
        fr, p = frames[i], ps[i]
        got = outs[i].cpu().numpy()
        p32 = J.params(p.xsize, p.ysize, out_format=0, **fr["params"])
        lin = ctx.empty_out(p32)
        ctx.decode(p32, dfs[i], lin, ctx.workspace(p32))
        np.testing.assert_array_equal(got, O.quantize_srgb(8, lin.cpu().numpy().astype(np.float64)))
        orc = O.decode_stages(O.params(fr["xsize"], fr["ysize"], **fr["params"]), fr)
        gpu = P.gpu_stages(ctx, p, dfs[i])
        np.testing.assert_array_equal(gpu["out"], got)
        eq, firm, maxd = P.srgb_codes_check(p, got, orc, gpu["epf"], 8)
        assert eq == firm and maxd <= 1, (i, eq, firm, maxd)


def test_batch1024_full_size_in_bench_configuration(ctx, tmp_path):
    f = wl.c1()
    frames = [f] * 1024
    ps, dfs, outs = _run_batch(ctx, frames, tmp_path / "schedules.json")
    _equals_single_frames(ctx, ps, dfs, outs)
    orc = O.decode_stages(O.params(f["xsize"], f["ysize"], **f["params"]), f)
    gpu = P.gpu_stages(ctx, ps[0], dfs[0])
    np.testing.assert_array_equal(gpu["out"], outs[0].cpu().numpy())
    cmp = P.compare_rgb(ps[0], gpu, orc)
    assert cmp["affected"] == 0 and cmp["max_err"] <= P.RGB_TOL, cmp
