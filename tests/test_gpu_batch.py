"""GPU tests of the batch entry points (persistent stage kernels over the
tiles of many uneven frames) and of the captured HIP graph.

A batch must give, frame by frame, exactly the bytes jxlr_decode gives for
that frame alone (both run the same per-tile code; only the tile schedule
differs), whatever the workgroup counts; graph replays must equal the eager
run.  Two frames of the batch are also checked against the FP64 oracle.
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


# Uneven sizes (ragged tails in both directions, one frame smaller than a
# tile), every EPF iteration count, all three output formats, Gaborish on
# and off.
MIX = [(96, 72, 2, 0, 1), (257, 66, 0, 1, 1), (8, 8, 1, 2, 0), (130, 97, 3, 1, 1),
       (64, 32, 1, 0, 0), (200, 136, 2, 2, 1), (33, 31, 0, 0, 1), (320, 64, 1, 1, 1)]


def _frames(mix, seed0=500):
    return [wl.frame(w, h, seed=seed0 + i, epf_iters=e, out_format=f, gab=g)
            for i, (w, h, e, f, g) in enumerate(mix)]


def _setup(ctx, frames):
    from paper_1908_03565_amd import jxlr as J
    ps, dfs, outs = [], [], []
    for fr in frames:
        p = J.params(fr["xsize"], fr["ysize"], out_format=fr["out_format"], **fr["params"])
        assert J.validate_maps_host(p, fr) == 0
        ps.append(p)
        dfs.append(J.DeviceFrame(fr))
        outs.append(ctx.empty_out(p))
    return ps, dfs, outs


def _singles(ctx, ps, dfs):
    res = []
    for p, df in zip(ps, dfs):
        out = ctx.empty_out(p)
        out.fill_(0)
        ctx.decode(p, df, out, ctx.workspace(p))
        res.append(out.cpu().numpy())
    return res


def _fill(outs):
    for o in outs:
        o.fill_(0x5A if o.dtype.is_floating_point is False else 7.0)


def test_batch_equals_single_frame_decode(ctx):
    import torch
    frames = _frames(MIX)
    ps, dfs, outs = _setup(ctx, frames)
    ref = _singles(ctx, ps, dfs)
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    ws = ctx.batch_workspace(ps)
    _fill(outs)
    ctx.decode_batch(ps, ios, ws)
    torch.cuda.synchronize()
    assert ctx.device_status() == 0
    for i, (o, r) in enumerate(zip(outs, ref)):
        np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg=f"frame {i} {MIX[i]}")


@pytest.mark.parametrize("grids", [(1, 1, 1, 1), (2, 3, 5, 7), (1, 64, 13, 2), (0, 0, 0, 0)])
def test_batch_any_grid(ctx, grids):
    import torch
    from paper_1908_03565_amd import jxlr as J
    frames = _frames(MIX, seed0=700)
    ps, dfs, outs = _setup(ctx, frames)
    ref = _singles(ctx, ps, dfs)
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    ws = ctx.batch_workspace(ps)
    plan = ctx.batch_prepare(ps, ios, ws)
    assert plan.n == len(ps)
    assert plan.total_tiles == sum(((p.xsize + 63) // 64) * ((p.ysize + 31) // 32) for p in ps)
    assert plan.max_epf_iters == 3
    _fill(outs)
    ctx.batch_run(plan, J.LaunchConfig(*grids))
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, ref)):
        np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg=f"frame {i}")


def test_batch_against_oracle(ctx):
    # two frames of a batch, end to end against the FP64 oracle
    import torch
    from paper_1908_03565_amd import jxlr as J
    frames = _frames([(96, 72, 2, 0, 1), (130, 97, 1, 1, 1)], seed0=900)
    ps, dfs, outs = _setup(ctx, frames)
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    ctx.decode_batch(ps, ios, ctx.batch_workspace(ps))
    torch.cuda.synchronize()
    # frame 0: f32 out; the stage-level run gives the flip statistics
    fr, p = frames[0], ps[0]
    q = O.params(fr["xsize"], fr["ysize"], **fr["params"])
    orc = O.decode_stages(q, fr)
    gpu = P.gpu_stages(ctx, p, dfs[0])
    np.testing.assert_array_equal(gpu["out"], outs[0].cpu().numpy())
    cmp = P.compare_rgb(p, gpu, orc)
    assert cmp["max_err"] <= P.RGB_TOL, cmp
    # frame 1: u8 sRGB.  The codes are the oracle's rounding of the linear
    # values the path exports (R27 of the readings: bit-exact); against the
    # all-binary64 oracle they may differ by one code where the value is within
    # the binary32 error of a boundary, and wherever an EPF decision flipped
    fr, p = frames[1], ps[1]
    got = outs[1].cpu().numpy()
    assert got.dtype == np.uint8
    p32 = J.params(fr["xsize"], fr["ysize"], out_format=0, **fr["params"])
    lin = ctx.empty_out(p32)
    ctx.decode(p32, dfs[1], lin, ctx.workspace(p32))
    ref = O.quantize_srgb(8, lin.cpu().numpy().astype(np.float64))
    np.testing.assert_array_equal(got, ref)
    q = O.params(fr["xsize"], fr["ysize"], **fr["params"])
    orc = O.decode_stages(q, fr)
    gpu = P.gpu_stages(ctx, p, dfs[1])
    np.testing.assert_array_equal(gpu["out"], got)
    eq, firm, maxd = P.srgb_codes_check(p, got, orc, gpu["epf"], 8)
    assert eq == firm and maxd <= 1, (eq, firm, maxd)


def test_graph_replays_equal_eager(ctx):
    import torch
    frames = _frames(MIX[:5], seed0=1100)
    ps, dfs, outs = _setup(ctx, frames)
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    ws = ctx.batch_workspace(ps)
    plan = ctx.batch_prepare(ps, ios, ws)
    ctx.batch_run(plan)
    torch.cuda.synchronize()
    eager = [o.cpu().numpy() for o in outs]
    g = ctx.graph(plan)
    for rep in range(4):
        _fill(outs)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for i, (o, e) in enumerate(zip(outs, eager)):
            np.testing.assert_array_equal(o.cpu().numpy(), e, err_msg=f"replay {rep} frame {i}")
        # eager work of the program between replays
        ctx.decode(ps[0], dfs[0], ctx.empty_out(ps[0]), ctx.workspace(ps[0]))
        torch.cuda.synchronize()
    # new input contents in the same buffers: the replay picks them up
    fresh = _frames(MIX[:5], seed0=1300)
    for df, fr in zip(dfs, fresh):
        df.ac.copy_(torch.from_numpy(fr["ac"]).to(df.ac.device))
        df.dc.copy_(torch.from_numpy(fr["dc"]).to(df.dc.device))
    torch.cuda.synchronize()
    g.launch()
    torch.cuda.synchronize()
    ref = _singles(ctx, ps, dfs)
    for i, (o, r) in enumerate(zip(outs, ref)):
        np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg=f"refilled frame {i}")
    g.close()


def test_batch_ill_formed_frame_isolated(ctx):
    # one frame with an overlapping DctSelect map: the device flag is set, that
    # frame's bad region is zero before the filters, and the other frames are
    # unchanged
    import torch
    frames = _frames(MIX[:4], seed0=1500)
    bad = frames[1]
    bad["strategy"] = bad["strategy"].copy()
    bad["strategy"][0, 0] = wl.DCT16
    bad["strategy"][0, 1] = wl.DCT16
    ps, dfs, outs = _setup_unchecked(ctx, frames)
    good = [0, 2, 3]
    ref = _singles(ctx, [ps[i] for i in good], [dfs[i] for i in good])
    assert ctx.device_status() == 0
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    ctx.decode_batch(ps, ios, ctx.batch_workspace(ps))
    torch.cuda.synchronize()
    assert ctx.device_status() != 0
    for k, i in enumerate(good):
        np.testing.assert_array_equal(outs[i].cpu().numpy(), ref[k], err_msg=f"frame {i}")


def _setup_unchecked(ctx, frames):
    from paper_1908_03565_amd import jxlr as J
    ps, dfs, outs = [], [], []
    for fr in frames:
        ps.append(J.params(fr["xsize"], fr["ysize"], out_format=fr["out_format"],
                           **fr["params"]))
        dfs.append(J.DeviceFrame(fr))
        outs.append(ctx.empty_out(ps[-1]))
    return ps, dfs, outs


def test_autotune_and_stages(ctx, tmp_path):
    # the tuned schedule, the cached schedule and a stage-by-stage run all give
    # the single-frame bytes
    import torch
    from paper_1908_03565_amd import jxlr as J
    from paper_1908_03565_amd import tuning
    frames = _frames(MIX, seed0=1700)
    ps, dfs, outs = _setup(ctx, frames)
    ref = _singles(ctx, ps, dfs)
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    ws = ctx.batch_workspace(ps)
    plan = ctx.batch_prepare(ps, ios, ws)
    path = str(tmp_path / "sched.json")
    cfg, info = tuning.tuned_config(ctx, plan, reps=2, path=path)
    assert not info["cached"] and info["tuned_ms"] > 0
    for o, r in zip(outs, ref):  # autotune leaves a full run's outputs
        np.testing.assert_array_equal(o.cpu().numpy(), r)
    cfg2, info2 = tuning.tuned_config(ctx, plan, path=path)
    assert info2["cached"] and cfg2.as_dict() == cfg.as_dict()
    _fill(outs)
    ctx.batch_stage(plan, J.STAGE_INFO, 0, 0, 0)
    ctx.batch_stage(plan, J.STAGE_RECON, cfg.grid_recon, cfg.order_recon, 0)
    for k in range(plan.max_epf_iters):
        ctx.batch_stage(plan, J.STAGE_EPF, cfg.grid_epf, cfg.order_epf, k)
    ctx.batch_stage(plan, J.STAGE_FINISH, cfg.grid_finish, cfg.order_finish, 0)
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, ref)):
        np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg=f"frame {i}")
    with pytest.raises(J.JxlrError):
        ctx.batch_stage(plan, J.STAGE_EPF, 0, 0, plan.max_epf_iters)


@pytest.mark.parametrize("order", [0, 1])
def test_batch_xcd_order(ctx, order):
    import torch
    from paper_1908_03565_amd import jxlr as J
    frames = _frames(MIX, seed0=1900)
    ps, dfs, outs = _setup(ctx, frames)
    ref = _singles(ctx, ps, dfs)
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    plan = ctx.batch_prepare(ps, ios, ctx.batch_workspace(ps))
    for grid in (8, 13, 24, 0):
        _fill(outs)
        ctx.batch_run(plan, J.LaunchConfig(0, grid, grid, grid, order, order, order))
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg=f"grid {grid} frame {i}")
