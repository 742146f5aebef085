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
    # the tile stages take the frames with EPF passes; the others are fused
    assert plan.total_tiles == sum(((p.xsize + 63) // 64) * ((p.ysize + 31) // 32) for p in ps
                                   if p.epf_iters > 0)
    assert plan.opt_frames[J.STAGE_FUSED - J.STAGE_PRED] == sum(p.epf_iters == 0 for p in ps)
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
    ctx.batch_stage(plan, J.STAGE_FUSED, 0, 0, 0)
    ctx.batch_stage(plan, J.STAGE_RECON, cfg.grid_recon, cfg.order_recon, 0)
    for k in range(plan.max_epf_iters):
        ctx.batch_stage(plan, J.STAGE_EPF, cfg.grid_epf, cfg.order_epf, k)
    ctx.batch_stage(plan, J.STAGE_SEAM, 0, 0, 0)
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


# Frames with the path's options, alone and together, beside plain ones:
# (w, h, epf_iters, out_format, gab, options).  "field" adds a DcQuantField
# with extra levels (1, 2, 3) under smoothing and AC prediction.
OPT_MIX = [
    (96, 72, 2, 0, 1, {}),
    (130, 97, 1, 1, 1, dict(ac_prediction=1, dc_smoothing=1)),
    (200, 136, 2, 0, 1, dict(qco=1)),
    (96, 72, 3, 2, 1, dict(qco=1)),
    (131, 77, 1, 0, 1, dict(patches=25)),
    (257, 66, 0, 1, 1, dict(noise=1)),
    (192, 136, 1, 0, 1, dict(dots=300, noise=1)),
    (160, 96, 2, 0, 0, dict(splines=6)),
    (136, 80, 2, 0, 1, dict(field=1, ac_prediction=1, dc_smoothing=1, qco=1)),
    (300, 264, 2, 0, 1, dict(ac_prediction=1, qco=1, patches=40, noise=1, dots=200, splines=5)),
    (64, 32, 0, 0, 0, dict(qco=1, patches=3)),
]
# frames whose option stages add with float atomics (order-dependent sums)
ATOMIC = ("patches", "dots", "splines")


def _opt_frames(mix, seed0):
    from paper_1908_03565_amd import jxlr as J
    frames, ps = [], []
    for i, (w, h, e, fmt, g, o) in enumerate(mix):
        seed = seed0 + i
        f = wl.frame(w, h, seed=seed, epf_iters=e, out_format=fmt, gab=g)
        kw = dict(f["params"])
        if o.get("field"):
            kw["extra_levels"] = (1, 2, 3)
            f["dc_quant"] = wl.dc_quant_field(np.random.default_rng(seed), f, (1, 2, 3))
        for k in ("ac_prediction", "dc_smoothing", "qco", "noise"):
            if o.get(k):
                kw[k] = 1
        if o.get("noise"):
            kw["noise_lut"] = np.linspace(0.01, 0.08, 16)
        if o.get("patches"):
            f = wl.with_patches(f, o["patches"], seed)
            kw["num_patches"] = o["patches"]
        if o.get("dots"):
            f = wl.with_dots(f, o["dots"], seed)
            kw["num_dots"] = o["dots"]
            kw["dot_colour_quant"] = (0.004, 0.02, 0.01)
        if o.get("splines"):
            f = wl.with_splines(f, o["splines"], seed)
            kw["num_splines"] = o["splines"]
            kw["num_spline_points"] = len(f["spline_points"])
        p = J.params(w, h, out_format=fmt, **kw)
        assert J.validate_maps_host(p, f) == 0
        frames.append(f)
        ps.append(p)
    return frames, ps


def _agree(got, ref, atomic, msg):
    """Bit-identical, except where float atomics sum in another order: then
    within binary32 rounding of the sums (f32), or one code on a few samples."""
    if not atomic:
        np.testing.assert_array_equal(got, ref, err_msg=msg)
    elif got.dtype == np.float32:
        scale = max(1.0, float(np.abs(ref).max()))
        assert np.abs(got.astype(np.float64) - ref).max() <= 1e-5 * scale, msg
    else:
        d = np.abs(got.astype(np.int64) - ref.astype(np.int64))
        assert d.max() <= 1 and (d > 0).mean() <= 1e-3, msg


def test_batch_with_options_equals_single_frame_decode(ctx):
    import torch
    from paper_1908_03565_amd import jxlr as J
    frames, ps = _opt_frames(OPT_MIX, 1700)
    dfs = [J.DeviceFrame(f) for f in frames]
    ref = _singles(ctx, ps, dfs)
    outs = [ctx.empty_out(p) for p in ps]
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    ws = ctx.batch_workspace(ps)
    plan = ctx.batch_prepare(ps, ios, ws)
    # every option stage has its frames
    names = ["ac_prediction", "qco", "num_patches", "noise", None, "num_dots", "num_splines"]
    for k, nm in enumerate(names):
        if nm is None:  # Gaborish as its own pass: gab with dots or splines
            want = sum(1 for p in ps if p.gab and (p.num_dots or p.num_splines))
        elif nm == "qco":
            want = sum(1 for p in ps if p.qco and p.epf_iters > 0)
        else:
            want = sum(1 for p in ps if getattr(p, nm))
        assert plan.opt_frames[k] == want, (k, nm)
    assert plan.any_noise == 1
    _fill(outs)
    ctx.batch_run(plan)
    torch.cuda.synchronize()
    assert ctx.device_status() == 0
    for i, (o, r) in enumerate(zip(outs, ref)):
        atomic = any(OPT_MIX[i][5].get(k) for k in ATOMIC)
        _agree(o.cpu().numpy(), r, atomic, f"frame {i} {OPT_MIX[i]}")
    # persistent grids for the tile stages change nothing
    _fill(outs)
    ctx.batch_run(plan, J.LaunchConfig(3, 5, 7, 2, 1, 0, 1))
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, ref)):
        atomic = any(OPT_MIX[i][5].get(k) for k in ATOMIC)
        _agree(o.cpu().numpy(), r, atomic, f"grid run, frame {i}")


def test_batch_with_options_graph_replays(ctx):
    import torch
    from paper_1908_03565_amd import jxlr as J
    frames, ps = _opt_frames(OPT_MIX[1:7], 1900)
    dfs = [J.DeviceFrame(f) for f in frames]
    outs = [ctx.empty_out(p) for p in ps]
    ios = [df.io(o) for df, o in zip(dfs, outs)]
    ws = ctx.batch_workspace(ps)
    plan = ctx.batch_prepare(ps, ios, ws)
    ctx.batch_run(plan)
    torch.cuda.synchronize()
    eager = [o.cpu().numpy() for o in outs]
    g = ctx.graph(plan)
    for rep in range(3):
        _fill(outs)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for i, (o, e) in enumerate(zip(outs, eager)):
            atomic = any(OPT_MIX[1 + i][5].get(k) for k in ATOMIC)
            _agree(o.cpu().numpy(), e, atomic, f"replay {rep} frame {i}")
        ctx.decode(ps[0], dfs[0], ctx.empty_out(ps[0]), ctx.workspace(ps[0]))
        torch.cuda.synchronize()
    g.close()
    assert ctx.device_status() == 0
