"""GPU test of the continuous-batching server: requests of uneven sizes,
EPF pass counts and output formats arrive in a burst under an HBM budget that
holds only part of them; every result must be bit-identical to decoding that
request alone, batches must hold several requests, and the admitted
footprint must never exceed the budget."""
import numpy as np
import pytest

from paper_1908_03565_amd import workload as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1908_03565_amd import jxlr as J
    return J.Context(0)


def _recipes(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W = int(np.clip(round(np.exp(rng.uniform(np.log(64), np.log(512))) / 8) * 8, 64, 512))
        H = int(np.clip(round(np.exp(rng.uniform(np.log(64), np.log(512))) / 8) * 8, 64, 512))
        x0 = 64 * int(rng.integers(0, (1024 - W) // 64 + 1))
        y0 = 64 * int(rng.integers(0, (1024 - H) // 64 + 1))
        # bursts of six simultaneous arrivals, 5 ms apart
        out.append((0.005 * (i // 6), (W, H, x0, y0, int(rng.integers(0, 4)), int(rng.integers(0, 3)))))
    return out


@pytest.mark.parametrize("split", [0, 1])
def test_served_equals_alone(ctx, split):
    import torch
    from paper_1908_03565_amd import jxlr as J
    from paper_1908_03565_amd import serving
    mother = wl.frame(1024, 1024, seed=55, epf_iters=2)
    arrivals = _recipes(24, 7 + split)
    make = lambda q: wl.crop(mother, q[2], q[3], q[0], q[1], epf_iters=q[4], out_format=q[5])
    fps = []
    for _, q in arrivals:
        fr = make(q)
        fps.append(serving.footprint_bytes(J.params(fr["xsize"], fr["ysize"],
                                                    out_format=fr["out_format"], **fr["params"])))
    budget = int(0.35 * sum(fps))
    assert budget >= max(fps)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    srv, wall = serving.run(ctx, arrivals, make, budget, split=split, max_batch=8, keep_every=1)
    assert len(srv.done) == len(arrivals)
    assert srv.peak_used <= budget
    # the accounting matches what the allocator actually handed out (batch
    # headers round per batch, not per request: a few KiB of slack)
    peak = torch.cuda.max_memory_allocated() - base
    print(f"budget {budget}, admitted peak {srv.peak_used}, allocated peak {peak}")
    assert peak <= budget + (64 << 10)
    assert srv.batches > 1 and max(srv.batch_sizes) > 1
    assert ctx.device_status() == 0
    for r in srv.done:
        df = J.DeviceFrame(r.frame)
        o = ctx.empty_out(r.params)
        ctx.decode(r.params, df, o, ctx.workspace(r.params))
        torch.cuda.synchronize()
        assert torch.equal(o.cpu(), r.host_out), f"request {r.rid} {r.params.xsize}x{r.params.ysize}"
    print(serving.summarize(srv, wall))


def test_request_over_budget_is_refused(ctx):
    from paper_1908_03565_amd import serving
    mother = wl.frame(256, 256, seed=56, epf_iters=1)
    make = lambda q: wl.crop(mother, 0, 0, 256, 256, epf_iters=1, out_format=1)
    with pytest.raises(RuntimeError, match="over the budget"):
        serving.run(ctx, [(0.0, None)], make, budget_bytes=1 << 20)


# option sets the served requests take in turn: AC prediction with DC
# smoothing, the quantization constraint, noise, patches (added with float
# atomics: order-dependent sums, compared to rounding), none
_OPTS = [dict(ac_prediction=1, dc_smoothing=1), dict(qco=1), dict(noise=1), dict(patches=12), {}]


def test_served_with_options_equals_alone(ctx):
    import torch
    from paper_1908_03565_amd import jxlr as J
    from paper_1908_03565_amd import serving
    mother = wl.frame(1024, 1024, seed=57, epf_iters=2)
    arrivals = [(t, q + (i % len(_OPTS),)) for i, (t, q) in enumerate(_recipes(20, 9))]

    def make(q):
        fr = wl.crop(mother, q[2], q[3], q[0], q[1], epf_iters=max(q[4], 1), out_format=0)
        o = dict(_OPTS[q[6]])
        kw = dict(fr["params"])
        n = o.pop("patches", 0)
        if n:
            fr = wl.with_patches(fr, n, q[2] + q[3])
            kw["num_patches"] = n
        if o.get("noise"):
            kw["noise_lut"] = np.linspace(0.01, 0.08, 16)
        kw.update(o)
        fr["params"] = kw
        return fr

    fps = []
    for _, q in arrivals:
        fr = make(q)
        fps.append(serving.footprint_bytes(J.params(fr["xsize"], fr["ysize"], out_format=0,
                                                    **fr["params"]), fr))
    budget = int(0.4 * sum(fps))
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    srv, wall = serving.run(ctx, arrivals, make, budget, max_batch=8, keep_every=1)
    assert len(srv.done) == len(arrivals)
    assert srv.peak_used <= budget
    peak = torch.cuda.max_memory_allocated() - base
    print(f"budget {budget}, admitted peak {srv.peak_used}, allocated peak {peak}")
    assert peak <= budget + (64 << 10)
    assert max(srv.batch_sizes) > 1
    assert ctx.device_status() == 0
    for r in srv.done:
        df = J.DeviceFrame(r.frame)
        o = ctx.empty_out(r.params)
        ctx.decode(r.params, df, o, ctx.workspace(r.params))
        torch.cuda.synchronize()
        got, ref = r.host_out.numpy(), o.cpu().numpy()
        msg = f"request {r.rid} {r.params.xsize}x{r.params.ysize}"
        if r.params.num_patches:
            assert np.abs(got.astype(np.float64) - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max()), msg
        else:
            np.testing.assert_array_equal(got, ref, err_msg=msg)
    print(serving.summarize(srv, wall))
