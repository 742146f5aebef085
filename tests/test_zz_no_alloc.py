"""jxlr_decode_noalloc (the entry point for callers that cannot allocate)
against jxlr_decode with a caller-owned workspace: the same stages over the
library's per-device scratch array must give the same output, bit for bit,
on two calls in a row (the second with a smaller frame, so the array holds
the first call's contents), and a frame whose workspace exceeds the array
is refused before any launch."""
import numpy as np
import pytest

from paper_1908_03565_amd import workload as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1908_03565_amd import jxlr as J
    return J.Context(0)


def _both(ctx, f, **over):
    import torch
    from paper_1908_03565_amd import jxlr as J
    kw = dict(f["params"])
    kw.update(over)
    p = J.params(f["xsize"], f["ysize"], out_format=f["out_format"], **kw)
    assert J.validate_maps_host(p, f) == 0
    df = J.DeviceFrame(f)
    ref = ctx.empty_out(p)
    ctx.decode(p, df, ref, ctx.workspace(p))
    out = ctx.empty_out(p)
    out.fill_(0)
    ctx.decode_noalloc(p, df, out)
    torch.cuda.synchronize()
    return J.workspace_bytes(p), ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_matches_decode_on_two_calls_in_a_row(ctx):
    from paper_1908_03565_amd import jxlr as J
    cap = J.lib().jxlr_noalloc_scratch_bytes()
    assert cap == 64 << 20
    # a 1920 x 1080 mixed frame with two EPF passes and AC prediction (the
    # block map, two XYB plane sets and the prediction sums in the array),
    # then a smaller 8-bit frame over the same array
    big = wl.frame(1920, 1080, seed=901, epf_iters=2)
    need, ref, out = _both(ctx, big, ac_prediction=1)
    print("1920x1080 workspace", need, "of", cap)
    assert 0.5 * cap < need <= cap
    np.testing.assert_array_equal(out, ref)
    small = wl.frame(200, 136, seed=902, epf_iters=1, out_format=1)
    need2, ref2, out2 = _both(ctx, small)
    assert need2 < need
    np.testing.assert_array_equal(out2, ref2)
    assert ctx.device_status() == 0


def test_noalloc_refuses_frames_beyond_the_array(ctx):
    from paper_1908_03565_amd import jxlr as J
    f = wl.frame(2048, 2048, seed=903, epf_iters=2)
    p = J.params(2048, 2048, **f["params"])
    assert J.workspace_bytes(p) > J.lib().jxlr_noalloc_scratch_bytes()
    df = J.DeviceFrame(f)
    with pytest.raises(J.JxlrError) as e:
        ctx.decode_noalloc(p, df, ctx.empty_out(p))
    assert e.value.status == 8  # JXLR_E_WORKSPACE
