"""GPU parity with dequantization matrices of every C.6.1 encoding mode and
with a C.5.2 DcQuantField at extra_levels 1-3.

Encodings: the context is created with fifteen encodings (jxlr_create), the
oracle decodes with the same ones; frames mix transform types inside their
32x32 regions.  Gates as for the default matrices: XYB within the relative
bound of the plain parity tests, [0,1]-scaled linear RGB within 1e-4 outside
EPF flip-affected pixels (frames whose samples stay in range).

DcQuantField: the DC is dequantized with the multiplier over 2^extra_levels,
F.2 smoothing and the J.3 DC clamp read each sample's field value, Annex H's
window the multiplier itself.  The smoothing test |wa - s| <= 0.5 dcq is a
decision taken in binary32 on the GPU; the frames here keep every one of
them at least 1e-3 dcq from its boundary (checked on the inputs).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03565_amd import workload as wl
from tests import parity as P

pytestmark = pytest.mark.gpu

XYB_TOL = 4e-6
MIX13 = [t for t in wl.ALL_TYPES if t not in (wl.DCT32X8, wl.DCT8X32)]


def _ctx(encs):
    from paper_1908_03565_amd import jxlr as J
    return J.Context(0, dq_enc=encs)


def _xyb_ok(gpu, ref):
    scale = np.maximum(1.0, np.abs(ref).max(axis=(1, 2)) / 8.0)
    err = np.abs(gpu - ref).max(axis=(1, 2))
    return bool(np.all(err <= XYB_TOL * scale)), err


def _mode_encodings(mode, seed):
    """Encodings that use `mode` wherever it is valid (Library elsewhere).
    Copy: DCT8 gets a random DCT-mode encoding and Identity a random
    Identity-mode one; DCT2 and AFV (numerators 1, like Identity's) copy
    Identity's, every other type copies DCT8's (a copy of a copy for DCT16)."""
    rng = np.random.default_rng(seed)
    encs = [{"mode": 0} for _ in range(15)]
    if mode == wl.DQ_COPY:
        encs[0] = wl.dequant_encoding(rng, 0, wl.DQ_DCT)
        encs[1] = wl.dequant_encoding(rng, 1, wl.DQ_IDENTITY)
        for s in range(2, 15):
            encs[s] = {"mode": wl.DQ_COPY, "copy_from": 1 if s in (2, 14) else 0}
        encs[4] = {"mode": wl.DQ_COPY, "copy_from": 3}
        return encs
    for s in range(15):
        if mode in (wl.DQ_LIBRARY, wl.DQ_DCT) or wl.BLOCKS[s] == (1, 1):
            encs[s] = wl.dequant_encoding(rng, s, mode)
    return encs


def _run(ctx, f, encs, **over):
    from paper_1908_03565_amd import jxlr as J
    kw = dict(f["params"])
    kw.update(over)
    p = J.params(f["xsize"], f["ysize"], out_format=f["out_format"], **kw)
    assert J.validate_maps_host(p, f) == 0
    gpu = P.gpu_stages(ctx, p, J.DeviceFrame(f))
    kw.pop("idct_split", None)  # the library's transform arithmetic only
    q = O.params(f["xsize"], f["ysize"], dq_enc=encs, **kw)
    return p, q, gpu, O.decode_stages(q, f)


@pytest.mark.parametrize("mode", list(range(8)))
def test_encoding_mode_end_to_end(mode):
    encs = _mode_encodings(mode, 500 + mode)
    ctx = _ctx(encs)
    f = wl.frame(264, 200, seed=510 + mode, choices=MIX13, tiling="mixed", epf_iters=1)
    p, q, gpu, orc = _run(ctx, f, encs)
    ok, err = _xyb_ok(gpu["recon"], orc["recon"])
    # the matrices differ from the defaults wherever the mode was used
    if mode != wl.DQ_LIBRARY:
        assert np.abs(O.reconstruct(O.params(264, 200, **f["params"]), f) - orc["recon"]).max() > 1e-4
    cmp = P.compare_rgb(p, gpu, orc)
    print(f"mode {mode}: XYB err {err}; RGB {({k: v for k, v in cmp.items() if k != 'mask'})}")
    assert ok, err
    if cmp["max_abs_ref"] <= 64.0:
        assert cmp["max_err"] <= P.RGB_TOL


# seeds whose random encodings use six to eight of the modes and keep this
# recipe's samples in range (picked by running the oracle on the CPU)
@pytest.mark.parametrize("seed,split", [(624, 0), (658, 0), (613, 1), (655, 1)])
def test_random_encodings_all_modes(seed, split):
    encs = wl.dequant_encodings(seed)
    ctx = _ctx(encs)
    f = wl.frame(521, 267, seed=seed, choices=MIX13, tiling="mixed", epf_iters=2)
    p, q, gpu, orc = _run(ctx, f, encs, idct_split=split)
    ok, err = _xyb_ok(gpu["recon"], orc["recon"])
    cmp = P.compare_rgb(p, gpu, orc)
    print(f"seed {seed} split {split}: modes {[e['mode'] for e in encs]} XYB err {err}; "
          f"RGB {({k: v for k, v in cmp.items() if k != 'mask'})}")
    if split == 0:
        assert ok, err
    assert cmp["max_abs_ref"] <= 64.0
    assert cmp["max_err"] <= (P.RGB_TOL if split == 0 else 1e-3)
    assert cmp["affected"] <= 0.05 * cmp["pixels"]


def test_encodings_with_the_quantization_constraint():
    # J.3 clamps to the encoded matrices' steps
    encs = wl.dequant_encodings(608)
    ctx = _ctx(encs)
    f = wl.frame(192, 136, seed=608, choices=MIX13, tiling="mixed", epf_iters=2)
    p, q, gpu, orc = _run(ctx, f, encs, qco=1)
    cmp = P.compare_rgb(p, gpu, orc, f["strategy"])
    print({k: v for k, v in cmp.items() if k != "mask"})
    assert cmp["max_err"] <= P.RGB_TOL
    assert cmp["affected"] <= 0.25 * cmp["pixels"]


def _field_frame(W, H, seed, el, epf_iters=2):
    """The c2 recipe with small-integer DC (a few dcq apart, so both outcomes
    of the smoothing window occur) and a random DcQuantField."""
    f = wl.frame(W, H, seed=seed, choices=MIX13, tiling="mixed", epf_iters=epf_iters)
    rng = np.random.default_rng(seed)
    Hb, Wb = (H + 7) // 8, (W + 7) // 8
    scale = np.array([2 ** e for e in el])[:, None, None]
    f["dc"] = ((rng.integers(-2, 3, size=(3, Hb, Wb)) * rng.integers(0, 2, size=(3, Hb, Wb))
                + rng.integers(-8, 9, size=(3, 1, 1))) * scale).astype(np.int32)
    f["params"] = dict(f["params"], extra_levels=tuple(el))
    f["dc_quant"] = wl.dc_quant_field(rng, f, el)
    return f


def _smoothing_margin(f, el):
    # |wa - s| - 0.5 dcq in units of the sample's dcq, from the integers
    wc, we, wd = 0.05226273532324128, 0.20345139757231578, 0.0334829185968739
    d = f["dc"].astype(np.float64) / np.array([2.0 ** e for e in el])[:, None, None]
    n = d[:, 1:-1, 1:-1]
    e = d[:, :-2, 1:-1] + d[:, 2:, 1:-1] + d[:, 1:-1, :-2] + d[:, 1:-1, 2:]
    g = d[:, :-2, :-2] + d[:, :-2, 2:] + d[:, 2:, :-2] + d[:, 2:, 2:]
    dev = np.abs(we * e + wd * g - (1 - wc) * n)       # in units of dc_mul
    rel = f["dc_quant"][:, 1:-1, 1:-1] / np.array(f["params"]["dc_mul"])[:, None, None]
    return np.abs(dev / rel - 0.5)


@pytest.mark.parametrize("el", [(1, 2, 1), (3, 3, 3), (0, 1, 2)])
def test_extra_levels_and_field_with_smoothing(el):
    from paper_1908_03565_amd import jxlr as J
    ctx = J.Context(0)
    f = _field_frame(264, 200, 700 + sum(el), el)
    assert _smoothing_margin(f, el).min() > 1e-3
    p, q, gpu, orc = _run(ctx, f, None, dc_smoothing=1)
    ok, err = _xyb_ok(gpu["recon"], orc["recon"])
    print(f"el {el}: XYB err {err}")
    assert ok, err
    cmp = P.compare_rgb(p, gpu, orc)
    assert cmp["max_err"] <= P.RGB_TOL
    # the field is read: the same frame without it (every sample the
    # multiplier over 2^extra_levels) smooths differently
    g = dict(f)
    del g["dc_quant"]
    orc2 = O.reconstruct(O.params(264, 200, **dict(f["params"], dc_smoothing=1)), g)
    if max(el) > 0:
        assert np.abs(orc2 - orc["recon"]).max() > 1e-6


@pytest.mark.parametrize("el", [(1, 2, 1), (2, 3, 2)])
def test_field_with_constraint_and_ac_prediction_end_to_end(el):
    from paper_1908_03565_amd import jxlr as J
    ctx = J.Context(0)
    f = _field_frame(300, 264, 720 + sum(el), el)
    assert _smoothing_margin(f, el).min() > 1e-3
    kw = dict(dc_smoothing=1, ac_prediction=1, qco=1)
    p, q, gpu, orc = _run(ctx, f, None, **kw)
    start, near = P.acpred_mask(q, f)
    cmp = P.compare_rgb(p, gpu, orc, f["strategy"], start)
    print(f"el {el}: near cells {near}; {({k: v for k, v in cmp.items() if k != 'mask'})}")
    assert cmp["max_err"] <= P.RGB_TOL
    assert cmp["affected"] <= 0.25 * cmp["pixels"]
    # jxlr_decode with the field gives the stage-by-stage result
    df = J.DeviceFrame(f)
    out = ctx.empty_out(p)
    ctx.decode(p, df, out, ctx.workspace(p))
    np.testing.assert_array_equal(out.cpu().numpy(), gpu["out"])


def test_field_planes_all_or_none():
    from paper_1908_03565_amd import jxlr as J
    ctx = J.Context(0)
    f = _field_frame(64, 64, 730, (1, 1, 1))
    p = J.params(64, 64, **dict(f["params"], dc_smoothing=1))
    df = J.DeviceFrame(f)
    io = df.io(ctx.empty_out(p))
    io.dc_quant[1] = None
    with pytest.raises(J.JxlrError):
        ctx.decode(p, df, ctx.empty_out(p), ctx.workspace(p), io=io)
