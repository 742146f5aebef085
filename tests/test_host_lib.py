"""CPU tests of the C-ABI library: exports, defaults, host validation, and the
library's host-built tables against the oracle's (both written independently
from the draft).  No GPU is touched."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03565_amd import jxlr as J
from paper_1908_03565_amd import workload as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "jxlr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(jxlr_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_header_function():
    names = _header_functions()
    assert len(names) >= 11
    lib = J.lib()
    for n in names:
        assert hasattr(lib, n), n
        assert n in J.exported_symbols(), n


def test_status_strings():
    for s in range(11):
        assert J.lib().jxlr_status_string(s)


def test_defaults_agree_with_oracle():
    p = J.params(64, 48)
    q = O.params(64, 48)
    for name, _ in J.FrameParams._fields_:
        # output format and transform arithmetic are the library's own; the
        # patch and dot counts travel with their arrays on the oracle's side
        if name in ("out_format", "idct_split", "num_patches", "num_dots", "num_splines",
                    "num_spline_points", "fuse"):
            continue
        a, b = getattr(p, name), getattr(q, name)
        if isinstance(a, C.Array):
            np.testing.assert_allclose(list(a), list(b), rtol=1e-7, err_msg=name)
        else:
            assert a == pytest.approx(b, rel=1e-7), name


def _frame(W=64, H=64, s=0):
    Wb, Hb = (W + 7) // 8, (H + 7) // 8
    return dict(strategy=np.full((Hb, Wb), s, np.uint8), qf=np.zeros((Hb, Wb), np.uint8),
                sharpness=np.zeros((Hb, Wb), np.uint8))


def test_validate_maps_host():
    p = J.params(64, 64)
    assert J.validate_maps_host(p, _frame()) == 0
    f = _frame(); f["strategy"][0, 1] = 4
    assert J.validate_maps_host(p, f) == 4  # misaligned
    f = _frame(); f["strategy"][0, 1] = 7; f["strategy"][1, 0] = 6
    assert J.validate_maps_host(p, f) == 4  # DCT16x8 at block (0,1) overlaps DCT8x16 at (1,0)
    p24 = J.params(24, 24)
    f = _frame(24, 24); f["strategy"][2, 2] = 4
    assert J.validate_maps_host(p24, f) == 4  # out of bounds
    for bad in (15, 16, 200):
        f = _frame(); f["strategy"][3, 3] = bad
        assert J.validate_maps_host(p, f) == 3
    f = _frame(s=4); f["qf"][1, 1] = 5
    assert J.validate_maps_host(p, f) == 5  # quant field not uniform in a varblock
    f = _frame(); f["sharpness"][2, 2] = 8
    assert J.validate_maps_host(p, f) == 7
    for fr in (wl.small(), wl.small(83, 45, seed=3), wl.c1()):
        assert J.validate_maps_host(J.params(fr["xsize"], fr["ysize"]), fr) == 0


def test_parameter_ranges():
    f = _frame()
    for k, v in [("epf_weight_min", 1.5), ("epf_sigma_max", 700), ("epf_sigma_shift", 9),
                 ("idct_split", 2), ("idct_split", -1), ("dc_smoothing", 2),
                 ("epf_iters", 4), ("global_scale", 0), ("target_nits_div50", 0),
                 ("out_format", 3)]:
        p = J.params(64, 64, **{k: v})
        assert J.validate_maps_host(p, f) == 7, k
        assert J.workspace_bytes(p) == 0
    assert J.validate_maps_host(J.params(0, 8), _frame(8, 8)) == 2
    # extra_levels 0..3, with smoothing, the constraint and AC prediction too
    for el in ((0, 1, 0), (1, 2, 1), (3, 3, 3)):
        for kw in (dict(dc_smoothing=1), dict(qco=1), dict(ac_prediction=1), {}):
            assert J.validate_maps_host(J.params(64, 64, extra_levels=el, **kw), f) == 0, (el, kw)
    for el in ((0, 4, 0), (-1, 0, 0)):
        assert J.validate_maps_host(J.params(64, 64, extra_levels=el), f) == 7
    # the quantization constraint: a flag and a finite non-negative multiplier
    for kw in (dict(qco=2), dict(qco=-1), dict(qco=1, qco_interval_mul=-0.25),
               dict(qco=1, qco_interval_mul=float("nan")), dict(qco=1, qco_interval_mul=float("inf"))):
        p = J.params(64, 64, **kw)
        assert J.validate_maps_host(p, f) == 7, kw
        assert J.workspace_bytes(p) == 0, kw
    assert J.validate_maps_host(J.params(64, 64, qco=1, qco_interval_mul=0.0), f) == 0
    assert J.validate_maps_host(J.params(64, 64, ac_prediction=2), f) == 7
    assert J.params(64, 64).ac_prediction == 0
    # every real-valued field must be finite (the oracle rejects the same)
    nan, inf = float("nan"), float("inf")
    for kw in (dict(epf_scale=(1.0, nan, 1.0)), dict(epf_range_max=inf), dict(epf_range_mul=nan),
               dict(epf_quant_mul=-inf), dict(dc_mul=(1.0, 1.0, nan)), dict(kx_dc=nan),
               dict(gab_w1=(0.1, inf, 0.1)), dict(opsin_inv=[1.0] * 8 + [nan]),
               dict(opsin_bias=(0.0, nan, 0.0)), dict(epf_sharp_lut=[0.0] * 7 + [inf]),
               dict(epf_weight_min=nan)):
        p = J.params(64, 64, **kw)
        assert J.validate_maps_host(p, f) == 7, kw
        q = O.params(64, 64, **kw)
        with pytest.raises(O.OracleError):
            O.reconstruct(q, dict(wl.small(64, 64, seed=1), params={}))
    # noise: a flag and a finite LUT
    lut = np.zeros(16)
    lut[3] = float("nan")
    for kw in (dict(noise=2), dict(noise=1, noise_lut=lut)):
        p = J.params(64, 64, **kw)
        assert J.validate_maps_host(p, f) == 7
        assert J.workspace_bytes(p) == 0
    assert J.params(64, 64).noise == 0
    for kw in (dict(num_patches=-1), dict(num_dots=-2), dict(dot_colour_quant=(0, float("inf"), 0)),
               dict(num_splines=-1), dict(num_splines=3, num_spline_points=2),
               dict(num_spline_points=(1 << 22) + 1), dict(num_spline_points=-1)):
        p = J.params(64, 64, **kw)
        assert J.validate_maps_host(p, f) == 7 and J.workspace_bytes(p) == 0, kw
    d = J.params(64, 64)
    assert d.qco == 0 and d.qco_interval_mul == 0.5  # C.10 defaults


def test_workspace_bytes():
    # block-info map (13 x 7 blocks, one 256-byte unit) plus, with EPF passes,
    # two XYB plane sets; with none, the reconstruction is fused with the
    # finish and only the seam records of the 2 x 2 tiles of 64 x 32 are kept
    # (rows 0, 1, h - 2, h - 1 of 3 x 64 samples and columns 0, 1, w - 2,
    # w - 1 of 3 x 32, binary32)
    p = J.params(100, 50, epf_iters=0)
    fused = J.workspace_bytes(p)
    seam = J.lib().jxlr_seam_bytes(C.byref(p))
    assert seam == 4 * (4 * 3 * 64 + 4 * 3 * 32) * 4
    assert fused == 256 + seam
    # with EPF passes: two XYB plane sets, plus the seam records when the
    # finish is fused into the last pass (nothing between the two)
    p1 = J.params(100, 50, epf_iters=1)
    xyb = (3 * 100 * 50 * 4 + 255) // 256 * 256
    assert J.workspace_bytes(p1) == 256 + 2 * xyb + seam
    assert J.lib().jxlr_seam_bytes(C.byref(p1)) == seam
    p2 = J.params(100, 50, epf_iters=2)
    assert J.workspace_bytes(p2) == J.workspace_bytes(p1) and J.workspace_bytes(p2) % 256 == 0
    # the quantization constraint keeps the reconstruction past a second
    # pass: one more plane set then, none with a single pass or none at all;
    # and the finish stays apart (no seam records)
    assert J.workspace_bytes(J.params(100, 50, epf_iters=2, qco=1)) == 256 + 3 * xyb
    assert J.workspace_bytes(J.params(100, 50, epf_iters=1, qco=1)) == 256 + 2 * xyb
    assert J.workspace_bytes(J.params(100, 50, epf_iters=0, qco=1)) == fused
    # noise adds the pseudorandom channels, one plane set (and keeps the
    # finish apart: one reconstruction plane set without EPF passes)
    assert J.workspace_bytes(J.params(100, 50, epf_iters=2, noise=1)) == 256 + 3 * xyb
    assert J.workspace_bytes(J.params(100, 50, epf_iters=0, noise=1)) == 256 + 2 * xyb
    assert J.workspace_bytes(J.params(100, 50, epf_iters=2, fuse=-1)) == 256 + 2 * xyb
    # fuse = -1 keeps the reconstruction and the finish apart: one plane set
    assert J.workspace_bytes(J.params(100, 50, epf_iters=0, fuse=-1)) == 256 + xyb
    for bad in (-2, 5):
        assert J.workspace_bytes(J.params(100, 50, fuse=bad)) == 0
    one = fused
    # AC prediction adds its sums, 3 x 4 floats per block (13 x 7 blocks)
    extra = J.workspace_bytes(J.params(100, 50, epf_iters=0, ac_prediction=1)) - one
    assert 12 * 4 * 13 * 7 <= extra < 12 * 4 * 13 * 7 + 256
    # dots or splines: Gaborish into a plane set of its own; splines add
    # their curve samples (3 doubles, 16 per control point)
    # (frames with dots or splines keep the finish apart: the base is the
    # unfused layout)
    gp = J.params(100, 50, epf_iters=2, gab=1, fuse=-1)
    base = J.workspace_bytes(gp)
    assert J.workspace_bytes(J.params(100, 50, epf_iters=2, gab=1, num_dots=5)) - base == xyb
    sp = J.params(100, 50, epf_iters=2, gab=1, num_splines=3, num_spline_points=40)
    sb = J.lib().jxlr_spline_scratch_bytes(C.byref(sp))
    assert 3 * 16 * 8 * 40 <= sb < 3 * 16 * 8 * 40 + 256 and sb % 256 == 0
    assert J.workspace_bytes(sp) - base == xyb + sb
    sp0 = J.params(100, 50, epf_iters=2, gab=0, num_splines=3, num_spline_points=40)
    assert J.workspace_bytes(sp0) - J.workspace_bytes(J.params(100, 50, epf_iters=2, gab=0,
                                                               fuse=-1)) == sb
    assert J.lib().jxlr_spline_scratch_bytes(C.byref(gp)) == 0


def test_batch_workspace_bytes():
    # header (descriptors and two prefix arrays) plus each frame's single-frame
    # workspace, so a batch of one needs more than jxlr_workspace_bytes alone
    ps = [J.params(100, 50, epf_iters=0), J.params(256, 256, epf_iters=2), J.params(8, 8)]
    total = J.batch_workspace_bytes(ps)
    assert total % 256 == 0
    assert total > sum(J.workspace_bytes(p) for p in ps)
    assert J.batch_workspace_bytes(ps[:1]) > J.workspace_bytes(ps[0])
    assert J.batch_workspace_bytes([]) == 0
    assert J.batch_workspace_bytes(ps + [J.params(64, 64, epf_iters=4)]) == 0
    # frames with options carry their single-frame workspace (prediction sums,
    # the constraint's third buffer, noise channels, the Gaborish plane,
    # spline samples) plus one table entry per option stage they take
    opts = [dict(qco=1, epf_iters=2), dict(ac_prediction=1), dict(noise=1), dict(num_patches=3),
            dict(num_dots=3, gab=1), dict(num_splines=1, num_spline_points=2)]
    for o in opts:
        q = J.params(64, 64, **o)
        extra = J.batch_workspace_bytes(ps + [q]) - total
        assert extra >= J.workspace_bytes(q), o
        assert extra <= J.workspace_bytes(q) + 256 * 8 + 4096, o


# --- the library's constant tables versus the oracle's --------------------

@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = tmp_path_factory.mktemp("shim") / "libtableshim.so"
    csrc = os.path.join(ROOT, "paper_1908_03565_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O2", "-shared", "-fPIC", "-I", csrc,
                    os.path.join(ROOT, "tests", "native", "table_shim.cpp"),
                    os.path.join(csrc, "jxlr_tables.cpp"), "-o", str(out)], check=True)
    L = C.CDLL(str(out))
    for f in ("shim_t8", "shim_t16", "shim_t32", "shim_m4", "shim_a16", "shim_a32", "shim_dq",
              "shim_dqs", "shim_a16s", "shim_a32s", "shim_b16s", "shim_b32s", "shim_pred_u",
              "shim_pred_v"):
        getattr(L, f).restype = C.POINTER(C.c_float)
    L.shim_noise_nib.restype = C.POINTER(C.c_uint64)
    L.shim_pred_sf.restype = C.c_float
    L.shim_pred_s8_1.restype = C.c_float
    L.shim_spline_scale.restype = C.POINTER(C.c_double)
    L.shim_mul.restype = C.POINTER(C.c_int32)
    L.shim_thr.restype = C.POINTER(C.c_float)
    L.shim_mfma.restype = C.POINTER(C.c_uint16)
    L.shim_start8.restype = C.POINTER(C.c_uint8)
    L.shim_afv.restype = C.POINTER(C.c_float)
    assert L.shim_build() == 1
    return L


def _arr(ptr, n):
    return np.ctypeslib.as_array(ptr, shape=(n,)).copy()


DQ_FLOATS = 3 * (4 * 64 + 256 + 1024 + 2 * 128 + 2 * 256 + 2 * 512 + 3 * 64)


def test_dequant_tables_match_oracle(shim):
    for s in range(15):
        bx, by = O.varblock_size(s)
        for c in range(3):
            buf = np.zeros(bx * by)
            assert shim.shim_dequant(s, c, buf.ctypes.data_as(C.POINTER(C.c_double))) == 1
            ref = O.dequant_matrix(s, c).ravel()
            np.testing.assert_allclose(buf[1:], ref[1:], rtol=1e-12, err_msg=f"{s},{c}")
            f32 = _arr(shim.shim_dq(), DQ_FLOATS)[shim.shim_dq_offset(s) + c * bx * by:][:bx * by]
            np.testing.assert_allclose(f32[1:], ref[1:], rtol=1e-7)


def test_encoded_dequant_tables_match_oracle(shim):
    # random encodings of every mode (the two sides build them independently)
    assert shim.shim_encoding_size() == C.sizeof(J.DequantEncoding)
    for seed in range(12):
        encs = wl.dequant_encodings(seed)
        arr = J.dequant_encodings(encs)
        for s in range(15):
            bx, by = O.varblock_size(s)
            for c in range(3):
                buf = np.zeros(bx * by)
                assert shim.shim_dequant_enc(s, c, C.cast(arr, C.c_void_p),
                                             buf.ctypes.data_as(C.POINTER(C.c_double))) == 1
                ref = O.dequant_matrix(s, c, encs).ravel()
                np.testing.assert_allclose(buf[1:], ref[1:], rtol=1e-12, err_msg=f"{seed},{s},{c}")
    # ill-formed encodings are rejected by both
    bad = [{"mode": 0}] * 15
    for s, e in ((4, {"mode": 1, "params": [[1.0] * 3] * 3}), (3, {"mode": 7, "copy_from": 3}),
                 (0, {"mode": 9}), (5, {"mode": 6, "num_bands": 1, "num_ecc_bands": 1,
                                        "dist_bands": [[1.0]] * 3, "ecc_bands": [[0.0]] * 3}),
                 (0, {"mode": 6, "num_bands": 2, "num_ecc_bands": 1,
                      "dist_bands": [[-1.0, 0.0]] * 3, "ecc_bands": [[0.0]] * 3})):
        encs = list(bad)
        encs[s] = e
        arr = J.dequant_encodings(encs)
        buf = np.zeros(1024)
        assert shim.shim_dequant_enc(s, 0, C.cast(arr, C.c_void_p),
                                     buf.ctypes.data_as(C.POINTER(C.c_double))) == 0, e
        with pytest.raises(O.OracleError):
            O.dequant_matrix(s, 0, encs)


def test_create_rejects_ill_formed_encodings_before_any_device_call():
    # the encodings are checked while the tables are built, before the
    # device is touched, so this runs without a GPU
    for s, e in ((4, {"mode": 1, "params": [[1.0] * 3] * 3}), (6, {"mode": 7, "copy_from": 9}),
                 (0, {"mode": 6, "num_bands": 2, "num_ecc_bands": 1,
                      "dist_bands": [[0.0, 0.0]] * 3, "ecc_bands": [[0.0]] * 3})):
        encs = [{"mode": 0}] * 15
        encs[s] = e
        h = C.c_void_p()
        st = J.lib().jxlr_create(C.byref(h), 0, C.cast(J.dequant_encodings(encs), C.c_void_p))
        assert st == 6 and not h.value, (s, e)


def test_cfl_and_dc_multiplier_helpers():
    # Annex G on every byte value, exact in binary32
    v = np.arange(256, dtype=np.uint8)
    kx, kb = J.cfl_from_u8(v, v)
    np.testing.assert_array_equal(kx, ((v.astype(np.float64) - 128) / 256).astype(np.float32))
    np.testing.assert_array_equal(kb, (0.935669 + (v.astype(np.float64) - 128) / 128).astype(np.float32))
    assert kx[128] == 0.0 and kb[128] == np.float32(0.935669)
    kx, kb = J.cfl_from_u8(x_factor=v)
    assert kb is None and kx[0] == -0.5
    # C.4.1: defaults {4096, 512, 256} over global_scale * quant_dc
    np.testing.assert_allclose(J.dc_mul_from_header(None, 1, 1), [4096, 512, 256])
    np.testing.assert_allclose(J.dc_mul_from_header(None, 8192, 16), [4096 / 131072, 512 / 131072,
                                                                       256 / 131072], rtol=1e-7)
    np.testing.assert_allclose(J.dc_mul_from_header([3.0, 5.0, 7.0], 2, 3), [0.5, 5 / 6, 7 / 6],
                               rtol=1e-7)
    assert J.params(8, 8).dc_mul[0] == J.dc_mul_from_header()[0]
    for args in (([1.0, 0.0, 1.0], 1, 1), (None, 0, 1), (None, 1, 0), (None, 65537, 1),
                 ([1.0, float("nan"), 1.0], 1, 1)):
        with pytest.raises(J.JxlrError):
            J.dc_mul_from_header(*args)


def test_afv_basis_matches_oracle(shim):
    np.testing.assert_allclose(_arr(shim.shim_afv(), 256).reshape(16, 16), O.afv_basis(),
                               rtol=0, atol=6e-8)


def test_transform_tables_match_oracle(shim):
    for n in (4, 8, 16, 32):
        buf = np.zeros(n * n)
        shim.shim_inverse(n, buf.ctypes.data_as(C.POINTER(C.c_double)))
        np.testing.assert_allclose(buf.reshape(n, n), O.idct_matrix(n), atol=1e-13)
    for n, f in ((8, shim.shim_t8), (16, shim.shim_t16), (32, shim.shim_t32)):
        np.testing.assert_allclose(_arr(f(), n * n).reshape(n, n), O.idct_matrix(n), rtol=2e-7,
                                   atol=2e-7)
    t4 = O.idct_matrix(4)
    m4 = _arr(shim.shim_m4(), 64).reshape(8, 8)
    ref = np.zeros((8, 8))
    for h in range(2):
        for j in range(4):
            for i in range(4):
                ref[4 * h + j, h + 2 * i] = t4[j, i]
    np.testing.assert_allclose(m4, ref, atol=2e-7)


def test_llf_tables_match_oracle(shim):
    # a16 / a32 are the one-axis LLF-from-DC factors: the oracle's I.2.7 on
    # DCT16x8 (2 x 1 DC samples) and DCT32x8 (4 x 1) gives them column by column.
    for s, n, f in ((6, 2, shim.shim_a16), (8, 4, shim.shim_a32)):
        a = _arr(f(), n * n).reshape(n, n)
        ref = np.stack([O.llf_from_dc(s, e.reshape(1, n)).ravel() for e in np.eye(n)], axis=1)
        np.testing.assert_allclose(a, ref, atol=2e-7)


def test_mul_tables_match_oracle(shim):
    for shift in range(0, 9):
        t = np.zeros(673, np.int32)
        shim.shim_mul_table(shift, t.ctypes.data_as(C.POINTER(C.c_int32)))
        np.testing.assert_array_equal(t, O.mul_table(shift))
        np.testing.assert_array_equal(_arr(shim.shim_mul(shift), 673), O.mul_table(shift))


def _col_scale(n):
    """The draft's per-frequency scales of the n-point inverse, read off the
    oracle's matrix: T_n[0][k] = s_n(k) cos(pi k / (2 n))."""
    t = O.idct_matrix(n)
    return np.array([t[0, k] / np.cos(np.pi * k / (2 * n)) for k in range(n)])


def test_prescaled_tables_match_oracle(shim):
    # dqs = dq times the scales that turn the draft's inverse into the plain
    # DCT-III the kernels run; likewise a16s/a32s on the output frequency.
    dqs = _arr(shim.shim_dqs(), DQ_FLOATS)
    for s in range(15):
        bx, by = O.varblock_size(s)
        s4, s8, half = _col_scale(4), _col_scale(8), np.arange(8) // 2
        if s == 3:
            sc = np.outer(s4[half], s4[half])
        elif s == 12:  # rows: interleaved 4-point, columns: 8-point
            sc = np.outer(s4[half], s8)
        elif s == 13:
            sc = np.outer(s8, s4[half])
        elif s in (1, 2, 14):
            sc = np.ones((8, 8))
        else:
            sc = np.outer(_col_scale(by), _col_scale(bx))
        for c in range(3):
            got = dqs[shim.shim_dq_offset(s) + c * bx * by:][:bx * by].reshape(by, bx)
            ref = O.dequant_matrix(s, c) * sc
            np.testing.assert_allclose(got.ravel()[1:], ref.ravel()[1:], rtol=2e-7)
    for s, n, f in ((6, 2, shim.shim_a16s), (8, 4, shim.shim_a32s)):
        a = _arr(f(), n * n).reshape(n, n)
        ref = np.stack([O.llf_from_dc(s, e.reshape(1, n)).ravel() for e in np.eye(n)], axis=1)
        ref = ref * _col_scale(8 * n)[:n, None]
        np.testing.assert_allclose(a, ref, atol=2e-7)


def test_dc_from_llf_tables_match_oracle(shim):
    # b16s / b32s take the scaled LLF of one axis back to DC samples: the
    # oracle's I.2.6 on DCT16x8 / DCT32x8 with the scale removed again
    for s, n, f, fa in ((6, 2, shim.shim_b16s, shim.shim_a16s), (8, 4, shim.shim_b32s, shim.shim_a32s)):
        b = _arr(f(), n * n).reshape(n, n)
        a = _arr(fa(), n * n).reshape(n, n)
        np.testing.assert_allclose(b @ a, np.eye(n), atol=1e-6)
        sc = _col_scale(8 * n)[:n]
        ref = np.stack([O.dc_from_llf(s, (e / sc).reshape(1, n)).ravel() for e in np.eye(n)], axis=1)
        np.testing.assert_allclose(b, ref, atol=2e-6)


def test_ac_prediction_tables_match_oracle(shim):
    # pred_u: cells from DC (I.2.7 then I.2.6 at N = 4), pred_v: scaled
    # coefficients from cells (I.2.7 at N = 4), per axis; their 2-D products
    # against the oracle's maps for every DCT-family type
    U = _arr(shim.shim_pred_u(), 3 * 8 * 4).reshape(3, 8, 4)
    V = _arr(shim.shim_pred_v(), 3 * 8 * 8).reshape(3, 8, 8)
    m_of = {1: 0, 2: 1, 4: 2}
    rng = np.random.default_rng(7)
    for s in (0, 4, 5, 6, 7, 8, 9, 10, 11):
        bx, by = O.varblock_size(s)
        cx, cy = bx // 8, by // 8
        Ux, Uy = U[m_of[cx], :2 * cx, :cx], U[m_of[cy], :2 * cy, :cy]
        D = rng.standard_normal((cy, cx))
        np.testing.assert_allclose(Uy @ D @ Ux.T, O.dc2x2_from_llf(s, O.llf_from_dc(s, D)), atol=2e-6)
        Vx, Vy = V[m_of[cx], :2 * cx, :2 * cx], V[m_of[cy], :2 * cy, :2 * cy]
        S = rng.standard_normal((2 * cy, 2 * cx))
        sc = np.outer(_col_scale(by)[:2 * cy], _col_scale(bx)[:2 * cx])
        np.testing.assert_allclose((Vy @ S @ Vx.T) / sc, O.llf2x2_from_dc2x2(s, S), atol=1e-5)
    assert shim.shim_pred_sf() == pytest.approx(O.scalef(2, 8, 1), rel=1e-7)
    assert shim.shim_pred_s8_1() == pytest.approx(_col_scale(8)[1], rel=1e-7)


def test_spline_scale_table(shim):
    # DCTScale(k) of K.4: the oracle's ContinuousIDCT of a unit coefficient
    # at t = -1/2, where every cosine is 1
    got = np.ctypeslib.as_array(shim.shim_spline_scale(), shape=(32,))
    for k in range(32):
        e = np.zeros(32, np.float32)
        e[k] = 1.0
        assert got[k] == pytest.approx(O.spline_idct(e, -0.5), rel=1e-15, abs=0)


def _nib_apply(T, a, b):
    # T: (32, 16, 2) uint64; state (a, b) -> XOR of the entries its nibbles select
    o0 = o1 = 0
    for p in range(32):
        v = ((a if p < 16 else b) >> (4 * (p % 16))) & 15
        o0 ^= int(T[p, v, 0])
        o1 ^= int(T[p, v, 1])
    return o0, o1


def test_noise_jump_tables(shim):
    # power 0 is one generator step (first word a, second b: a' = b,
    # b' = u ^ b ^ (u >> 18) ^ (b >> 5), u = a ^ (a << 23)); each power is the
    # square of the one before; the entry of nibble value 0 is 0
    M = 2 ** 64 - 1
    T = np.ctypeslib.as_array(shim.shim_noise_nib(), shape=(14 * 32 * 16 * 2,)).reshape(14, 32, 16, 2)
    assert not T[:, :, 0, :].any()
    rng = np.random.default_rng(9)
    for _ in range(4):
        a, b = (int(v) for v in rng.integers(0, 2 ** 63, size=2, dtype=np.int64))
        a |= 1 << 63
        u = (a ^ (a << 23)) & M
        assert _nib_apply(T[0], a, b) == (b, (u ^ b ^ (u >> 18) ^ (b >> 5)) & M)
        for k in (0, 5, 12):
            twice = _nib_apply(T[k], *_nib_apply(T[k], a, b))
            assert twice == _nib_apply(T[k + 1], a, b), k


def test_schedule_cache_roundtrip(tmp_path):
    from paper_1908_03565_amd import tuning
    path = str(tmp_path / "d" / "s.json")
    assert tuning._load(path) == {}
    tuning._store(path, {"k": {"grid_recon": 3}})
    assert tuning._load(path) == {"k": {"grid_recon": 3}}
    plan = J.BatchPlan()
    plan.total_tiles, plan.max_epf_iters = 1000, 2
    assert tuning.batch_key("dev", plan) == "dev|tiles~1024|epf2"
    open(path, "w").write("not json")
    assert tuning._load(path) == {}


@pytest.mark.parametrize("bits", [8, 16])
def test_srgb_thresholds_match_oracle_rounding(shim, bits):
    # thr[k] is the first binary32 value the oracle's binary64 rounding sends
    # to code k, and the float just below it goes to k - 1
    maxv = (1 << bits) - 1
    thr = _arr(shim.shim_thr(bits), maxv + 2)
    assert thr[0] == -np.inf and thr[-1] == np.inf
    t = thr[1:-1].astype(np.float32)
    below = np.nextafter(t, np.float32(-1))
    k = np.arange(1, maxv + 1)
    assert np.all(np.diff(t) > 0)
    np.testing.assert_array_equal(O.quantize_srgb(bits, t.astype(np.float64)), k)
    np.testing.assert_array_equal(O.quantize_srgb(bits, below.astype(np.float64)), k - 1)


def test_srgb_8bit_bucket_code_is_oracle_rounding(shim):
    # the kernel's 8-bit code (bucket of the clamped value's bit pattern, then
    # one threshold) equals the oracle's rounding over a dense sweep of binary32
    # values in and around [0, 1], every bucket boundary and every threshold
    B0, nb = shim.shim_bucket0(), shim.shim_buckets()
    start = _arr(shim.shim_start8(), nb).astype(np.int64)
    thr = _arr(shim.shim_thr(8), 257).astype(np.float32)

    def code8(v):
        v = np.asarray(v, np.float32)
        c = np.fmin(np.fmax(v, np.float32(0)), np.float32(1))  # as fminf / fmaxf
        b = np.maximum((c.view(np.uint32) >> 16).astype(np.int64) - B0, 0)
        s = start[b]
        return s + (c >= thr[s + 1])

    sweep = np.arange(0, 0x3F800001, 997, dtype=np.uint32).view(np.float32)
    edges = (np.arange(B0, B0 + nb, dtype=np.uint32) << 16).view(np.float32)
    t = thr[1:-1]
    vals = np.concatenate([sweep, edges, np.nextafter(edges, np.float32(-1)), t,
                           np.nextafter(t, np.float32(-1)), np.nextafter(t, np.float32(2)),
                           np.float32([-1.0, -0.0, 1.0, 1.5, 3e38, -np.inf, np.inf])])
    ref = O.quantize_srgb(8, vals.astype(np.float64))
    np.testing.assert_array_equal(code8(vals), ref)
    # each bucket spans at most two codes, as the kernel relies on
    assert np.all(np.diff(start) >= 0) and start[0] == 0 and start[-1] == 255


@pytest.mark.parametrize("m", [0, 1, 2])
def test_split_transform_operands(shim, m):
    # the split matrices, put back in matrix order, are 16 times the
    # block-diagonal plain DCT-III of 8 << m points; hi is the binary16
    # rounding of each entry and hi + lo is within 2^-21 of it (in units of
    # the unscaled matrix)
    raw = np.ctypeslib.as_array(shim.shim_mfma(m), shape=(2 * 2 * 64 * 8,)).copy()
    parts = raw.view(np.float16).reshape(2, 2, 64, 8).astype(np.float64) / 16.0
    A = np.zeros((2, 32, 32))
    for part in range(2):
        for step in range(2):
            for lane in range(64):
                for e in range(8):
                    A[part, lane % 32, 16 * step + 8 * (lane // 32) + e] = parts[part, step, lane, e]
    N = 8 << m
    i, k = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    ref = np.where(i // N == k // N, np.cos(np.pi * (2 * (i % N) + 1) * (k % N) / (2 * N)), 0.0)
    assert np.abs(A[0] + A[1] - ref).max() <= 2.0 ** -21
    assert np.all(np.abs(A[0] - ref) <= np.abs(ref) * 2.0 ** -11 + 1e-30)
    assert np.array_equal(np.float16(16.0 * ref).astype(np.float64) / 16.0, A[0])


def test_crops_are_well_formed_frames():
    mother = wl.frame(1024, 768, seed=57, epf_iters=2)
    rng = np.random.default_rng(3)
    for _ in range(40):
        W = int(rng.integers(1, 129)) * 8
        H = int(rng.integers(1, 97)) * 8
        x0 = 64 * int(rng.integers(0, (1024 - W) // 64 + 1))
        y0 = 64 * int(rng.integers(0, (768 - H) // 64 + 1))
        f = wl.crop(mother, x0, y0, W, H, epf_iters=1, out_format=2)
        p = J.params(W, H, out_format=f["out_format"], **f["params"])
        assert J.validate_maps_host(p, f) == 0, (W, H, x0, y0)
        # coefficients and DC are the mother's, position for position
        np.testing.assert_array_equal(f["ac"][:, :8, :8], mother["ac"][:, y0:y0 + 8, x0:x0 + 8])
        assert f["cfl_kx"].shape == ((H + 63) // 64, (W + 63) // 64)


def test_serving_requests_recipe():
    reqs = wl.c5_requests()
    assert 11000 < len(reqs) < 13000          # Poisson 200/s over 60 s
    t = np.array([q[0] for q in reqs])
    assert np.all(np.diff(t) > 0) and t[-1] < 60.0
    W = np.array([q[1] for q in reqs]); H = np.array([q[2] for q in reqs])
    assert W.min() >= 64 and W.max() <= 4096 and np.all(W % 8 == 0) and np.all(H % 8 == 0)
    u16 = np.mean([q[6] == 2 for q in reqs])
    assert 0.27 < u16 < 0.33
    assert set(q[5] for q in reqs) == {0, 1, 2, 3}
    assert all(q[3] + q[1] <= 4096 and q[4] + q[2] <= 4096 and q[3] % 64 == 0 for q in reqs)


def test_footprint_covers_workspace():
    from paper_1908_03565_amd import serving
    p = J.params(640, 480, epf_iters=2, out_format=2)
    fp = serving.footprint_bytes(p)
    assert fp >= J.workspace_bytes(p) + 640 * 480 * 12 + 3 * 640 * 480 * 2  # AC in, u16 out


def test_jpeg1_params_blocks_and_workspace():
    from paper_1908_03565_amd import workload as wl
    j = wl.jpeg1(100, 60, 1)
    jp = J.jpeg1_params(j)
    got = []
    for c in range(3):
        w, h = C.c_int32(), C.c_int32()
        assert J.lib().jxlr_jpeg1_blocks(C.byref(jp), c, C.byref(w), C.byref(h)) == 0
        got.append((w.value, h.value))
    # whole 16 x 16 MCUs over 100 x 60: 7 x 4 of them
    assert got == [(14, 8), (7, 4), (7, 4)]
    assert [c.shape for c in j["coef"]] == [(64, 112), (32, 56), (32, 56)]
    ws = J.lib().jxlr_jpeg1_workspace_bytes(C.byref(jp))
    assert ws == 112 * 64 * 4 + 2 * 56 * 32 * 4
    bad = []
    for field, val in (("num_components", 2), ("xsize", 0)):
        q = J.jpeg1_params(j)
        setattr(q, field, val)
        bad.append(q)
    q = J.jpeg1_params(j)
    q.h_samp[1] = 3
    bad.append(q)
    q = J.jpeg1_params(j)
    q.h_samp[1] = 2
    q.h_samp[0] = 1  # the luma must carry the largest factors
    bad.append(q)
    q = J.jpeg1_params(j)
    q.quant[2][5] = 0
    bad.append(q)
    for q in bad:
        assert J.lib().jxlr_jpeg1_workspace_bytes(C.byref(q)) == 0
