"""ctypes front end of the FP64 oracle (test infrastructure only).

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this module.  It loads oracle/liboracle.so (building it with gcc when it is
missing) and marshals numpy arrays; all arithmetic is in jxl_oracle.c.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None


class OrcParams(C.Structure):
    _fields_ = [
        ("xsize", C.c_int32), ("ysize", C.c_int32),
        ("global_scale", C.c_int32),
        ("dc_mul", C.c_double * 3),
        ("extra_levels", C.c_int32 * 3),
        ("kx_dc", C.c_double), ("kb_dc", C.c_double),
        ("gab", C.c_int32),
        ("gab_w1", C.c_double * 3), ("gab_w2", C.c_double * 3),
        ("epf_iters", C.c_int32),
        ("epf_weight_min", C.c_double),
        ("epf_scale", C.c_double * 3),
        ("epf_sharp_lut", C.c_double * 8),
        ("epf_range_max", C.c_double), ("epf_range_mul", C.c_double),
        ("epf_quant_mul", C.c_double),
        ("epf_sigma_max", C.c_int32),
        ("epf_sigma_shift", C.c_int32),
        ("opsin_inv", C.c_double * 9),
        ("opsin_bias", C.c_double * 3),
        ("target_nits_div50", C.c_int32),
        ("dc_smoothing", C.c_int32),
        ("qco", C.c_int32),
        ("qco_interval_mul", C.c_double),
        ("ac_prediction", C.c_int32),
        ("noise", C.c_int32),
        ("noise_lut", C.c_double * 16),
        ("dot_colour_quant", C.c_double * 3),
        ("dq_enc", C.c_void_p),
        ("dc_quant_field", C.c_void_p),
    ]


class OrcDequantEncoding(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("copy_from", C.c_int32),
        ("num_bands", C.c_int32), ("num_ecc_bands", C.c_int32),
        ("dist_bands", (C.c_double * 17) * 3),
        ("ecc_bands", (C.c_double * 8) * 3),
        ("params", (C.c_double * 6) * 3),
        ("afv_weights", (C.c_double * 8) * 3),
    ]


def _encoding_struct(e):
    """OrcDequantEncoding from a dict (mode, copy_from, num_bands,
    num_ecc_bands, dist_bands [3][<=17], ecc_bands [3][<=8], params [3][<=6],
    afv_weights [3][8]); absent keys are 0."""
    out = OrcDequantEncoding()
    for k in ("mode", "copy_from", "num_bands", "num_ecc_bands"):
        setattr(out, k, int(e.get(k, 0)))
    for k in ("dist_bands", "ecc_bands", "params", "afv_weights"):
        if k in e:
            arr = getattr(out, k)
            for c, row in enumerate(e[k]):
                for i, v in enumerate(row):
                    arr[c][i] = float(v)
    return out


def _encoding_dict(st):
    return {"mode": st.mode, "copy_from": st.copy_from, "num_bands": st.num_bands,
            "num_ecc_bands": st.num_ecc_bands,
            "dist_bands": [list(st.dist_bands[c])[:st.num_bands] for c in range(3)],
            "ecc_bands": [list(st.ecc_bands[c])[:st.num_ecc_bands] for c in range(3)],
            "params": [list(st.params[c]) for c in range(3)],
            "afv_weights": [list(st.afv_weights[c]) for c in range(3)]}


_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.POINTER(OrcParams)
        L.orc_params_default.argtypes = [P, C.c_int32, C.c_int32]
        L.orc_varblock_size.argtypes = [C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_idct_matrix.argtypes = [C.c_int32, _f64p]
        L.orc_fdct_matrix.argtypes = [C.c_int32, _f64p]
        for f in ("orc_scale_I", "orc_scale_D"):
            getattr(L, f).argtypes = [C.c_int32, C.c_int32]
            getattr(L, f).restype = C.c_double
        L.orc_scalef.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        L.orc_scalef.restype = C.c_double
        L.orc_inverse_transform.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_forward_transform.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_llf_from_dc.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_dc_from_llf.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_dc2x2_from_llf.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_llf2x2_from_dc2x2.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_ac_prediction_image.argtypes = [P, C.c_int32, C.c_int32, _u8p, _f64p, _f64p,
                                              C.c_void_p]
        L.orc_dequant_matrix.argtypes = [C.c_int, C.c_int, _f64p]
        L.orc_dequant_matrix_enc.argtypes = [C.c_int, C.c_int, C.c_void_p, _f64p]
        L.orc_default_encoding.argtypes = [C.c_int, C.POINTER(OrcDequantEncoding)]
        L.orc_afv_basis.argtypes = [_f64p]
        L.orc_dc_smooth.argtypes = [P, C.c_int32, C.c_int32, _f64p]
        ptr3 = C.c_void_p * 3
        L.orc_reconstruct.argtypes = [P, ptr3, ptr3, _u8p, _u8p, _f32p, _f32p, _f64p]
        L.orc_epf_mul_table.argtypes = [C.c_int32, _i32p]
        L.orc_epf_weight.argtypes = [C.c_int32, C.c_int32]
        L.orc_epf_weight.restype = C.c_float
        L.orc_epf_pass.argtypes = [P, _u8p, _u8p, _u8p, _f64p, _f64p, C.c_void_p, C.c_void_p]
        L.orc_qco.argtypes = [P, _u8p, _u8p, _f64p, _f64p, _f64p]
        L.orc_gaborish.argtypes = [P, _f64p, _f64p]
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_noise_step.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.orc_noise_step.restype = C.c_uint64
        L.orc_noise_channels.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _f32p]
        L.orc_noise.argtypes = [P, _f64p, _f64p]
        L.orc_patches.argtypes = [P, _i32p, C.c_int32, _i32p, _f64p]
        L.orc_decode_features.argtypes = [P, ptr3, ptr3, _u8p, _u8p, _u8p, _f32p, _f32p,
                                          C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                          C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                          C.c_void_p, _f64p]
        L.orc_dots.argtypes = [P, _i32p, C.c_int32, _f64p]
        L.orc_jpeg1_component.argtypes = [_i32p, C.c_int32, C.c_int32, _i32p, _f64p]
        L.orc_jpeg1_gaborish.argtypes = [_f64p, C.c_int32, C.c_int32, _u8p]
        L.orc_upsample2.argtypes = [_f64p, C.c_int32, C.c_size_t, _f64p, C.c_size_t]
        L.orc_upsample2.restype = None
        L.orc_jpeg1_rasterize.argtypes = [C.c_int32, C.c_void_p * 3, _i32p, _i32p, _i32p, _i32p,
                                          C.c_int32, C.c_int32, _f64p]
        L.orc_spline_idct.argtypes = [_f32p, C.c_double]
        L.orc_spline_idct.restype = C.c_double
        L.orc_spline_curve.argtypes = [_i32p, C.c_int32, _f64p, _f64p]
        L.orc_spline_curve.restype = C.c_int32
        L.orc_spline_walk.argtypes = [_f64p, _f64p, C.c_int32, C.c_void_p, C.c_int32,
                                      C.POINTER(C.c_double)]
        L.orc_spline_walk.restype = C.c_int32
        L.orc_splines.argtypes = [P, _i32p, C.c_int32, _i32p, _f32p, _f64p, C.c_void_p]
        L.orc_xyb_to_rgb.argtypes = [P, _f64p, _f64p]
        L.orc_quantize_srgb.argtypes = [C.c_int32, C.c_int64, _f64p, _u16p]
        L.orc_decode.argtypes = [P, ptr3, ptr3, _u8p, _u8p, _u8p, _f32p, _f32p, _f64p]
        L.orc_num_threads.restype = C.c_int
        _LIB = L
    return _LIB


class OracleError(RuntimeError):
    pass


def _check(st):
    if st != 0:
        raise OracleError(f"oracle returned status {st}")


# Transform types in the order of the C.5.4 table.
STRATEGY_NAMES = ["DCT8", "IDENTITY", "DCT2", "DCT4", "DCT16", "DCT32", "DCT16X8",
                  "DCT8X16", "DCT32X8", "DCT8X32", "DCT32X16", "DCT16X32",
                  "DCT4X8", "DCT8X4", "AFV"]
SUPPORTED = list(range(15))


def varblock_size(s):
    bx, by = C.c_int32(), C.c_int32()
    if not lib().orc_varblock_size(s, C.byref(bx), C.byref(by)):
        raise OracleError(f"unknown transform type {s}")
    return bx.value, by.value


def params(xsize, ysize, dq_enc=None, **overrides):
    """Oracle parameter struct: the draft's defaults, then `overrides`.
    dq_enc: None (the C.6.1.1 defaults) or 15 encoding dicts (see
    _encoding_struct), indexed by transform type."""
    p = OrcParams()
    lib().orc_params_default(C.byref(p), int(xsize), int(ysize))
    p._keep = {}
    if dq_enc is not None:
        if len(dq_enc) != 15:
            raise ValueError("dq_enc needs 15 encodings")
        arr = (OrcDequantEncoding * 15)(*[_encoding_struct(e) for e in dq_enc])
        p._keep["dq_enc"] = arr
        p.dq_enc = C.cast(arr, C.c_void_p)
    for k, v in overrides.items():
        cur = getattr(p, k)
        if isinstance(cur, C.Array):
            arr = np.asarray(v, dtype=np.float64).ravel()
            if len(arr) != len(cur):
                raise ValueError(k)
            for i, x in enumerate(arr):
                cur[i] = type(cur[0])(x) if not isinstance(cur[0], float) else float(x)
        else:
            setattr(p, k, v)
    return p


def idct_matrix(N):
    out = np.zeros(N * N)
    _check(lib().orc_idct_matrix(N, out))
    return out.reshape(N, N)


def fdct_matrix(N):
    out = np.zeros(N * N)
    _check(lib().orc_fdct_matrix(N, out))
    return out.reshape(N, N)


def scale_I(N, u):
    return lib().orc_scale_I(N, u)


def scale_D(N, u):
    return lib().orc_scale_D(N, u)


def scalef(N, n, x):
    return lib().orc_scalef(N, n, x)


def inverse_transform(s, coeffs):
    bx, by = varblock_size(s)
    K = np.ascontiguousarray(coeffs, dtype=np.float64).reshape(by, bx)
    out = np.zeros((by, bx))
    _check(lib().orc_inverse_transform(s, K, out))
    return out


def forward_transform(s, samples):
    bx, by = varblock_size(s)
    S = np.ascontiguousarray(samples, dtype=np.float64).reshape(by, bx)
    out = np.zeros((by, bx))
    _check(lib().orc_forward_transform(s, S, out))
    return out


def llf_from_dc(s, dc):
    bx, by = varblock_size(s)
    cx, cy = bx // 8, by // 8
    if s not in (0, 4, 5, 6, 7, 8, 9, 10, 11):
        cx = cy = 1
    D = np.ascontiguousarray(dc, dtype=np.float64).reshape(cy, cx)
    out = np.zeros((cy, cx))
    _check(lib().orc_llf_from_dc(s, D, out))
    return out


def dc_from_llf(s, llf):
    bx, by = varblock_size(s)
    cx, cy = bx // 8, by // 8
    if s not in (0, 4, 5, 6, 7, 8, 9, 10, 11):
        cx = cy = 1
    L = np.ascontiguousarray(llf, dtype=np.float64).reshape(cy, cx)
    out = np.zeros((cy, cx))
    _check(lib().orc_dc_from_llf(s, L, out))
    return out


def _lf_shape(s):
    bx, by = varblock_size(s)
    if s not in (0, 4, 5, 6, 7, 8, 9, 10, 11):
        return 1, 1
    return bx // 8, by // 8


def dc2x2_from_llf(s, llf):
    """I.2.6 at N = 4: LLF (cy, cx) -> cells (2cy, 2cx)."""
    cx, cy = _lf_shape(s)
    L = np.ascontiguousarray(llf, dtype=np.float64).reshape(cy, cx)
    out = np.zeros((2 * cy, 2 * cx))
    _check(lib().orc_dc2x2_from_llf(s, L, out))
    return out


def llf2x2_from_dc2x2(s, cells):
    """I.2.7 at N = 4: cells (2cy, 2cx) -> the top (2cy, 2cx) coefficients."""
    cx, cy = _lf_shape(s)
    D = np.ascontiguousarray(cells, dtype=np.float64).reshape(2 * cy, 2 * cx)
    out = np.zeros((2 * cy, 2 * cx))
    _check(lib().orc_llf2x2_from_dc2x2(s, D, out))
    return out


def ac_prediction_image(p, strategy, dcq, want_margin=False):
    """Annex H image step: smoothed cells (3, 2Hb, 2Wb) from DC (3, Hb, Wb);
    with want_margin also each cell's |wa - s| - 1.7 dcq."""
    d = np.ascontiguousarray(dcq, dtype=np.float64)
    Hb, Wb = d.shape[1], d.shape[2]
    out = np.zeros((3, 2 * Hb, 2 * Wb))
    margin = np.zeros((3, 2 * Hb, 2 * Wb))
    lib().orc_ac_prediction_image(C.byref(p), Wb, Hb,
                                  np.ascontiguousarray(strategy, np.uint8), d, out,
                                  margin.ctypes.data if want_margin else None)
    return (out, margin) if want_margin else out


def dc_smooth(p, dcq, field=None):
    """F.2 adaptive DC smoothing of a dequantized DC image (3, Hb, Wb);
    field: its DcQuantField (3, Hb, Wb), or None."""
    d = np.array(dcq, dtype=np.float64, order="C", copy=True)
    with _Field(p, {"dc_quant": field} if field is not None else None):
        lib().orc_dc_smooth(C.byref(p), d.shape[2], d.shape[1], d)
    return d


def afv_basis():
    out = np.zeros(256)
    lib().orc_afv_basis(out)
    return out.reshape(16, 16)


def dequant_matrix(s, c, dq_enc=None):
    """Dequantization matrix (by, bx) of type s and channel c under the
    encodings dq_enc (None: the C.6.1.1 defaults)."""
    bx, by = varblock_size(s)
    out = np.zeros(bx * by)
    if dq_enc is None:
        _check(lib().orc_dequant_matrix(s, c, out))
    else:
        arr = (OrcDequantEncoding * 15)(*[_encoding_struct(e) for e in dq_enc])
        _check(lib().orc_dequant_matrix_enc(s, c, C.cast(arr, C.c_void_p), out))
    return out.reshape(by, bx)


def default_encoding(s):
    """The C.6.1.1 default encoding of type s, as a dict."""
    st = OrcDequantEncoding()
    _check(lib().orc_default_encoding(s, C.byref(st)))
    return _encoding_dict(st)


class _Field:
    """Points p.dc_quant_field at frame["dc_quant"] (C.5.2 DcQuantField,
    float (3, Hb, Wb)) for the duration of a call, if the frame has one."""

    def __init__(self, p, frame):
        self.p, self.frame = p, frame

    def __enter__(self):
        f = self.frame.get("dc_quant") if self.frame is not None else None
        self.old = self.p.dc_quant_field
        if f is not None:
            self.arr = np.ascontiguousarray(f, np.float32)
            Hb, Wb = (self.p.ysize + 7) // 8, (self.p.xsize + 7) // 8
            if self.arr.shape != (3, Hb, Wb):
                raise ValueError("dc_quant must be (3, Hb, Wb)")
            self.p.dc_quant_field = self.arr.ctypes.data
        return self

    def __exit__(self, *a):
        self.p.dc_quant_field = self.old


def _planes(arrs, dtype):
    keep = [np.ascontiguousarray(a, dtype=dtype) for a in arrs]
    ptrs = (C.c_void_p * 3)(*[a.ctypes.data for a in keep])
    return keep, ptrs


def reconstruct(p, frame):
    """frame: dict with ac (3, 8Hb, 8Wb) int32, dc (3, Hb, Wb) int32,
    strategy, qf (Hb, Wb) uint8, cfl_kx, cfl_kb float32 tiles.
    Returns XYB (3, ysize, xsize) float64."""
    ka, pa = _planes(frame["ac"], np.int32)
    kd, pd = _planes(frame["dc"], np.int32)
    out = np.zeros((3, p.ysize, p.xsize))
    with _Field(p, frame):
        _check(lib().orc_reconstruct(
            C.byref(p), pa, pd, np.ascontiguousarray(frame["strategy"], np.uint8),
            np.ascontiguousarray(frame["qf"], np.uint8),
            np.ascontiguousarray(frame["cfl_kx"], np.float32),
            np.ascontiguousarray(frame["cfl_kb"], np.float32), out))
    return out


def mul_table(shift=0):
    t = np.zeros(673, dtype=np.int32)
    _check(lib().orc_epf_mul_table(shift, t))
    return t


def epf_weight(sad, mul):
    return lib().orc_epf_weight(int(sad), int(mul))


def epf_pass(p, frame, xyb, want_debug=False):
    """One J.2 pass.  Returns out, or (out, guide u8 (3,H,W), sigma int32 (Hb,Wb))."""
    xyb = np.ascontiguousarray(xyb, dtype=np.float64)
    out = np.zeros_like(xyb)
    Hb, Wb = (p.ysize + 7) // 8, (p.xsize + 7) // 8
    guide = np.zeros((3, p.ysize, p.xsize), np.uint8)
    sigma = np.zeros((Hb, Wb), np.int32)
    _check(lib().orc_epf_pass(
        C.byref(p), np.ascontiguousarray(frame["strategy"], np.uint8),
        np.ascontiguousarray(frame["qf"], np.uint8),
        np.ascontiguousarray(frame["sharpness"], np.uint8), xyb, out,
        guide.ctypes.data if want_debug else None,
        sigma.ctypes.data if want_debug else None))
    if want_debug:
        return out, guide, sigma
    return out


def qco(p, frame, orig, filt):
    """J.3 quantization constraint: orig is the input of the first EPF pass,
    filt the output of the last; returns the constrained frame."""
    orig = np.ascontiguousarray(orig, dtype=np.float64)
    filt = np.ascontiguousarray(filt, dtype=np.float64)
    out = np.zeros_like(filt)
    with _Field(p, frame):
        _check(lib().orc_qco(
            C.byref(p), np.ascontiguousarray(frame["strategy"], np.uint8),
            np.ascontiguousarray(frame["qf"], np.uint8), orig, filt, out))
    return out


def patches(p, place, samples, xyb):
    """K.3: placements (n, 5) = (x, y, xsize, ysize, sample offset) over the
    flat integer samples; returns the image with the patches added."""
    out = np.array(xyb, dtype=np.float64, order="C", copy=True)
    pl = np.ascontiguousarray(place, np.int32).reshape(-1, 5)
    sm = np.ascontiguousarray(samples, np.int32).ravel()
    _check(lib().orc_patches(C.byref(p), pl, len(pl), sm if sm.size else np.zeros(1, np.int32), out))
    return out


def dots(p, quantized, xyb):
    """K.2: quantized dots (n, 10) added to a copy of the image."""
    out = np.array(xyb, dtype=np.float64, order="C", copy=True)
    q = np.ascontiguousarray(quantized, np.int32).reshape(-1, 10)
    _check(lib().orc_dots(C.byref(p), q if len(q) else np.zeros((1, 10), np.int32), len(q), out))
    return out


def spline_idct(dct, t):
    """K.4 ContinuousIDCT of 32 coefficients at t."""
    return lib().orc_spline_idct(np.ascontiguousarray(dct, np.float32).ravel(), float(t))


def spline_curve(points):
    """K.4 step 1: the sequence C (m, 2) of the centripetal Catmull-Rom
    curve through the control points (n, 2); None if two consecutive control
    points coincide."""
    pts = np.ascontiguousarray(points, np.int32).reshape(-1, 2)
    n = len(pts)
    cap = 16 * (n - 1) + 1
    cx, cy = np.zeros(cap), np.zeros(cap)
    m = lib().orc_spline_curve(pts.ravel(), n, cx, cy)
    return None if m < 0 else np.stack([cx[:m], cy[:m]], axis=1)


def spline_walk(curve):
    """K.4 steps 2-3: the points P (np, 4) of (x, y, l, d) at unit arc
    length along the polyline through C, and its length L."""
    c = np.ascontiguousarray(curve, np.float64).reshape(-1, 2)
    cx, cy = np.ascontiguousarray(c[:, 0]), np.ascontiguousarray(c[:, 1])
    L = C.c_double()
    n = lib().orc_spline_walk(cx, cy, len(c), None, 0, C.byref(L))
    P = np.zeros((n, 4))
    lib().orc_spline_walk(cx, cy, len(c), P.ctypes.data, n, C.byref(L))
    return P, L.value


def splines(p, offsets, points, dct, xyb, want_near=False):
    """K.4: splines added to a copy of the image.  offsets (n + 1,), points
    (m, 2) int32, dct (n, 4, 32) float32.  With want_near, also the [H][W]
    mask of pixels whose footprint test is within 1e-9 of its bound."""
    out = np.array(xyb, dtype=np.float64, order="C", copy=True)
    off = np.ascontiguousarray(offsets, np.int32).ravel()
    pts = np.ascontiguousarray(points, np.int32).reshape(-1, 2)
    d = np.ascontiguousarray(dct, np.float32).reshape(-1, 4, 32)
    near = np.zeros((p.ysize, p.xsize), np.uint8)
    _check(lib().orc_splines(C.byref(p), off, len(off) - 1,
                             pts.ravel() if pts.size else np.zeros(2, np.int32),
                             d.ravel() if d.size else np.zeros(128, np.float32), out,
                             near.ctypes.data))
    return (out, near.astype(bool)) if want_near else out


def jpeg1_component(qcoef, quant):
    """M.6.1-M.6.2: pixels [8 hib][8 wib] of one component's quantized
    coefficients (natural order per 8x8 block) and its quantization table."""
    q = np.ascontiguousarray(qcoef, np.int32)
    hib, wib = q.shape[0] // 8, q.shape[1] // 8
    out = np.zeros(q.shape)
    _check(lib().orc_jpeg1_component(q, wib, hib, np.ascontiguousarray(quant, np.int32).ravel(),
                                     out))
    return out


def jpeg1_gaborish(pix, code):
    """M.6.3 on one component's pixels [8 hib][8 wib]; code: the side
    channel's four bytes (weight1 * 1024, weight2 * 1024, threshold * 16,
    limit).  Returns the filtered plane."""
    out = np.array(pix, dtype=np.float64, order="C", copy=True)
    _check(lib().orc_jpeg1_gaborish(out, out.shape[1] // 8, out.shape[0] // 8,
                                    np.ascontiguousarray(code, np.uint8)))
    return out


def upsample2(a):
    """M.6.4 on a 1-D array."""
    a = np.ascontiguousarray(a, np.float64)
    out = np.zeros(2 * len(a))
    lib().orc_upsample2(a, len(a), 1, out, 1)
    return out


def jpeg1_rasterize(pixels, hs, vs, xsize, ysize):
    """M.6.4-M.6.6: RGB (3, ysize, xsize) from 1 or 3 component planes."""
    pl = [np.ascontiguousarray(p_, np.float64) for p_ in pixels]
    ptrs = (C.c_void_p * 3)(*([p_.ctypes.data for p_ in pl] + [None] * (3 - len(pl))))
    wib = np.array([p_.shape[1] // 8 for p_ in pl] + [1] * (3 - len(pl)), np.int32)
    hib = np.array([p_.shape[0] // 8 for p_ in pl] + [1] * (3 - len(pl)), np.int32)
    out = np.zeros((3, ysize, xsize))
    _check(lib().orc_jpeg1_rasterize(len(pl), ptrs, wib, hib,
                                     np.array(list(hs) + [1] * (3 - len(hs)), np.int32),
                                     np.array(list(vs) + [1] * (3 - len(vs)), np.int32),
                                     xsize, ysize, out))
    return out


def jpeg1_decode(j):
    """Whole M.6 path of a synthetic JPEG1 frame dict (see workload.jpeg1);
    with j["gab"] (one four-byte code per component) the M.6.3 side
    channel is applied."""
    pix = [jpeg1_component(c, q) for c, q in zip(j["coef"], j["quant"])]
    if j.get("gab") is not None:
        pix = [jpeg1_gaborish(p_, g) for p_, g in zip(pix, j["gab"])]
    return jpeg1_rasterize(pix, j["hs"], j["vs"], j["xsize"], j["ysize"])


def splitmix64(z):
    return lib().orc_splitmix64(int(z) & (2**64 - 1))


def noise_step(s0, s1):
    """One K.5.2 generator step on the state (s0, s1): returns (batch, s0', s1')."""
    a, b = C.c_uint64(int(s0) & (2**64 - 1)), C.c_uint64(int(s1) & (2**64 - 1))
    out = lib().orc_noise_step(C.byref(a), C.byref(b))
    return int(out), int(a.value), int(b.value)


def noise_channels(gw, gh, x0, y0):
    """K.5.2 pseudorandom channels (3, gh, gw), binary32."""
    out = np.zeros((3, gh, gw), np.float32)
    lib().orc_noise_channels(gw, gh, x0, y0, out)
    return out


def noise(p, xyb):
    """K.5 noise over a cropped XYB frame."""
    xyb = np.ascontiguousarray(xyb, dtype=np.float64)
    out = np.zeros_like(xyb)
    _check(lib().orc_noise(C.byref(p), xyb, out))
    return out


def gaborish(p, xyb):
    xyb = np.ascontiguousarray(xyb, dtype=np.float64)
    out = np.zeros_like(xyb)
    _check(lib().orc_gaborish(C.byref(p), xyb, out))
    return out


def xyb_to_rgb(p, xyb):
    xyb = np.ascontiguousarray(xyb, dtype=np.float64)
    out = np.zeros_like(xyb)
    _check(lib().orc_xyb_to_rgb(C.byref(p), xyb, out))
    return out


def quantize_srgb(bits, lin):
    lin = np.ascontiguousarray(lin, dtype=np.float64)
    out = np.zeros(lin.shape, np.uint16)
    _check(lib().orc_quantize_srgb(bits, lin.size, lin, out))
    return out


def decode(p, frame):
    """Whole path: returns [0,1]-scaled linear RGB (3, ysize, xsize) float64.
    Patches (K.3) come from frame["patch_place"] / frame["patch_samples"],
    dots (K.2) from frame["dots"], splines (K.4) from frame["spline_offsets"]
    / frame["spline_points"] / frame["spline_dct"]."""
    ka, pa = _planes(frame["ac"], np.int32)
    kd, pd = _planes(frame["dc"], np.int32)
    out = np.zeros((3, p.ysize, p.xsize))
    pl = frame.get("patch_place")
    n = 0 if pl is None else len(pl)
    pl = np.ascontiguousarray(pl, np.int32) if n else None
    sm = np.ascontiguousarray(frame["patch_samples"], np.int32) if n else None
    dt = frame.get("dots")
    nd = 0 if dt is None else len(dt)
    dt = np.ascontiguousarray(dt, np.int32) if nd else None
    so = frame.get("spline_offsets")
    ns = 0 if so is None else len(so) - 1
    so = np.ascontiguousarray(so, np.int32) if ns else None
    sp = np.ascontiguousarray(frame["spline_points"], np.int32) if ns else None
    sd = np.ascontiguousarray(frame["spline_dct"], np.float32) if ns else None
    with _Field(p, frame):
        _decode_features(p, frame, pa, pd, pl, n, sm, dt, nd, so, ns, sp, sd, out)
    return out


def _decode_features(p, frame, pa, pd, pl, n, sm, dt, nd, so, ns, sp, sd, out):
    _check(lib().orc_decode_features(
        C.byref(p), pa, pd, np.ascontiguousarray(frame["strategy"], np.uint8),
        np.ascontiguousarray(frame["qf"], np.uint8),
        np.ascontiguousarray(frame["sharpness"], np.uint8),
        np.ascontiguousarray(frame["cfl_kx"], np.float32),
        np.ascontiguousarray(frame["cfl_kb"], np.float32),
        pl.ctypes.data if n else None, n, sm.ctypes.data if n else None,
        dt.ctypes.data if nd else None, nd, so.ctypes.data if ns else None, ns,
        sp.ctypes.data if ns else None, sd.ctypes.data if ns else None, out))


def decode_stages(p, frame):
    """Whole path with every intermediate kept (for stage-by-stage comparison).
    Returns dict: recon, epf (list of (out, guide, sigma)), qco (when
    applied), gab, noise (when applied), rgb."""
    res = {"recon": reconstruct(p, frame), "epf": []}
    cur = res["recon"]
    for _ in range(p.epf_iters):
        out, g, s = epf_pass(p, frame, cur, want_debug=True)
        res["epf"].append((out, g, s))
        cur = out
    if p.qco and p.epf_iters > 0:
        cur = qco(p, frame, res["recon"], cur)
        res["qco"] = cur
    if frame.get("patch_place") is not None and len(frame["patch_place"]):
        cur = patches(p, frame["patch_place"], frame["patch_samples"], cur)
        res["patches"] = cur
    if p.gab:
        cur = gaborish(p, cur)
    res["gab"] = cur
    if frame.get("dots") is not None and len(frame["dots"]):
        cur = dots(p, frame["dots"], cur)
        res["dots"] = cur
    if frame.get("spline_offsets") is not None and len(frame["spline_offsets"]) > 1:
        cur = splines(p, frame["spline_offsets"], frame["spline_points"], frame["spline_dct"], cur)
        res["splines"] = cur
    if p.noise:
        cur = noise(p, cur)
        res["noise"] = cur
    res["rgb"] = xyb_to_rgb(p, cur)
    return res


def num_threads():
    return lib().orc_num_threads()
