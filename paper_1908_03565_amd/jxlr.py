"""ctypes binding of libjxlr.so (C ABI in include/jxlr.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
library.  PyTorch provides device memory (tensors) and streams.  Loading fails
loudly when the library has not been built; nothing here falls back to a CPU
implementation.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjxlr.so")

JXLR_OUT_F32, JXLR_OUT_U8_SRGB, JXLR_OUT_U16_SRGB = 0, 1, 2
STATUS = ["ok", "null", "size", "strategy", "align", "quant", "dequant", "param",
          "workspace", "hip", "device_validation"]


class FrameParams(C.Structure):
    _fields_ = [
        ("xsize", C.c_uint32), ("ysize", C.c_uint32),
        ("global_scale", C.c_uint32),
        ("dc_mul", C.c_float * 3),
        ("extra_levels", C.c_int32 * 3),
        ("kx_dc", C.c_float), ("kb_dc", C.c_float),
        ("gab", C.c_int32),
        ("gab_w1", C.c_float * 3), ("gab_w2", C.c_float * 3),
        ("epf_iters", C.c_int32),
        ("epf_weight_min", C.c_float),
        ("epf_scale", C.c_float * 3),
        ("epf_sharp_lut", C.c_float * 8),
        ("epf_range_max", C.c_float), ("epf_range_mul", C.c_float),
        ("epf_quant_mul", C.c_float),
        ("epf_sigma_max", C.c_int32),
        ("epf_sigma_shift", C.c_int32),
        ("opsin_inv", C.c_float * 9),
        ("opsin_bias", C.c_float * 3),
        ("target_nits_div50", C.c_int32),
        ("out_format", C.c_int32),
        ("idct_split", C.c_int32),
        ("dc_smoothing", C.c_int32),
        ("qco", C.c_int32),
        ("qco_interval_mul", C.c_float),
        ("ac_prediction", C.c_int32),
        ("noise", C.c_int32),
        ("noise_lut", C.c_float * 16),
        ("num_patches", C.c_int32),
        ("num_dots", C.c_int32),
        ("dot_colour_quant", C.c_float * 3),
        ("num_splines", C.c_int32),
        ("num_spline_points", C.c_int32),
        ("fuse", C.c_int32),
    ]


class FrameIO(C.Structure):
    _fields_ = [
        ("ac", C.c_void_p * 3), ("ac_stride", C.c_size_t),
        ("dc", C.c_void_p * 3), ("dc_stride", C.c_size_t),
        ("strategy", C.c_void_p), ("qf_minus_1", C.c_void_p), ("sharpness", C.c_void_p),
        ("map_stride", C.c_size_t),
        ("cfl_kx", C.c_void_p), ("cfl_kb", C.c_void_p), ("cfl_stride", C.c_size_t),
        ("out", C.c_void_p * 3), ("out_stride", C.c_size_t),
        ("ac_pred", C.c_void_p),
        ("noise_raw", C.c_void_p),
        ("patch_place", C.c_void_p), ("patch_samples", C.c_void_p),
        ("patch_samples_count", C.c_size_t),
        ("dots", C.c_void_p),
        ("spline_offsets", C.c_void_p),
        ("spline_points", C.c_void_p),
        ("spline_dct", C.c_void_p),
        ("dc_quant", C.c_void_p * 3), ("dc_quant_stride", C.c_size_t),
    ]


class DequantEncoding(C.Structure):
    """jxlr_dequant_encoding (C.6.1)."""
    _fields_ = [
        ("mode", C.c_int32), ("copy_from", C.c_int32),
        ("num_bands", C.c_int32), ("num_ecc_bands", C.c_int32),
        ("dist_bands", (C.c_double * 17) * 3),
        ("ecc_bands", (C.c_double * 8) * 3),
        ("params", (C.c_double * 6) * 3),
        ("afv_weights", (C.c_double * 8) * 3),
    ]


def dequant_encodings(encs):
    """A jxlr_dequant_encoding array from 15 dicts (mode, copy_from,
    num_bands, num_ecc_bands, dist_bands, ecc_bands, params, afv_weights;
    absent keys 0), indexed by transform type."""
    if len(encs) != 15:
        raise ValueError("15 encodings, one per transform type")
    arr = (DequantEncoding * 15)()
    for j, e in enumerate(encs):
        for k in ("mode", "copy_from", "num_bands", "num_ecc_bands"):
            setattr(arr[j], k, int(e.get(k, 0)))
        for k in ("dist_bands", "ecc_bands", "params", "afv_weights"):
            dst = getattr(arr[j], k)
            for c, row in enumerate(e.get(k, [])):
                for i, v in enumerate(row):
                    dst[c][i] = float(v)
    return arr


class BatchPlan(C.Structure):
    _fields_ = [
        ("ws", C.c_void_p), ("ws_bytes", C.c_size_t),
        ("n", C.c_int), ("total_tiles", C.c_int), ("total_regions", C.c_int),
        ("max_epf_iters", C.c_int),
        ("frames_offset", C.c_size_t), ("tile_frame_offset", C.c_size_t),
        ("tile_start_offset", C.c_size_t),
        ("region_start_offset", C.c_size_t),
        ("any_split", C.c_int), ("any_noise", C.c_int),
        ("opt_frames", C.c_int * 9), ("opt_units", C.c_int * 9),
        ("opt_entries_offset", C.c_size_t * 9), ("opt_start_offset", C.c_size_t * 9),
    ]


class LaunchConfig(C.Structure):
    _fields_ = [("grid_info", C.c_int), ("grid_recon", C.c_int), ("grid_epf", C.c_int),
                ("grid_finish", C.c_int), ("order_recon", C.c_int), ("order_epf", C.c_int),
                ("order_finish", C.c_int)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


STAGE_INFO, STAGE_RECON, STAGE_EPF, STAGE_FINISH = 0, 1, 2, 3
(STAGE_PRED, STAGE_QCO, STAGE_PATCHES, STAGE_NOISE, STAGE_GABORISH, STAGE_DOTS,
 STAGE_SPLINES, STAGE_FUSED, STAGE_SEAM) = range(4, 13)


class Jpeg1Params(C.Structure):
    _fields_ = [("xsize", C.c_int32), ("ysize", C.c_int32), ("num_components", C.c_int32),
                ("h_samp", C.c_int32 * 3), ("v_samp", C.c_int32 * 3),
                ("quant", (C.c_int32 * 64) * 3),
                ("gab", C.c_int32), ("gab_code", (C.c_uint8 * 4) * 3)]


def jpeg1_params(j):
    """Jpeg1Params of a synthetic JPEG1 frame dict (workload.jpeg1)."""
    p = Jpeg1Params()
    p.xsize, p.ysize, p.num_components = j["xsize"], j["ysize"], len(j["coef"])
    for c in range(len(j["coef"])):
        p.h_samp[c], p.v_samp[c] = j["hs"][c], j["vs"][c]
        for i, q in enumerate(np.asarray(j["quant"][c]).ravel()):
            p.quant[c][i] = int(q)
    if j.get("gab") is not None:
        p.gab = 1
        for c, code in enumerate(j["gab"]):
            for i, v in enumerate(code):
                p.gab_code[c][i] = int(v)
    return p


class JxlrError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"jxlr {what}: status {status} ({name})")


_LIB = None

# Entry points declared in include/jxlr.h, with their ctypes signatures.
_SIGS = {
    "jxlr_status_string": ([C.c_int], C.c_char_p),
    "jxlr_params_default": ([C.POINTER(FrameParams), C.c_uint32, C.c_uint32], C.c_int),
    "jxlr_create": ([C.POINTER(C.c_void_p), C.c_int, C.c_void_p], C.c_int),
    "jxlr_cfl_from_u8": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p], C.c_int),
    "jxlr_dc_mul_from_header": ([C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(C.c_float)],
                                C.c_int),
    "jxlr_destroy": ([C.c_void_p], None),
    "jxlr_validate_maps_host": ([C.POINTER(FrameParams), C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_size_t], C.c_int),
    "jxlr_workspace_bytes": ([C.POINTER(FrameParams)], C.c_size_t),
    "jxlr_decode": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                     C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_decode_noalloc": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p],
                            C.c_int),
    "jxlr_noalloc_scratch_bytes": ([], C.c_size_t),
    "jxlr_block_info": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                         C.c_void_p], C.c_int),
    "jxlr_reconstruct": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                          C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_epf_pass": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                       C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p],
                      C.c_int),
    "jxlr_ac_prediction": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                            C.c_void_p, C.c_void_p], C.c_int),
    "jxlr_patches": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                      C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_gaborish": ([C.c_void_p, C.POINTER(FrameParams), C.c_void_p, C.c_void_p, C.c_size_t,
                       C.c_void_p], C.c_int),
    "jxlr_dots": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p, C.c_size_t,
                   C.c_void_p], C.c_int),
    "jxlr_spline_scratch_bytes": ([C.POINTER(FrameParams)], C.c_size_t),
    "jxlr_jpeg1_blocks": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
                          C.c_int),
    "jxlr_jpeg1_workspace_bytes": ([C.c_void_p], C.c_size_t),
    "jxlr_jpeg1_idct": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                         C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_jpeg1_gaborish": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                             C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_jpeg1_color": ([C.c_void_p, C.c_void_p, C.c_void_p * 3, C.c_size_t * 3,
                          C.c_void_p * 3, C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_jpeg1_decode": ([C.c_void_p, C.c_void_p, C.c_void_p * 3, C.c_size_t * 3,
                           C.c_void_p * 3, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p],
                          C.c_int),
    "jxlr_splines": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                      C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_noise_channels": ([C.c_void_p, C.POINTER(FrameParams), C.c_void_p, C.c_void_p], C.c_int),
    "jxlr_qco_pass": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                       C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_finish": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                     C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_seam_bytes": ([C.POINTER(FrameParams)], C.c_size_t),
    "jxlr_epf_finish": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO), C.c_void_p,
                         C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_reconstruct_finish": ([C.c_void_p, C.POINTER(FrameParams), C.POINTER(FrameIO),
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_batch_workspace_bytes": ([C.c_int, C.POINTER(FrameParams)], C.c_size_t),
    "jxlr_batch_prepare": ([C.c_void_p, C.c_int, C.POINTER(FrameParams), C.POINTER(FrameIO),
                            C.c_void_p, C.c_size_t, C.POINTER(BatchPlan), C.c_void_p], C.c_int),
    "jxlr_batch_run": ([C.c_void_p, C.POINTER(BatchPlan), C.POINTER(LaunchConfig), C.c_void_p],
                       C.c_int),
    "jxlr_batch_stage": ([C.c_void_p, C.POINTER(BatchPlan), C.c_int, C.c_int, C.c_int, C.c_int,
                          C.c_void_p], C.c_int),
    "jxlr_autotune": ([C.c_void_p, C.POINTER(BatchPlan), C.c_int, C.POINTER(LaunchConfig),
                       C.POINTER(C.c_float), C.c_void_p], C.c_int),
    "jxlr_decode_batch": ([C.c_void_p, C.c_int, C.POINTER(FrameParams), C.POINTER(FrameIO),
                           C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "jxlr_graph_create": ([C.c_void_p, C.POINTER(BatchPlan), C.POINTER(LaunchConfig),
                          C.POINTER(C.c_void_p)], C.c_int),
    "jxlr_graph_launch": ([C.c_void_p, C.c_void_p], C.c_int),
    "jxlr_graph_destroy": ([C.c_void_p], None),
    "jxlr_get_device_status": ([C.c_void_p, C.c_void_p], C.c_int),
}


def lib():
    """Loads libjxlr.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1908_03565_amd/build.py "
                "(or __graft_entry__.build()); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def exported_symbols():
    return list(_SIGS)


def _check(st, what):
    if st != 0:
        raise JxlrError(st, what)


def params(xsize, ysize, **overrides):
    """Frame parameters: the library's defaults, then `overrides`."""
    p = FrameParams()
    _check(lib().jxlr_params_default(C.byref(p), int(xsize), int(ysize)), "params_default")
    for k, v in overrides.items():
        cur = getattr(p, k)
        if isinstance(cur, C.Array):
            vals = list(np.asarray(v).ravel())
            if len(vals) != len(cur):
                raise ValueError(k)
            for i, x in enumerate(vals):
                cur[i] = type(cur[0])(x) if isinstance(cur[0], int) else float(x)
        else:
            setattr(p, k, v)
    return p


def validate_maps_host(p, frame):
    st = np.ascontiguousarray(frame["strategy"], np.uint8)
    qf = np.ascontiguousarray(frame["qf"], np.uint8)
    sh = np.ascontiguousarray(frame["sharpness"], np.uint8) if "sharpness" in frame else None
    return lib().jxlr_validate_maps_host(C.byref(p), st.ctypes.data, qf.ctypes.data,
                                         sh.ctypes.data if sh is not None else None,
                                         st.shape[1])


def cfl_from_u8(x_factor=None, b_factor=None):
    """Annex G: kX, kB (float32 arrays) of u8 XFromY / BFromY values."""
    xf = None if x_factor is None else np.ascontiguousarray(x_factor, np.uint8)
    bf = None if b_factor is None else np.ascontiguousarray(b_factor, np.uint8)
    n = (xf if xf is not None else bf).size
    kx = None if xf is None else np.empty(xf.shape, np.float32)
    kb = None if bf is None else np.empty(bf.shape, np.float32)
    _check(lib().jxlr_cfl_from_u8(None if xf is None else xf.ctypes.data,
                                  None if bf is None else bf.ctypes.data, n,
                                  None if kx is None else kx.ctypes.data,
                                  None if kb is None else kb.ctypes.data), "cfl_from_u8")
    return kx, kb


def dc_mul_from_header(weights=None, global_scale=1, quant_dc=1):
    """C.4.1 DC multipliers (3 floats)."""
    w = None if weights is None else np.ascontiguousarray(weights, np.float32)
    out = (C.c_float * 3)()
    _check(lib().jxlr_dc_mul_from_header(None if w is None else w.ctypes.data, global_scale,
                                         quant_dc, out), "dc_mul_from_header")
    return [float(v) for v in out]


def workspace_bytes(p):
    return lib().jxlr_workspace_bytes(C.byref(p))


def batch_workspace_bytes(ps):
    arr = (FrameParams * len(ps))(*ps)
    return lib().jxlr_batch_workspace_bytes(len(ps), arr)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class DeviceFrame:
    """A frame's input planes resident in device memory (torch tensors)."""

    PLANES = (("ac", np.int32), ("dc", np.int32), ("strategy", np.uint8), ("qf", np.uint8),
              ("sharpness", np.uint8), ("cfl_kx", np.float32), ("cfl_kb", np.float32))

    def __init__(self, frame, device="cuda", non_blocking=False):
        """frame: dict of numpy arrays, or of CPU tensors (pinned ones can be
        copied with non_blocking=True on the current stream; the caller keeps
        them alive until that copy has run)."""
        import torch

        def t(a, dt):
            if isinstance(a, torch.Tensor):
                return a.to(device, non_blocking=non_blocking)
            return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)

        self.xsize, self.ysize = int(frame["xsize"]), int(frame["ysize"])
        self.ac = t(frame["ac"], np.int32)
        self.dc = t(frame["dc"], np.int32)
        self.strategy = t(frame["strategy"], np.uint8)
        self.qf = t(frame["qf"], np.uint8)
        self.sharpness = t(frame["sharpness"], np.uint8)
        self.cfl_kx = t(frame["cfl_kx"], np.float32)
        self.cfl_kb = t(frame["cfl_kb"], np.float32)
        # K.3 patches, if the frame has any
        pl = frame.get("patch_place")
        self.patch_place = t(pl, np.int32) if pl is not None and len(pl) else None
        self.patch_samples = (t(frame["patch_samples"], np.int32)
                              if self.patch_place is not None else None)
        dt = frame.get("dots")
        self.dots = t(dt, np.int32) if dt is not None and len(dt) else None
        # C.5.2 DcQuantField, if the frame has one
        dq = frame.get("dc_quant")
        self.dc_quant = t(dq, np.float32) if dq is not None else None
        # K.4 splines, if the frame has any
        so = frame.get("spline_offsets")
        has = so is not None and len(so) > 1
        self.spline_offsets = t(so, np.int32) if has else None
        self.spline_points = t(frame["spline_points"], np.int32) if has else None
        self.spline_dct = t(frame["spline_dct"], np.float32) if has else None

    def clone(self):
        """A copy in distinct device memory."""
        c = DeviceFrame.__new__(DeviceFrame)
        c.xsize, c.ysize = self.xsize, self.ysize
        for k in ("ac", "dc", "strategy", "qf", "sharpness", "cfl_kx", "cfl_kb"):
            setattr(c, k, getattr(self, k).clone())
        c.patch_place = None if self.patch_place is None else self.patch_place.clone()
        c.patch_samples = None if self.patch_samples is None else self.patch_samples.clone()
        c.dots = None if self.dots is None else self.dots.clone()
        dq = getattr(self, "dc_quant", None)
        c.dc_quant = None if dq is None else dq.clone()
        for k in ("spline_offsets", "spline_points", "spline_dct"):
            v = getattr(self, k, None)
            setattr(c, k, None if v is None else v.clone())
        return c

    def io(self, out=None, ac_pred=None, noise_raw=None):
        io = FrameIO()
        io.ac_pred = ac_pred.data_ptr() if ac_pred is not None else None
        io.noise_raw = noise_raw.data_ptr() if noise_raw is not None else None
        if getattr(self, "patch_place", None) is not None:
            io.patch_place = self.patch_place.data_ptr()
            io.patch_samples = self.patch_samples.data_ptr()
            io.patch_samples_count = self.patch_samples.numel()
        if getattr(self, "dots", None) is not None:
            io.dots = self.dots.data_ptr()
        if getattr(self, "dc_quant", None) is not None:
            for c in range(3):
                io.dc_quant[c] = self.dc_quant[c].data_ptr()
            io.dc_quant_stride = self.dc_quant.shape[2]
        if getattr(self, "spline_offsets", None) is not None:
            io.spline_offsets = self.spline_offsets.data_ptr()
            io.spline_points = self.spline_points.data_ptr()
            io.spline_dct = self.spline_dct.data_ptr()
        for c in range(3):
            io.ac[c] = self.ac[c].data_ptr()
            io.dc[c] = self.dc[c].data_ptr()
        io.ac_stride = self.ac.shape[2]
        io.dc_stride = self.dc.shape[2]
        io.strategy = self.strategy.data_ptr()
        io.qf_minus_1 = self.qf.data_ptr()
        io.sharpness = self.sharpness.data_ptr()
        io.map_stride = self.strategy.shape[1]
        io.cfl_kx = self.cfl_kx.data_ptr()
        io.cfl_kb = self.cfl_kb.data_ptr()
        io.cfl_stride = self.cfl_kx.shape[1]
        if out is not None:
            for c in range(3):
                io.out[c] = out[c].data_ptr()
            io.out_stride = out.shape[2]
        return io


_OUT_DTYPE = {JXLR_OUT_F32: "float32", JXLR_OUT_U8_SRGB: "uint8", JXLR_OUT_U16_SRGB: "uint16"}


class Context:
    """A jxlr context on one HIP device."""

    def __init__(self, device=0, dq_enc=None):
        """dq_enc: None (the C.6.1.1 defaults) or 15 encoding dicts, one per
        transform type (see dequant_encodings)."""
        import torch
        # torch's HIP runtime is initialised first: the buffers and streams
        # this binding hands to the library are torch's, and a runtime that
        # the library brought up first can leave torch without devices
        torch.cuda.init()
        self.device = device
        h = C.c_void_p()
        enc = None if dq_enc is None else dequant_encodings(dq_enc)
        _check(lib().jxlr_create(C.byref(h), int(device), None if enc is None else C.cast(enc, C.c_void_p)),
               "create")
        self.handle = h

    def close(self):
        if self.handle:
            lib().jxlr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- allocation helpers (torch device memory) ---
    # --- JPEG1 direct rasterization (M.6) ---
    def jpeg1_upload(self, j):
        """Device copies of a synthetic JPEG1 frame's coefficient planes."""
        import torch
        return [torch.from_numpy(np.ascontiguousarray(c, np.int32)).to(f"cuda:{self.device}")
                for c in j["coef"]]

    def jpeg1_empty_rgb(self, jp):
        import torch
        return torch.empty((3, jp.ysize, jp.xsize), dtype=torch.float32,
                           device=f"cuda:{self.device}")

    def jpeg1_workspace(self, jp):
        import torch
        return torch.empty(max(1, lib().jxlr_jpeg1_workspace_bytes(C.byref(jp))),
                           dtype=torch.uint8, device=f"cuda:{self.device}")

    def jpeg1_idct(self, jp, c, coef, pix, stream=None):
        _check(lib().jxlr_jpeg1_idct(self.handle, C.byref(jp), c, coef.data_ptr(), coef.shape[1],
                                     pix.data_ptr(), pix.shape[1], _stream_handle(stream)),
               "jpeg1_idct")

    def jpeg1_gaborish(self, jp, c, pix_in, pix_out, stream=None):
        _check(lib().jxlr_jpeg1_gaborish(self.handle, C.byref(jp), c, pix_in.data_ptr(),
                                         pix_in.shape[1], pix_out.data_ptr(), pix_out.shape[1],
                                         _stream_handle(stream)), "jpeg1_gaborish")

    def jpeg1_color(self, jp, pix, rgb, stream=None):
        ptr = (C.c_void_p * 3)(*([q.data_ptr() for q in pix] + [None] * (3 - len(pix))))
        strides = (C.c_size_t * 3)(*([q.shape[1] for q in pix] + [0] * (3 - len(pix))))
        out = (C.c_void_p * 3)(*[rgb[c].data_ptr() for c in range(3)])
        _check(lib().jxlr_jpeg1_color(self.handle, C.byref(jp), ptr, strides, out, rgb.shape[2],
                                      _stream_handle(stream)), "jpeg1_color")

    def jpeg1_decode(self, jp, coefs, rgb, ws, stream=None):
        ptr = (C.c_void_p * 3)(*([q.data_ptr() for q in coefs] + [None] * (3 - len(coefs))))
        strides = (C.c_size_t * 3)(*([q.shape[1] for q in coefs] + [0] * (3 - len(coefs))))
        out = (C.c_void_p * 3)(*[rgb[c].data_ptr() for c in range(3)])
        _check(lib().jxlr_jpeg1_decode(self.handle, C.byref(jp), ptr, strides, out, rgb.shape[2],
                                       ws.data_ptr(), ws.numel(), _stream_handle(stream)),
               "jpeg1_decode")

    def empty_xyb(self, p):
        import torch
        return torch.empty((3, p.ysize, p.xsize), dtype=torch.float32, device=f"cuda:{self.device}")

    def empty_out(self, p):
        import torch
        dt = getattr(torch, _OUT_DTYPE[p.out_format])
        return torch.empty((3, p.ysize, p.xsize), dtype=dt, device=f"cuda:{self.device}")

    def empty_info(self, p):
        import torch
        return torch.empty(((p.ysize + 7) // 8, (p.xsize + 7) // 8), dtype=torch.uint8,
                           device=f"cuda:{self.device}")

    def workspace(self, p):
        import torch
        return torch.empty(workspace_bytes(p), dtype=torch.uint8, device=f"cuda:{self.device}")

    # --- entry points ---
    def block_info(self, p, df, info, stream=None):
        _check(lib().jxlr_block_info(self.handle, C.byref(p), C.byref(df.io()), info.data_ptr(),
                                     _stream_handle(stream)), "block_info")

    def empty_pred(self, p):
        import torch
        Hb, Wb = (p.ysize + 7) // 8, (p.xsize + 7) // 8
        return torch.empty((3, 2 * Hb, 2 * Wb), dtype=torch.float32, device=f"cuda:{self.device}")

    def ac_prediction(self, p, df, info, pred, stream=None):
        _check(lib().jxlr_ac_prediction(self.handle, C.byref(p), C.byref(df.io()), info.data_ptr(),
                                        pred.data_ptr(), _stream_handle(stream)), "ac_prediction")

    def reconstruct(self, p, df, info, xyb, stream=None, pred=None):
        _check(lib().jxlr_reconstruct(self.handle, C.byref(p), C.byref(df.io(ac_pred=pred)),
                                      info.data_ptr(), xyb.data_ptr(), xyb.shape[2],
                                      _stream_handle(stream)),
               "reconstruct")

    def epf_pass(self, p, df, info, xyb_in, xyb_out, guide=None, sigma=None, stream=None):
        _check(lib().jxlr_epf_pass(self.handle, C.byref(p), C.byref(df.io()), info.data_ptr(),
                                   xyb_in.data_ptr(), xyb_out.data_ptr(), xyb_in.shape[2],
                                   guide.data_ptr() if guide is not None else None,
                                   sigma.data_ptr() if sigma is not None else None,
                                   _stream_handle(stream)), "epf_pass")

    def patches(self, p, df, xyb, stream=None):
        _check(lib().jxlr_patches(self.handle, C.byref(p), C.byref(df.io()), xyb.data_ptr(),
                                  xyb.shape[2], _stream_handle(stream)), "patches")

    def gaborish(self, p, xyb_in, xyb_out, stream=None):
        _check(lib().jxlr_gaborish(self.handle, C.byref(p), xyb_in.data_ptr(), xyb_out.data_ptr(),
                                   xyb_in.shape[2], _stream_handle(stream)), "gaborish")

    def dots(self, p, df, xyb, stream=None):
        _check(lib().jxlr_dots(self.handle, C.byref(p), C.byref(df.io()), xyb.data_ptr(),
                               xyb.shape[2], _stream_handle(stream)), "dots")

    def spline_scratch(self, p):
        import torch
        return torch.empty(max(1, lib().jxlr_spline_scratch_bytes(C.byref(p))), dtype=torch.uint8,
                           device=f"cuda:{self.device}")

    def splines(self, p, df, xyb, scratch=None, stream=None):
        if scratch is None:
            scratch = self.spline_scratch(p)
        _check(lib().jxlr_splines(self.handle, C.byref(p), C.byref(df.io()), xyb.data_ptr(),
                                  xyb.shape[2], scratch.data_ptr(), scratch.numel(),
                                  _stream_handle(stream)), "splines")

    def noise_channels(self, p, raw, stream=None):
        _check(lib().jxlr_noise_channels(self.handle, C.byref(p), raw.data_ptr(),
                                         _stream_handle(stream)), "noise_channels")

    def finish(self, p, df, xyb, out, stream=None, noise_raw=None):
        _check(lib().jxlr_finish(self.handle, C.byref(p), C.byref(df.io(out, noise_raw=noise_raw)),
                                 xyb.data_ptr(), xyb.shape[2], _stream_handle(stream)), "finish")

    def seam_buffer(self, p):
        import torch
        return torch.empty(max(1, lib().jxlr_seam_bytes(C.byref(p))), dtype=torch.uint8,
                           device=f"cuda:{self.device}")

    def reconstruct_finish(self, p, df, info, out, seam=None, stream=None, pred=None):
        """The reconstruction and the finish without an XYB frame (frames with
        no EPF pass, patches, dots, splines or noise)."""
        if seam is None:
            seam = self.seam_buffer(p)
        _check(lib().jxlr_reconstruct_finish(self.handle, C.byref(p),
                                             C.byref(df.io(out, ac_pred=pred)), info.data_ptr(),
                                             seam.data_ptr(), seam.numel(),
                                             _stream_handle(stream)), "reconstruct_finish")

    def epf_finish(self, p, df, info, xyb_in, out, seam=None, stream=None):
        """The last EPF pass and the finish without storing the pass's output
        (frames with nothing between the two)."""
        if seam is None:
            seam = self.seam_buffer(p)
        _check(lib().jxlr_epf_finish(self.handle, C.byref(p), C.byref(df.io(out)),
                                     info.data_ptr(), xyb_in.data_ptr(), xyb_in.shape[2],
                                     seam.data_ptr(), seam.numel(), _stream_handle(stream)),
               "epf_finish")

    def qco_pass(self, p, df, info, xyb_orig, xyb_io, stream=None):
        _check(lib().jxlr_qco_pass(self.handle, C.byref(p), C.byref(df.io()), info.data_ptr(),
                                   xyb_orig.data_ptr(), xyb_io.data_ptr(), xyb_io.shape[2],
                                   _stream_handle(stream)), "qco_pass")

    def decode(self, p, df, out, ws, stream=None, io=None):
        io = df.io(out) if io is None else io
        _check(lib().jxlr_decode(self.handle, C.byref(p), C.byref(io), ws.data_ptr(),
                                 ws.numel(), _stream_handle(stream)), "decode")

    def decode_noalloc(self, p, df, out, stream=None, io=None):
        """jxlr_decode on the library's own per-device scratch array."""
        io = df.io(out) if io is None else io
        _check(lib().jxlr_decode_noalloc(self.handle, C.byref(p), C.byref(io),
                                         _stream_handle(stream)), "decode_noalloc")

    # --- batches ---
    def batch_workspace(self, ps):
        import torch
        n = batch_workspace_bytes(ps)
        if n == 0:
            raise JxlrError(7, "batch_workspace_bytes")
        return torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")

    def batch_prepare(self, ps, ios, ws, stream=None):
        """ps, ios: lists of FrameParams / FrameIO; ws: device workspace tensor.
        The descriptors are written in order on `stream` (default: the current
        stream), which the call synchronizes.  Returns the plan."""
        n = len(ps)
        parr = (FrameParams * n)(*ps)
        iarr = (FrameIO * n)(*ios)
        plan = BatchPlan()
        _check(lib().jxlr_batch_prepare(self.handle, n, parr, iarr, ws.data_ptr(), ws.numel(),
                                        C.byref(plan), _stream_handle(stream)), "batch_prepare")
        return plan

    def batch_run(self, plan, cfg=None, stream=None):
        _check(lib().jxlr_batch_run(self.handle, C.byref(plan),
                                    C.byref(cfg) if cfg is not None else None,
                                    _stream_handle(stream)), "batch_run")

    def batch_stage(self, plan, stage, grid=0, order=0, epf_pass=0, stream=None):
        _check(lib().jxlr_batch_stage(self.handle, C.byref(plan), stage, grid, order, epf_pass,
                                      _stream_handle(stream)), "batch_stage")

    def autotune(self, plan, reps=5, stream=None):
        """Returns (LaunchConfig, tuned ms per run)."""
        cfg = LaunchConfig()
        ms = C.c_float()
        _check(lib().jxlr_autotune(self.handle, C.byref(plan), reps, C.byref(cfg), C.byref(ms),
                                   _stream_handle(stream)), "autotune")
        return cfg, float(ms.value)

    def decode_batch(self, ps, ios, ws, stream=None):
        n = len(ps)
        parr = (FrameParams * n)(*ps)
        iarr = (FrameIO * n)(*ios)
        _check(lib().jxlr_decode_batch(self.handle, n, parr, iarr, ws.data_ptr(), ws.numel(),
                                       _stream_handle(stream)), "decode_batch")

    def graph(self, plan, cfg=None):
        return Graph(self, plan, cfg)

    def device_status(self, stream=None):
        return lib().jxlr_get_device_status(self.handle, _stream_handle(stream))


class Graph:
    """A prepared batch captured into a HIP graph (jxlr_graph_*)."""

    def __init__(self, ctx, plan, cfg=None):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().jxlr_graph_create(ctx.handle, C.byref(plan),
                                       C.byref(cfg) if cfg is not None else None, C.byref(h)),
               "graph_create")
        self.handle = h

    def launch(self, stream=None):
        _check(lib().jxlr_graph_launch(self.handle, _stream_handle(stream)), "graph_launch")

    def close(self):
        if self.handle:
            lib().jxlr_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pin_frame(frame):
    """A copy of a frame dict whose planes are pinned CPU tensors (for
    asynchronous uploads)."""
    import torch
    out = dict(frame)
    for k, dt in DeviceFrame.PLANES:
        a = np.ascontiguousarray(frame[k], dtype=dt)
        t = torch.empty(a.shape, dtype=getattr(torch, np.dtype(dt).name), pin_memory=True)
        t.numpy()[...] = a
        out[k] = t
    return out
