"""GPU parity on DctSelect maps that mix transform types inside each 32x32
region.  C.5.4 allows any tiling by naturally aligned varblocks; here every
region is tiled in raster order by types drawn among those that fit
(workload.mixed_tiling_map).  This exercises the block-info raster scan, the
per-varblock (owner) paths of the reconstruction, the per-varblock sigma of
the EPF and, in the split form, the boundary between matrix-core regions
(one type over the whole region) and binary32 ones.

Gates: XYB reconstruction against the oracle within the relative bound of
the plain parity tests; end to end, [0,1]-scaled linear RGB within 1e-4
(plain) or 1e-3 (split) outside EPF flip-affected pixels, per transform type.
DCT32x8 and DCT8x32 are left out of the end-to-end frames: their default
B-channel tables turn this recipe's coefficients into samples hundreds of
times the XYB range, where an absolute RGB gate says nothing; they are in the
reconstruction tests, which use the relative XYB bound.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03565_amd import workload as wl
from tests import parity as P

pytestmark = pytest.mark.gpu

XYB_TOL = 4e-6
SPLIT_TOL = 1e-3
MIX13 = [t for t in wl.ALL_TYPES if t not in (wl.DCT32X8, wl.DCT8X32)]


@pytest.fixture(scope="module")
def ctx():
    from paper_1908_03565_amd import jxlr as J
    return J.Context(0)


def _mixed_regions(smap):
    Hb, Wb = smap.shape
    n = 0
    for ry in range(0, Hb - 3, 4):
        for rx in range(0, Wb - 3, 4):
            r = smap[ry:ry + 4, rx:rx + 4]
            n += int(r.min() != r.max())
    return n


def _run(ctx, f, split):
    from paper_1908_03565_amd import jxlr as J
    p = J.params(f["xsize"], f["ysize"], out_format=f["out_format"], idct_split=split,
                 **f["params"])
    assert J.validate_maps_host(p, f) == 0
    return p, P.gpu_stages(ctx, p, J.DeviceFrame(f))


def _xyb_per_type(f, gpu, ref):
    H, W = ref.shape[1:]
    types = np.kron(f["strategy"], np.ones((8, 8), np.uint8))[:H, :W]
    e = np.abs(gpu - ref).max(axis=0)
    return {int(t): float(e[types == t].max()) for t in np.unique(types)}


@pytest.mark.parametrize("W,H,seed", [(200, 136, 300), (521, 267, 301), (64, 64, 303)])
def test_mixed_regions_reconstruction_all_types(ctx, W, H, seed):
    f = wl.frame(W, H, seed=seed, tiling="mixed", epf_iters=0)
    assert _mixed_regions(f["strategy"]) > 0 or W * H <= 64 * 64
    q = O.params(W, H, **f["params"])
    ref = O.reconstruct(q, f)
    scale = np.maximum(1.0, np.abs(ref).max(axis=(1, 2)) / 8.0)
    for split in (0, 1):
        _, g = _run(ctx, f, split)
        err = np.abs(g["recon"] - ref).max(axis=(1, 2))
        print(f"{W}x{H} split={split}: XYB err {err} (scale {scale}); per type "
              f"{_xyb_per_type(f, g['recon'], ref)}")
        tol = XYB_TOL if split == 0 else 1e-4
        assert np.all(err <= tol * scale), err


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("W,H,seed", [(2048, 2048, 302), (1001, 603, 304)])
def test_mixed_regions_end_to_end(ctx, W, H, seed, split):
    f = wl.frame(W, H, seed=seed, choices=MIX13, tiling="mixed", epf_iters=2)
    n_mixed = _mixed_regions(f["strategy"])
    assert n_mixed > 0
    q = O.params(W, H, **f["params"])
    orc = O.decode_stages(q, f)
    p, g = _run(ctx, f, split)
    cmp = P.compare_rgb(p, g, orc)
    per = P.max_err_by_type(f, g, orc, cmp["mask"])
    tol = P.RGB_TOL if split == 0 else SPLIT_TOL
    print(f"mixed {W}x{H} split={split}: {n_mixed} mixed regions; max err {cmp['max_err']:.3g} "
          f"(affected {cmp['affected']} of {cmp['pixels']}, {cmp['passes']}, inside "
          f"{cmp['max_err_affected']:.3g}); per type {per}")
    assert cmp["max_err"] <= tol
    assert max(per.values()) <= tol
    assert set(per) == set(np.unique(f["strategy"]).tolist())
    assert cmp["affected"] <= 0.02 * cmp["pixels"]
