"""Seeded synthetic inputs for VarDCT reconstruction.

This module draws entropy-decoded inputs (quantized coefficient planes, DC
planes, DctSelect, quant field, sharpness and chroma-from-luma maps) and the
frame-parameter overrides of each workload.  It holds none of the method's
arithmetic: both the GPU path and the FP64 oracle consume its arrays as they
are.  Only numpy is imported.

Workloads (the frame shapes and value distributions stand in for decoded
JPEG XL codestreams; no codestream or image data is involved):
  c1      256x256, every varblock DCT8x8, quant field 8, CfL 0, Gaborish on,
          EPF off, seed 0
  c2      2048x2048, DctSelect drawn per 32x32 region from ten transform types,
          quant field U{1..32} per varblock, CfL U[-1,1] per 64x64 tile,
          Gaborish on, EPF 2 passes, seed 2
  c3      4096x4096, half of the 32x32 regions DCT32x32, the rest as c2, seed 3
  c4      a batch of 64 frames, sides log-uniform in [256, 3072] rounded to 8,
          EPF 1 pass, 8-bit sRGB output, seed 4
  small   the c2 recipe at a size the oracle finishes in seconds
  c5      serving requests: sides log-uniform in [64, 4096] rounded to 8, 30%
          16-bit / 70% 8-bit sRGB output, EPF passes U{0..3}, cut at 64-pixel
          aligned offsets out of one 4096x4096 frame of the c2 recipe (seed 5)
          with Poisson arrivals at 200 per second (seed 5)
"""
import math

import numpy as np

# Transform types by their C.5.4 numbers.
DCT8, IDENTITY, DCT2, DCT4, DCT16, DCT32 = 0, 1, 2, 3, 4, 5
DCT16X8, DCT8X16, DCT32X8, DCT8X32, DCT32X16, DCT16X32 = 6, 7, 8, 9, 10, 11
DCT4X8, DCT8X4, AFV = 12, 13, 14

# Varblock size in 8x8 blocks, (columns, rows), of each transform type.
BLOCKS = {0: (1, 1), 1: (1, 1), 2: (1, 1), 3: (1, 1), 4: (2, 2), 5: (4, 4),
          6: (2, 1), 7: (1, 2), 8: (4, 1), 9: (1, 4), 10: (4, 2), 11: (2, 4),
          12: (1, 1), 13: (1, 1), 14: (1, 1)}

# The ten transform types the mixed workloads draw from.
MIXED = [DCT8, DCT4, DCT2, IDENTITY, DCT16, DCT32, DCT8X16, DCT16X8, DCT16X32, DCT32X16]
# Every C.5.4 type (test frames beyond the workloads).
ALL_TYPES = list(range(15))

# Frame-parameter overrides common to every workload: global_scale = 65536 so
# that AcMul = 1 / QF, in [1/32, 1] for QF in [1, 32]; DC multipliers that give
# XYB DC extents of about +-0.03 (X) and +-0.5 (Y, B) for DC values in
# [-512, 512].  The coefficient distributions are fixed by the workload
# definitions; these two scale factors are free, and are chosen so that linear
# RGB stays within a few times the sRGB range (99.9% of samples within
# [-3.2, 3.2] on the [0,1] scale at 2048x2048).
BASE_PARAMS = dict(global_scale=65536, dc_mul=(2.0 ** -14, 2.0 ** -10, 2.0 ** -10),
                   extra_levels=(0, 0, 0))


_BX = np.array([BLOCKS[s][0] for s in range(len(BLOCKS))], np.int32)
_BY = np.array([BLOCKS[s][1] for s in range(len(BLOCKS))], np.int32)


def _fits(s, wb, hb):
    cx, cy = BLOCKS[s]
    return wb % cx == 0 and hb % cy == 0


def strategy_map(rng, Wb, Hb, choices, p_dct32=None):
    """DctSelect per 32x32 region (4x4 blocks): one transform type per region,
    tiled with its varblocks.  Regions clipped by the frame edge draw among the
    types whose varblocks tile the clipped region.  Every block of a varblock
    holds the type (only the top-left entry is read)."""
    smap = np.zeros((Hb, Wb), np.uint8)
    for ry in range(0, Hb, 4):
        for rx in range(0, Wb, 4):
            wb, hb = min(4, Wb - rx), min(4, Hb - ry)
            ok = [s for s in choices if _fits(s, wb, hb)]
            if p_dct32 is not None and _fits(DCT32, wb, hb) and rng.random() < p_dct32:
                s = DCT32
            else:
                pool = ok if p_dct32 is None else [s for s in ok if s != DCT32] or ok
                s = pool[rng.integers(len(pool))] if pool else DCT8
            smap[ry:ry + hb, rx:rx + wb] = s
    return smap


def mixed_tiling_map(rng, Wb, Hb, choices=None):
    """DctSelect with several transform types inside each 32x32 region: the
    region's blocks are visited in raster order (the order of C.5.4) and each
    one not yet covered starts a varblock of a type drawn uniformly among
    `choices` (default: all fifteen) whose varblock is naturally aligned there,
    stays inside the region and the frame, and overlaps no earlier varblock.
    Every block of a varblock holds its type."""
    choices = ALL_TYPES if choices is None else list(choices)
    smap = np.zeros((Hb, Wb), np.uint8)
    for ry in range(0, Hb, 4):
        for rx in range(0, Wb, 4):
            nbx, nby = min(4, Wb - rx), min(4, Hb - ry)
            covered = np.zeros((nby, nbx), bool)
            for by in range(nby):
                for bx in range(nbx):
                    if covered[by, bx]:
                        continue
                    ok = []
                    for s in choices:
                        cx, cy = BLOCKS[s]
                        if bx % cx or by % cy or bx + cx > nbx or by + cy > nby:
                            continue
                        if covered[by:by + cy, bx:bx + cx].any():
                            continue
                        ok.append(s)
                    s = ok[rng.integers(len(ok))] if ok else DCT8
                    cx, cy = BLOCKS[s]
                    covered[by:by + cy, bx:bx + cx] = True
                    smap[ry + by:ry + by + cy, rx + bx:rx + bx + cx] = s
    return smap


def _varblock_geometry(smap):
    """Per coefficient position: (x, y) inside its varblock and the varblock
    size in pixels, for a map produced by strategy_map."""
    Hb, Wb = smap.shape
    cx = np.vectorize(lambda s: BLOCKS[int(s)][0])(smap).astype(np.int32)
    cy = np.vectorize(lambda s: BLOCKS[int(s)][1])(smap).astype(np.int32)
    bxs = np.arange(Wb)[None, :]
    bys = np.arange(Hb)[:, None]
    # Varblocks are naturally aligned, so a block's offset inside its varblock
    # is its index modulo the varblock size (in blocks).
    offx = (bxs % cx)
    offy = (bys % cy)
    px = np.arange(8 * Wb)
    py = np.arange(8 * Hb)
    B = lambda a: np.repeat(np.repeat(a, 8, axis=0), 8, axis=1)
    xin = B(offx) * 8 + (px[None, :] % 8)
    yin = B(offy) * 8 + (py[:, None] % 8)
    return xin, yin, B(cx) * 8, B(cy) * 8


def frame(W, H, seed, choices=None, p_dct32=None, qf_const=None, cfl_zero=False,
          epf_iters=2, gab=1, out_format=0, name="frame", tiling="region"):
    """One synthetic frame as a dict of numpy arrays plus parameter overrides.
    tiling: "region" draws one transform type per 32x32 region
    (strategy_map), "mixed" mixes types inside each region
    (mixed_tiling_map over `choices`, default all fifteen)."""
    rng = np.random.default_rng(seed)
    Wb, Hb = (W + 7) // 8, (H + 7) // 8
    if tiling == "mixed":
        smap = mixed_tiling_map(rng, Wb, Hb, choices)
    else:
        choices = MIXED if choices is None else choices
        smap = strategy_map(rng, Wb, Hb, choices, p_dct32)

    # DC: uniform integers in [-512, 512] per block and channel.
    dc = rng.integers(-512, 513, size=(3, Hb, Wb), dtype=np.int64).astype(np.int32)

    # AC: Laplacian, scale 4 at the lowest AC frequency falling to 0.5 at the
    # highest of an 8x8 block: b = max(0.5, 4 * 8^(-(r - 1) / 13)) with
    # r = 8x/bx + 8y/by; rounded half away from zero; the LLF corner is 0.
    xin, yin, bxp, byp = _varblock_geometry(smap)
    r = 8.0 * xin / bxp + 8.0 * yin / byp
    b = np.maximum(0.5, 4.0 * 8.0 ** (-(r - 1.0) / 13.0))
    llf = (xin < bxp // 8) & (yin < byp // 8)
    ac = np.empty((3, 8 * Hb, 8 * Wb), np.int32)
    for c in range(3):
        v = rng.laplace(0.0, 1.0, size=b.shape) * b
        q = np.sign(v) * np.floor(np.abs(v) + 0.5)
        q[llf] = 0
        ac[c] = q.astype(np.int32)

    # Quant field (dv = QF - 1): per 8x8 block, then every block of a varblock
    # takes the value of its top-left block.
    if qf_const is not None:
        qf = np.full((Hb, Wb), qf_const - 1, np.uint8)
    else:
        raw = rng.integers(1, 33, size=(Hb, Wb)) - 1
        cxb = np.vectorize(lambda s: BLOCKS[int(s)][0])(smap)
        cyb = np.vectorize(lambda s: BLOCKS[int(s)][1])(smap)
        ty = (np.arange(Hb)[:, None] // cyb) * cyb
        tx = (np.arange(Wb)[None, :] // cxb) * cxb
        qf = raw[ty, tx].astype(np.uint8)

    sharp = rng.integers(0, 8, size=(Hb, Wb)).astype(np.uint8)

    Wt, Ht = (W + 63) // 64, (H + 63) // 64
    if cfl_zero:
        kx = np.zeros((Ht, Wt), np.float32)
        kb = np.zeros((Ht, Wt), np.float32)
        dc_cfl = dict(kx_dc=0.0, kb_dc=0.0)
    else:
        kx = rng.uniform(-1.0, 1.0, size=(Ht, Wt)).astype(np.float32)
        kb = rng.uniform(-1.0, 1.0, size=(Ht, Wt)).astype(np.float32)
        dc_cfl = dict(kx_dc=0.0, kb_dc=0.935669)  # x/b_factor_dc = 128

    params = dict(BASE_PARAMS)
    params.update(dc_cfl)
    params.update(epf_iters=epf_iters, gab=gab)
    return dict(name=name, xsize=W, ysize=H, ac=ac, dc=dc, strategy=smap, qf=qf,
                sharpness=sharp, cfl_kx=kx, cfl_kb=kb, params=params,
                out_format=out_format)


# C.6.1 encoding modes and the mode each transform type's default encoding
# (C.6.1.1) is written in.
DQ_LIBRARY, DQ_IDENTITY, DQ_DCT2, DQ_DCT4, DQ_DCT4X8, DQ_AFV, DQ_DCT, DQ_COPY = range(8)
DEFAULT_MODE = {0: DQ_DCT, 1: DQ_IDENTITY, 2: DQ_DCT2, 3: DQ_DCT4, 4: DQ_DCT, 5: DQ_DCT,
                6: DQ_DCT, 7: DQ_DCT, 8: DQ_DCT, 9: DQ_DCT, 10: DQ_DCT, 11: DQ_DCT,
                12: DQ_DCT4X8, 13: DQ_DCT4X8, 14: DQ_AFV}


def _is64(s):
    return BLOCKS[s] == (1, 1)


# Weight scale per transform type and channel for synthetic encodings:
# about the first distance band of the type's default encoding (C.6.1.1),
# and for the types whose numerators are 1 (Identity, DCT2, AFV) about the
# bulk of Identity's default weights.  Every mode's parameters for type s
# are drawn around WEIGHT_SCALE[s], so that the decoded samples stay in the
# range the default matrices give.
WEIGHT_SCALE = {0: (5.0, 1.1, 1.0), 1: (220.0, 30.0, 9.0), 2: (220.0, 30.0, 9.0),
                3: (32.0, 6.0, 4.0), 4: (3.2, 0.78, 0.22), 5: (0.48, 0.22, 0.12),
                6: (5.0, 1.0, 0.35), 7: (5.0, 1.0, 0.35), 8: (0.9, 0.36, 0.25),
                9: (0.9, 0.36, 0.25), 10: (1.13, 0.39, 0.1), 11: (1.13, 0.39, 0.1),
                12: (17.0, 4.6, 0.8), 13: (17.0, 4.6, 0.8), 14: (220.0, 30.0, 9.0)}


def _bands(rng, scale, nmax=17):
    """Random distance and eccentricity bands: the first distance band of
    each channel is the type's weight scale times U[0.5, 2]; later bands move
    it by factors mostly below 1 towards high frequencies, their product
    between about 1/35 and 2 whatever the band count (the defaults' products
    span 1/10 to 1/70)."""
    nb = int(rng.integers(2, nmax + 1))
    ne = int(rng.integers(1, 9))
    a = 4.0 / (nb - 1)
    db = [[b * rng.uniform(0.5, 2.0)] + list(rng.uniform(-a, 0.2 * a, nb - 1)) for b in scale]
    eb = [list(rng.uniform(-0.3, 0.3, ne) / ne) for _ in range(3)]
    return dict(num_bands=nb, num_ecc_bands=ne, dist_bands=db, ecc_bands=eb)


def dequant_encoding(rng, s, mode, copy_from=0):
    """One synthetic C.6.1 encoding of mode `mode` for transform type s, its
    parameters drawn around the type's weight scale in the proportions the
    draft's defaults of that mode show."""
    e = {"mode": mode}
    sc = WEIGHT_SCALE[s]
    if mode == DQ_COPY:
        e["copy_from"] = copy_from
    elif mode == DQ_IDENTITY:
        e["params"] = [[w, w * rng.uniform(1, 30), w * rng.uniform(1, 20)]
                       for w in (b * rng.uniform(0.5, 2.0) for b in sc)]
    elif mode == DQ_DCT2:
        e["params"] = [list(b * rng.uniform(0.5, 2.0) * np.array([12, 8, 4, 2, 1.5, 1]) *
                            rng.uniform(0.7, 1.3, 6)) for b in sc]
    elif mode in (DQ_DCT4, DQ_DCT4X8, DQ_DCT):
        e.update(_bands(rng, sc))
        e["params"] = [list(rng.uniform(0.5, 1.5, 2)) for _ in range(3)]
    elif mode == DQ_AFV:
        e["afv_weights"] = [list(b * rng.uniform(0.5, 2.0, 4) * np.array([19, 0.7, 1.3, 0.7])) +
                            [b * rng.uniform(0.5, 2.0)] + list(rng.uniform(-2.5, 0.2, 3)) for b in sc]
        e["params"] = [list(rng.uniform(0.5, 1.5, 2)) for _ in range(3)]
    return e


def dequant_encodings(seed, modes=None):
    """Fifteen synthetic C.6.1 encodings (one per transform type, already
    read from a stream).  Each type draws a mode among `modes` (default all
    eight) that is valid for its matrix: the 64-entry modes only for the
    7 types with 64 coefficients, Copy only of an earlier matrix whose
    encoding (Library resolved to its default mode) suits this one and
    whose numerators are of the same kind (1 for Identity, DCT2 and AFV,
    DCT scale factors for the others), so that values stay in range."""
    rng = np.random.default_rng(seed)
    modes = list(range(8)) if modes is None else list(modes)
    unit = (1, 2, 14)
    encs, resolved = [], []

    def sources(s):
        return [j for j in range(s) if (_is64(s) or resolved[j] == DQ_DCT)
                and ((j in unit) == (s in unit))]

    for s in range(15):
        ok = []
        for m in modes:
            if m in (DQ_IDENTITY, DQ_DCT2, DQ_DCT4, DQ_DCT4X8, DQ_AFV) and not _is64(s):
                continue
            if m == DQ_COPY and not sources(s):
                continue
            ok.append(m)
        if not ok:
            ok = [DQ_LIBRARY]
        m = ok[int(rng.integers(len(ok)))]
        src = 0
        if m == DQ_COPY:
            cand = sources(s)
            src = cand[int(rng.integers(len(cand)))]
        encs.append(dequant_encoding(rng, s, m, src))
        resolved.append(resolved[src] if m == DQ_COPY else DEFAULT_MODE[s] if m == DQ_LIBRARY else m)
    return encs


def dc_quant_field(rng, frame_dict, extra_levels):
    """A C.5.2 DcQuantField for a frame: per DC sample and channel
    dc_mul[c] / 2^k, k drawn uniformly in 0..extra_levels[c] (the values the
    decoded deltas can give), float32 (3, Hb, Wb)."""
    Hb, Wb = frame_dict["dc"].shape[1:]
    dc_mul = frame_dict["params"]["dc_mul"]
    out = np.empty((3, Hb, Wb), np.float32)
    for c in range(3):
        k = rng.integers(0, extra_levels[c] + 1, size=(Hb, Wb))
        out[c] = (np.float32(dc_mul[c]) / (2.0 ** k)).astype(np.float32)
    return out


def c1():
    return frame(256, 256, seed=0, choices=[DCT8], qf_const=8, cfl_zero=True,
                 epf_iters=0, gab=1, name="c1_256x256_dct8")


def c2():
    return frame(2048, 2048, seed=2, epf_iters=2, gab=1, name="c2_2048x2048_mixed_epf2")


def c2t():
    """The 2048x2048 recipe with regions drawn from every C.5.4 type except
    DCT32x8 / DCT8x32 (whose default tables drive samples out of range)."""
    types = [t for t in ALL_TYPES if t not in (DCT32X8, DCT8X32)]
    return frame(2048, 2048, seed=2, choices=types, epf_iters=2, gab=1,
                 name="c2t_2048x2048_13types_epf2")


def c3():
    return frame(4096, 4096, seed=3, p_dct32=0.5, epf_iters=2, gab=1,
                 name="c3_4096x4096_half_dct32")


def small(W=96, H=72, seed=11, epf_iters=2, **kw):
    """The c2 recipe at a size the oracle finishes in well under a second."""
    return frame(W, H, seed=seed, epf_iters=epf_iters, name=f"small_{W}x{H}", **kw)


def c4_sizes(seed=4, n=64):
    rng = np.random.default_rng(seed)
    lo, hi = math.log(256), math.log(3072)
    sides = np.exp(rng.uniform(lo, hi, size=(n, 2)))
    sides = np.clip(np.round(sides / 8) * 8, 256, 3072).astype(int)
    return [(int(w), int(h)) for w, h in sides]


def c4(n=64, seed=4):
    return [frame(w, h, seed=seed * 1000 + i, epf_iters=1, gab=1, out_format=1,
                  name=f"c4_{i}_{w}x{h}") for i, (w, h) in enumerate(c4_sizes(seed, n))]


def crop(mother, x0, y0, W, H, epf_iters=None, out_format=None, name=None):
    """The W x H part of `mother` at pixel offset (x0, y0), both multiples of
    64 (so the 32x32 regions and the 64x64 chroma-from-luma tiles stay
    aligned), as a frame of its own.  Varblocks cut by the new right or bottom
    edge become DCT8 blocks, so the DctSelect map stays well-formed."""
    assert x0 % 64 == 0 and y0 % 64 == 0
    assert x0 + W <= mother["xsize"] and y0 + H <= mother["ysize"]
    bx0, by0 = x0 // 8, y0 // 8
    Wb, Hb = (W + 7) // 8, (H + 7) // 8
    smap = mother["strategy"][by0:by0 + Hb, bx0:bx0 + Wb].copy()
    cx = _BX[smap]
    cy = _BY[smap]
    # a varblock's blocks sit at offsets (bx mod cx, by mod cy); it is cut when
    # its last column or row falls outside
    end_x = (np.arange(Wb)[None, :] // cx) * cx + cx
    end_y = (np.arange(Hb)[:, None] // cy) * cy + cy
    smap[(end_x > Wb) | (end_y > Hb)] = DCT8
    params = dict(mother["params"])
    if epf_iters is not None:
        params["epf_iters"] = epf_iters
    Wt, Ht = (W + 63) // 64, (H + 63) // 64
    return dict(name=name or f"crop_{W}x{H}", xsize=W, ysize=H,
                ac=np.ascontiguousarray(mother["ac"][:, 8 * by0:8 * (by0 + Hb), 8 * bx0:8 * (bx0 + Wb)]),
                dc=np.ascontiguousarray(mother["dc"][:, by0:by0 + Hb, bx0:bx0 + Wb]),
                strategy=smap,
                qf=np.ascontiguousarray(mother["qf"][by0:by0 + Hb, bx0:bx0 + Wb]),
                sharpness=np.ascontiguousarray(mother["sharpness"][by0:by0 + Hb, bx0:bx0 + Wb]),
                cfl_kx=np.ascontiguousarray(mother["cfl_kx"][y0 // 64:y0 // 64 + Ht, x0 // 64:x0 // 64 + Wt]),
                cfl_kb=np.ascontiguousarray(mother["cfl_kb"][y0 // 64:y0 // 64 + Ht, x0 // 64:x0 // 64 + Wt]),
                params=params,
                out_format=mother["out_format"] if out_format is None else out_format)


def splines(W, H, n, seed, max_points=12, step=(8, 48), sigma=(0.6, 3.0), value=0.3):
    """Synthetic already-decoded splines (K.4) for a W x H frame: n splines of
    1..max_points integer control points, a random walk of steps up to
    `step` pixels starting anywhere in (or just outside) the frame, no two
    consecutive points equal; DCT32 coefficients of X, Y, B with a DC of
    magnitude up to 32 * value and decaying higher terms, and of sigma with
    a DC of 32 * U(sigma) and small higher terms.  Returns (offsets (n + 1,)
    int32, points (m, 2) int32, dct (n, 4, 32) float32)."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(1, max_points + 1, size=n)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    pts = []
    for c in counts:
        x, y = int(rng.integers(-16, W + 16)), int(rng.integers(-16, H + 16))
        pts.append((x, y))
        for _ in range(c - 1):
            while True:
                ang = rng.uniform(0, 2 * np.pi)
                r = rng.uniform(*step)
                nx, ny = x + int(round(r * np.cos(ang))), y + int(round(r * np.sin(ang)))
                if (nx, ny) != (x, y):
                    break
            x, y = nx, ny
            pts.append((x, y))
    dct = np.zeros((n, 4, 32), np.float32)
    decay = 1.0 / (1.0 + np.arange(32))
    dct[:, :3, :] = (rng.standard_normal((n, 3, 32)) * decay * 32 * value / 3).astype(np.float32)
    dct[:, :3, 0] = rng.uniform(-32 * value, 32 * value, size=(n, 3))
    dct[:, 3, :] = (rng.standard_normal((n, 32)) * decay * 2.0).astype(np.float32)
    dct[:, 3, 0] = 32 * rng.uniform(*sigma, size=n)
    return offsets, np.array(pts, np.int32), dct


def with_splines(f, n, seed, **kw):
    """The frame dict f with n synthetic splines added (see splines())."""
    off, pts, dct = splines(f["xsize"], f["ysize"], n, seed, **kw)
    f = dict(f)
    f["spline_offsets"], f["spline_points"], f["spline_dct"] = off, pts, dct
    return f


def with_patches(f, n, seed):
    """The frame dict f with n already-decoded patch placements (K.3): six
    patch types of random sizes 1..16 with small integer residual samples
    in [-4, 4] (larger ones push XYB far out of range and linear RGB, a
    cube, to thousands), placed inside the frame, every fifth one against
    the right edge and every seventh against the bottom edge."""
    rng = np.random.default_rng(seed)
    W, H = f["xsize"], f["ysize"]
    sizes = [(int(rng.integers(1, 17)), int(rng.integers(1, 17))) for _ in range(6)]
    samples, offs = [], []
    off = 0
    for xs, ys in sizes:
        xs, ys = min(xs, W), min(ys, H)
        offs.append(off)
        samples.append(rng.integers(-4, 5, size=3 * xs * ys))
        off += 3 * xs * ys
    sizes = [(min(xs, W), min(ys, H)) for xs, ys in sizes]
    place = []
    for k in range(n):
        t = int(rng.integers(0, 6))
        xs, ys = sizes[t]
        x = int(rng.integers(0, W - xs + 1)) if k % 5 else W - xs
        y = int(rng.integers(0, H - ys + 1)) if k % 7 else H - ys
        place.append([x, y, xs, ys, offs[t]])
    f = dict(f)
    f["patch_place"] = np.array(place, np.int32)
    f["patch_samples"] = np.concatenate(samples).astype(np.int32)
    return f


def with_dots(f, n, seed):
    """The frame dict f with n already-decoded dots (C.4.5's ten integers
    each): centres in fifths of a pixel over the frame and a pixel past it,
    every size, angle, sign and colour code, about half of them circular
    (then the two sizes agree)."""
    rng = np.random.default_rng(seed)
    W, H = f["xsize"], f["ysize"]
    d = np.zeros((n, 10), np.int64)
    d[:, 0] = rng.integers(-5, 5 * W + 5, size=n)
    d[:, 1] = rng.integers(-5, 5 * H + 5, size=n)
    d[:, 2] = rng.integers(0, 16, size=n)
    d[:, 3] = rng.integers(0, 16, size=n)
    d[:, 4] = rng.integers(0, 8, size=n)
    d[:, 5] = rng.integers(0, 8, size=n)
    d[:, 6] = rng.integers(0, 10, size=n)
    d[:, 7] = rng.integers(0, 36, size=n)
    d[:, 8] = rng.integers(0, 10, size=n)
    d[:, 9] = rng.integers(0, 2, size=n)
    d[d[:, 9] == 1, 3] = d[d[:, 9] == 1, 2]
    d[:, 0] = np.clip(d[:, 0], 0, None)  # positions are unsigned
    d[:, 1] = np.clip(d[:, 1], 0, None)
    f = dict(f)
    f["dots"] = d.astype(np.int32)
    return f


def jpeg1(W, H, seed, hs=(2, 1, 1), vs=(2, 1, 1), grey=False):
    """A synthetic recompressed JPEG1 frame (M.4 already decoded) of W x H
    pixels: per component the quantized coefficients int32 [8 hib][8 wib]
    in natural order per block (whole MCUs of 8 hs[0] x 8 vs[0] pixels;
    component c has hs[c] x vs[c] blocks per MCU), and a quantization table
    growing with frequency (8 + 3 (u + v) for luma, 10 + 4 (u + v) for
    chroma).  DC uniform in [-64, 63] (chroma [-24, 23]); AC Laplacian with
    scale 6 / (1 + u + v), rounded half away from zero (most high-frequency
    coefficients zero)."""
    rng = np.random.default_rng(seed)
    n = 1 if grey else 3
    mx, my = -(-W // (8 * hs[0])), -(-H // (8 * vs[0]))
    coef, quant = [], []
    uu, vv = np.mgrid[0:8, 0:8]
    for c in range(n):
        wib, hib = mx * hs[c], my * vs[c]
        scale = np.tile(6.0 / (1.0 + uu + vv), (hib, wib))
        a = rng.laplace(0.0, scale)
        q = np.sign(a) * np.floor(np.abs(a) + 0.5)
        dc = rng.integers(-64, 64, size=(hib, wib)) if c == 0 else rng.integers(-24, 24, size=(hib, wib))
        q[::8, ::8] = dc
        coef.append(q.astype(np.int32))
        quant.append((8 + 3 * (uu + vv) if c == 0 else 10 + 4 * (uu + vv)).astype(np.int32))
    return {"xsize": W, "ysize": H, "coef": coef, "quant": quant, "hs": list(hs[:n]),
            "vs": list(vs[:n]), "name": f"jpeg1_{W}x{H}_{'grey' if grey else 'ycbcr'}"}


def jpeg1_gab_codes(seed, n=3):
    """Synthetic M.6.3 side-channel bytes per component: gab_weight1 * 1024,
    gab_weight2 * 1024 (around the J.4 defaults' 118 and 63), threshold * 16
    (0.5 to 6) and limit (1 to 36 of a block's interior pixels)."""
    rng = np.random.default_rng(seed)
    return [[int(rng.integers(60, 181)), int(rng.integers(20, 101)), int(rng.integers(8, 97)),
             int(rng.integers(1, 37))] for _ in range(n)]


def j1():
    """JPEG1 rasterization workload: 4096 x 4096, 4:2:0."""
    f = jpeg1(4096, 4096, seed=9)
    f["name"] = "j1_jpeg1_4096x4096_420"
    return f


def c5_mother():
    return frame(4096, 4096, seed=5, epf_iters=2, gab=1, name="c5_mother_4096x4096")


def c5_requests(rate=200.0, seconds=60.0, seed=5, lo=64, hi=4096):
    """Arrival times (seconds, Poisson process) and per-request recipes:
    (t, W, H, x0, y0, epf_iters, out_format)."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        w, h = np.exp(rng.uniform(math.log(lo), math.log(hi), size=2))
        W = int(min(hi, max(lo, round(w / 8) * 8)))
        H = int(min(hi, max(lo, round(h / 8) * 8)))
        x0 = 64 * int(rng.integers(0, (4096 - W) // 64 + 1))
        y0 = 64 * int(rng.integers(0, (4096 - H) // 64 + 1))
        epf = int(rng.integers(0, 4))
        fmt = 2 if rng.random() < 0.3 else 1
        reqs.append((t, W, H, x0, y0, epf, fmt))
    return reqs
