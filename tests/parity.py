"""Parity helpers shared by the GPU tests, smoke() and bench.py.

Runs a frame through the GPU path stage by stage (via the C-ABI binding) and
through the FP64 oracle, and compares them.  The edge-preserving filter turns
real values into integers twice (the 8-bit guide samples and the truncated
sigma, J.2.2 and J.2.4); binary32 and binary64 inputs that differ in the last
bits can land on different sides of such a boundary.  Both sides' integer
decisions are compared directly; pixels whose filter footprint contains a
differing decision are counted and reported separately, and the tolerance is
applied to all other pixels.
"""
import numpy as np

# Max-abs tolerance on [0,1]-scaled linear RGB for the FP32 form.
RGB_TOL = 1e-4


def mirror_index(idx, size):
    """6.5 mirroring of an index array."""
    idx = np.asarray(idx).copy()
    while np.any((idx < 0) | (idx >= size)):
        idx = np.where(idx < 0, -idx - 1, idx)
        idx = np.where(idx >= size, 2 * size - 1 - idx, idx)
    return idx


def dilate(mask, dxs, dys):
    """out[y, x] = any mask[mirror(y + dy), mirror(x + dx)] over the offsets."""
    H, W = mask.shape
    out = np.zeros_like(mask)
    if not mask.any():
        return out
    for dy in dys:
        rows = mask[mirror_index(np.arange(H) + dy, H)]
        for dx in dxs:
            out |= rows[:, mirror_index(np.arange(W) + dx, W)]
    return out


# Footprint of one EPF output pixel: guide samples at x-4..x+6, y-4..y+4
# (patches of x-1..x+2, y-1..y+1 around offsets -3..4, -3..3); input samples
# inside that.
EPF_DX = range(-4, 7)
EPF_DY = range(-4, 5)


def affected_mask(p, gpu_passes, orc_passes, start=None):
    """Pixels whose value may legitimately differ because an integer decision
    differs.  gpu_passes / orc_passes: lists of (guide (3,H,W) u8, sigma (Hb,Wb));
    start: pixels already affected before the first pass (or None)."""
    H, W = p.ysize, p.xsize
    bad = np.zeros((H, W), bool) if start is None else start.copy()
    stats = []
    for (gg, sg), (go, so) in zip(gpu_passes, orc_passes):
        gmis = np.any(gg != go, axis=0)
        smis_b = sg != so
        smis = np.kron(smis_b, np.ones((8, 8), bool))[:H, :W]
        new = dilate(gmis | bad, EPF_DX, EPF_DY) | smis
        stats.append(dict(guide_flips=int(gmis.sum()), sigma_flips=int(smis_b.sum())))
        bad = new
    return bad, stats


def gpu_stages(ctx, p, df):
    """Runs the stage entry points; returns numpy arrays of every stage."""
    import torch
    info = ctx.empty_info(p)
    ctx.block_info(p, df, info)
    xyb = ctx.empty_xyb(p)
    pred = None
    if p.ac_prediction:
        pred = ctx.empty_pred(p)
        ctx.ac_prediction(p, df, info, pred)
    ctx.reconstruct(p, df, info, xyb, pred=pred)
    res = {"recon": xyb.cpu().numpy(), "epf": []}
    Hb, Wb = (p.ysize + 7) // 8, (p.xsize + 7) // 8
    cur = xyb
    for _ in range(p.epf_iters):
        nxt = ctx.empty_xyb(p)
        guide = torch.empty((3, p.ysize, p.xsize), dtype=torch.uint8, device=cur.device)
        sigma = torch.empty((Hb, Wb), dtype=torch.int32, device=cur.device)
        ctx.epf_pass(p, df, info, cur, nxt, guide, sigma)
        res["epf"].append((nxt.cpu().numpy(), guide.cpu().numpy(), sigma.cpu().numpy()))
        cur = nxt
    if p.qco and p.epf_iters > 0:
        ctx.qco_pass(p, df, info, xyb, cur)
        res["qco"] = cur.cpu().numpy()
    if p.num_patches:
        if cur is xyb:  # keep the reconstruction as it was
            cur = xyb.clone()
        ctx.patches(p, df, cur)
        res["patches"] = cur.cpu().numpy()
    if p.num_dots or p.num_splines:
        # Gaborish as its own pass before them
        if p.gab:
            g = ctx.empty_xyb(p)
            ctx.gaborish(p, cur, g)
            cur = g
        elif cur is xyb:
            cur = xyb.clone()
        res["gab"] = cur.cpu().numpy()
    if p.num_dots:
        ctx.dots(p, df, cur)
        res["dots"] = cur.cpu().numpy()
    if p.num_splines:
        ctx.splines(p, df, cur)
        res["splines"] = cur.cpu().numpy()
    out = ctx.empty_out(p)
    raw = None
    if p.noise:
        raw = ctx.empty_xyb(p)
        ctx.noise_channels(p, raw)
        res["noise_raw"] = raw.cpu().numpy()
    ctx.finish(p, df, cur, out, noise_raw=raw)
    res["out"] = out.cpu().numpy()
    torch.cuda.synchronize()
    return res


def varblock_ids(strategy):
    """Varblock index of every block of a DctSelect map (raster order of the
    top-left blocks, each varblock cx x cy blocks of its type)."""
    from oracle import oracle as O
    Hb, Wb = strategy.shape
    ids = -np.ones((Hb, Wb), np.int64)
    n = 0
    for by in range(Hb):
        for bx in range(Wb):
            if ids[by, bx] >= 0:
                continue
            bw, bh = O.varblock_size(int(strategy[by, bx]))
            ids[by:by + bh // 8, bx:bx + bw // 8] = n
            n += 1
    return ids


def spread_to_varblocks(mask, strategy):
    """Every pixel of a varblock that holds a masked pixel (the quantization
    constraint mixes the samples of a varblock)."""
    H, W = mask.shape
    ids = varblock_ids(strategy)
    Hb, Wb = ids.shape
    pad = np.zeros((8 * Hb, 8 * Wb), bool)
    pad[:H, :W] = mask
    hit_blocks = pad.reshape(Hb, 8, Wb, 8).any(axis=(1, 3))
    hit = np.isin(ids, np.unique(ids[hit_blocks]))
    return np.kron(hit, np.ones((8, 8), bool))[:H, :W]


def acpred_mask(q, frame, rel=1e-5):
    """AC prediction's smoothing test (|wa - s| <= 1.7 dcq) is taken in
    binary32 on the GPU: the pixels of every varblock holding a cell whose
    test is within rel of its boundary (relative to dcq and the cell's size),
    from the oracle's margins.  q: oracle parameters."""
    from oracle import oracle as O
    Hb, Wb = frame["strategy"].shape
    dq = frame["dc"].astype(np.float64) * np.array(q.dc_mul)[:, None, None]
    dq /= (2.0 ** np.array(list(q.extra_levels)))[:, None, None]
    if q.dc_smoothing:
        dq = O.dc_smooth(q, dq, frame.get("dc_quant"))
    dq[0] += q.kx_dc * dq[1]
    dq[2] += q.kb_dc * dq[1]
    cells, margin = O.ac_prediction_image(q, frame["strategy"], dq, want_margin=True)
    tol = rel * (np.array(q.dc_mul)[:, None, None] + np.abs(cells))
    near = (np.abs(margin) <= tol).any(axis=0)
    blocks = near.reshape(Hb, 2, Wb, 2).any(axis=(1, 3))
    ids = varblock_ids(frame["strategy"])
    hit = np.isin(ids, np.unique(ids[blocks]))
    return np.kron(hit, np.ones((8, 8), bool))[:q.ysize, :q.xsize], int(near.sum())


def compare_rgb(p, gpu, orc, strategy=None, start=None):
    """Max-abs error of the final [0,1]-scaled RGB outside flip-affected
    pixels, plus the flip statistics.  With the quantization constraint on,
    pass the DctSelect map: the mask spreads over whole varblocks.  start:
    pixels affected before the filters (AC prediction's near-boundary
    varblocks)."""
    mask, stats = affected_mask(p, [(g, s) for _, g, s in gpu["epf"]],
                                [(g, s) for _, g, s in orc["epf"]], start)
    if p.qco and p.epf_iters > 0:
        mask = spread_to_varblocks(mask, strategy)
    if p.gab:
        mask = dilate(mask, range(-1, 2), range(-1, 2))
    err = np.abs(gpu["out"].astype(np.float64) - orc["rgb"])
    ok = ~mask
    return dict(max_err=float(err[:, ok].max()) if ok.any() else 0.0,
                max_err_affected=float(err[:, mask].max()) if mask.any() else 0.0,
                affected=int(mask.sum()), pixels=int(mask.size), passes=stats,
                max_abs_ref=float(np.abs(orc["rgb"]).max()), mask=mask)


def max_err_by_type(frame, gpu, orc, mask):
    """Max-abs RGB error over the pixels of each transform type's varblocks,
    outside the flip-affected mask; keys are type numbers."""
    H, W = mask.shape
    types = np.kron(frame["strategy"], np.ones((8, 8), np.uint8))[:H, :W]
    e = np.abs(gpu["out"].astype(np.float64) - orc["rgb"]).max(axis=0)
    res = {}
    for t in np.unique(types):
        sel = (types == t) & ~mask
        if sel.any():
            res[int(t)] = float(e[sel].max())
    return res


def srgb_codes_check(p, codes, orc, gpu_epf, bits):
    """Compares 8/16-bit output codes with the oracle's rounding (sRGB OETF,
    then round half up).  Returns (n_firm_equal, n_firm, max_code_diff): codes
    must equal where the oracle's pre-rounding value is not within the FP32
    error bound of a rounding boundary and no EPF decision differs; elsewhere
    (outside flip-affected pixels) a neighbouring code is allowed."""
    from oracle import oracle as O
    codes = np.asarray(codes).astype(np.int64)
    lin = orc["rgb"]
    ref = O.quantize_srgb(bits, lin).astype(np.int64)
    maxv = (1 << bits) - 1
    v = np.clip(lin, 0, 1)
    e = np.where(v <= 0.0031308, 12.92 * v, 1.055 * np.power(v, 1 / 2.4) - 0.055) * maxv + 0.5
    frac = e - np.floor(e)
    near = np.minimum(frac, 1 - frac) < maxv * RGB_TOL * 13 + 1e-3  # OETF slope <= 12.92
    mask, _ = affected_mask(p, [(g, s) for _, g, s in gpu_epf], [(g, s) for _, g, s in orc["epf"]])
    if p.gab:
        mask = dilate(mask, range(-1, 2), range(-1, 2))
    firm = ~near & ~mask[None]
    diff = np.abs(codes - ref)[~mask[None].repeat(3, 0)]
    return (int((codes[firm] == ref[firm]).sum()), int(firm.sum()),
            int(diff.max()) if diff.size else 0)
