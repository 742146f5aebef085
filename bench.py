"""Benchmark: decoded megapixels per second, coefficients -> RGB, on one GPU.

Workload: one 2048x2048 frame, DctSelect drawn per 32x32 region from ten
transform types, quant field U{1..32}, chroma-from-luma U[-1, 1] per 64x64
tile, two edge-preserving filter passes, Gaborish, binary32 linear RGB out
(synthetic inputs, seeded).  A step is one whole reconstruction of the frame
with its inputs already resident in device memory: reconstruct, two EPF
passes, Gaborish + XYB -> RGB.  The steps call the same stage entry points as
jxlr_decode, with HIP events recorded between them on the launch stream, so
that each kernel's duration is measured inside the timed region.

After timing, the last step's output is compared with the FP64 oracle on the
full frame (max-abs error on [0,1]-scaled RGB outside pixels whose EPF
integer decisions differ between binary32 and binary64), and the oracle's
wall time for that same decode on the host cores is the CPU baseline.

Prints one JSON line.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peaks of one MI355X used for the roofline fractions.
HBM_PEAK_GBS = 8000.0
# Plain 32-bit VALU issue: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (one op per
# lane per clock, FMA counted once).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic work per pixel of one EPF pass (separable formulation): for each
# of the 56 window offsets, one packed 3-channel SAD of the new sample pair,
# 3 + 2 adds of the 4x3 patch box sum, 6 ops of Weight and the threshold,
# 4 FMAs of the weighted sums (3 channels and the weight total).
EPF_OPS_PER_PX = 56 * (1 + 5 + 7 + 4)
# Algorithmic HBM bytes per pixel of the other kernels (int32 AC in, f32 XYB
# out for reconstruct; f32 XYB in, f32 RGB out for finish).
RECON_BYTES_PER_PX = 12 + 12
FINISH_BYTES_PER_PX = 12 + 12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--no-check", action="store_true", help="skip the oracle comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1908_03565_amd import jxlr as J
    from paper_1908_03565_amd import workload as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log(f"bench: generating workload {args.workload}")
    frame = getattr(wl, args.workload)()
    W, H = frame["xsize"], frame["ysize"]
    p = J.params(W, H, **frame["params"])
    st = J.validate_maps_host(p, frame)
    assert st == 0, st
    ctx = J.Context(0)
    df = J.DeviceFrame(frame)
    bufs = [ctx.empty_xyb(p), ctx.empty_xyb(p)]
    info = ctx.empty_info(p)
    out = ctx.empty_out(p)
    stream = torch.cuda.current_stream()
    n_epf = p.epf_iters

    def step(evs):
        # block info + reconstruct -> EPF passes -> Gaborish + XYB -> RGB; an
        # event after each
        evs[0].record(stream)
        ctx.block_info(p, df, info, stream=stream)
        ctx.reconstruct(p, df, info, bufs[0], stream=stream)
        evs[1].record(stream)
        cur = 0
        for i in range(n_epf):
            ctx.epf_pass(p, df, info, bufs[cur], bufs[1 - cur], stream=stream)
            cur = 1 - cur
            evs[2 + i].record(stream)
        ctx.finish(p, df, bufs[cur], out, stream=stream)
        evs[2 + n_epf].record(stream)

    n_ev = 3 + n_epf
    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(n_ev)]
    warm = mk()
    for _ in range(args.warmup):
        step(warm)
    torch.cuda.synchronize()
    log(f"bench: warmup done ({args.warmup} steps); timing {args.steps} steps")
    events = [mk() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert ctx.device_status() == 0
    total_ms = events[0][0].elapsed_time(events[-1][-1])
    ms_per_step = total_ms / args.steps
    lat = [e[0].elapsed_time(e[-1]) for e in events]
    recon_ms = statistics.mean(e[0].elapsed_time(e[1]) for e in events)
    epf_ms = [statistics.mean(e[1 + i].elapsed_time(e[2 + i]) for e in events) for i in range(n_epf)]
    fin_ms = statistics.mean(e[1 + n_epf].elapsed_time(e[2 + n_epf]) for e in events)
    mp = W * H / 1e6
    value = mp / (ms_per_step / 1e3)
    log(f"bench: {ms_per_step:.4f} ms/step, {value:.1f} MP/s; recon {recon_ms:.4f} ms, "
        f"epf {['%.4f' % x for x in epf_ms]} ms, finish {fin_ms:.4f} ms")

    px = W * H
    kernels = {"recon_kernel": dict(ms=recon_ms, bound="hbm",
                                    achieved=px * RECON_BYTES_PER_PX / (recon_ms / 1e3) / 1e9),
               "finish_kernel": dict(ms=fin_ms, bound="hbm",
                                     achieved=px * FINISH_BYTES_PER_PX / (fin_ms / 1e3) / 1e9)}
    if n_epf:
        e_ms = statistics.mean(epf_ms)
        kernels["epf_kernel"] = dict(ms=e_ms, bound="alu",
                                     achieved=px * EPF_OPS_PER_PX / (e_ms / 1e3) / 1e12)
    dominant = max(kernels, key=lambda k: kernels[k]["ms"] * (n_epf if k == "epf_kernel" else 1))
    dk = kernels[dominant]
    if dk["bound"] == "alu":
        roofline = dict(bound="alu", kernel=dominant, achieved=round(dk["achieved"], 3),
                        peak=round(ALU_PEAK_TOPS, 3), unit="Top/s",
                        frac=round(dk["achieved"] / ALU_PEAK_TOPS, 4),
                        avg_ms=round(dk["ms"], 5), ops_per_px=EPF_OPS_PER_PX, traffic=None)
    else:
        roofline = dict(bound="hbm", kernel=dominant, achieved=round(dk["achieved"], 1),
                        peak=HBM_PEAK_GBS, unit="GB/s", frac=round(dk["achieved"] / HBM_PEAK_GBS, 4),
                        avg_ms=round(dk["ms"], 5), traffic=None)

    err = None
    cpu = None
    if not args.no_check or not args.no_cpu_baseline:
        from oracle import oracle as O
        from tests import parity as P
        q = O.params(W, H, **frame["params"])
        log("bench: running the FP64 oracle on the full frame")
        t = time.perf_counter()
        orc = O.decode_stages(q, frame)
        cpu_s = time.perf_counter() - t
        cpu = dict(value=round(mp / cpu_s, 4), unit="MP/s", cores=O.num_threads(), kind="oracle",
                   sample=f"one full {W}x{H} decode ({cpu_s:.2f} s), FP64 scalar C, OpenMP")
        if not args.no_check:
            from tests.parity import gpu_stages, compare_rgb
            gpu = gpu_stages(ctx, p, df)
            np.testing.assert_array_equal(gpu["out"], out.cpu().numpy())
            cmp = compare_rgb(p, gpu, orc)
            err = dict(max_abs_err=cmp["max_err"], tol=P.RGB_TOL,
                       flip_affected_px=cmp["affected"],
                       max_abs_err_flip_affected=cmp["max_err_affected"], passes=cmp["passes"])
            log(f"bench: max-abs err {cmp['max_err']:.3g} (tol {P.RGB_TOL}); "
                f"flip-affected {cmp['affected']} px")
        if args.no_cpu_baseline:
            cpu = None

    res = {
        "metric": "decoded MP/s (coeffs->RGB) at stated max-abs err vs FP64; p50/p99 latency",
        "value": round(value, 2),
        "unit": "MP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": frame["name"], "xsize": W, "ysize": H, "epf_iters": n_epf,
                   "gaborish": bool(p.gab), "output": "f32 linear RGB / 255",
                   "frames_per_step": 1},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 5),
                       "p99": round(float(np.percentile(lat, 99)), 5)},
        "stage_ms": {"reconstruct": round(recon_ms, 5), "epf": [round(x, 5) for x in epf_ms],
                     "finish": round(fin_ms, 5)},
        "host_wall_ms_per_step": round(wall / args.steps * 1e3, 5),
        "error": err,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
