"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a one-line JSON message and exit status 2."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_traffic_figures_match_the_kernel_sources():
    # the stored HBM counter figures are reported only for the sources they
    # were taken on; a changed source turns them into null
    bench = _bench()
    assert bench.sources_sha256() == bench.PMC_SOURCES_SHA256
    key = ("c4_batch64_loguniform_256_3072_epf1_u8srgb", "epf_batch_kernel")
    f, w = bench.PMC_KIB[key]
    assert bench.traffic_bytes(*key) == int(round(1024 * (2.0 * f + 1.0 * w)))
    assert bench.traffic_bytes(key[0] + "_nofuse", key[1]) is None
    saved = bench.PMC_SOURCES_SHA256
    try:
        bench.PMC_SOURCES_SHA256 = "0" * 64
        assert bench.traffic_bytes(*key) is None
    finally:
        bench.PMC_SOURCES_SHA256 = saved


def test_roofline_of_picks_the_dominant_kernel_and_its_units():
    bench = _bench()
    px = 1000000
    kernels = {
        "recon_kernel": dict(ms=0.05, bound="hbm", bytes_per_px=24,
                             achieved=px * 24 / 0.05e-3 / 1e9),
        "epf_kernel": dict(ms=0.1, bound="alu",
                           achieved=px * bench.EPF_OPS_PER_PX / 0.1e-3 / 1e12),
    }
    r = bench.roofline_of(kernels, {"epf_kernel": 2}, None, px, 15)
    assert r["kernel"] == "epf_kernel" and r["bound"] == "alu" and r["unit"] == "Top/s"
    assert abs(r["frac"] - r["achieved"] / bench.ALU_PEAK_TOPS) < 1e-3
    assert r["algorithmic_bytes"] == 15 * px and r["ops_per_px"] == 700
    # 56 window offsets x 12.5 lane operations of the strip formulation
    assert bench.EPF_OPS_PER_PX == 56 * 12.5
    kernels["recon_kernel"]["ms"] = 0.5
    r = bench.roofline_of(kernels, {"epf_kernel": 2}, None, px)
    assert r["kernel"] == "recon_kernel" and r["unit"] == "GB/s"
    assert r["peak"] == bench.HBM_PEAK_GBS and r["algorithmic_bytes"] == 24 * px
