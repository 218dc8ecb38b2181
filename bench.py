#!/usr/bin/env python3
"""Throughput of the EPIC imager hot path on one MI355X.

A step is one whole cadence through image_cadence: every channel and every
time sample of the workload is gridded, transformed, squared and averaged
(Eq. 3 then Eq. 2).  The default workload is the station-scale layout: 256
elements in a 38 m circle (1.5 m minimum spacing), 150 MHz, 64x64 grid at
lambda/2, 3x3 Gaussian kernel, 2 pols, 1024 channels, 2048 samples per
cadence, int8 complex voltages (sigma 16), FP32 FFT path.  Inputs are seeded,
synthetic and already resident in HBM when the timed region starts.

Prints one JSON line: grid pixel-samples/s (sum over stations of
nx*ny*n_chan*n_time per cadence, divided by the cadence time), the roofline
of the dominant kernel (timed live with HIP events on its own stream), and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_HBM_GBS = 8000.0
# FP32 vector peak without packed FP32 math (the library is built with it off):
# 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz.  The 157.3 TFLOP/s figure
# counts packed FP32 (two FMAs per lane per instruction).
PEAK_FP32_VALU_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
PEAK_FP16_MFMA_TFLOPS = 2500.0
PEAK_INT8_MFMA_TOPS = 5000.0          # dense int8 matrix cores
PEAK_FP32_MFMA_TFLOPS = 157.3         # dense FP32 matrix cores
PREC_NAMES = {"fp32": W.FP32_FFT, "fp16": W.FP16_SPLIT, "bf16": W.BF16_SPLIT}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Sources of each timed kernel: a counter summary under profiles/ is only used
# while the hash of these files matches the one recorded with the counters.
KERNEL_SOURCES = {
    "fused_fft_cadence": ["k_fused.hip", "fft_lds.hpp", "volts.hpp"],
    "fused_dft_cadence": ["k_fused_dft.hip", "mfma_split.hpp", "volts.hpp"],
}


def measured_traffic(kernel: str, workload: str, chunk):
    """HBM bytes per launch from profiles/<kernel>_<workload>_hbm_bytes.md, or
    None if there is no summary, the kernel changed since it was taken, or it
    was taken at another time-chunk length (the partial-sum writes scale with
    1/chunk)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_bytes.md")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    text = open(path).read()
    m_b = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    m_h = re.search(r"source_sha256_16: ([0-9a-f]+)", text)
    m_c = re.search(r"chunk: (\d+)", text)
    if not (m_b and m_h and m_c) or chunk is None or int(m_c.group(1)) != chunk:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        p = os.path.join(ROOT, "paper_2411_17804_amd", "csrc", f)
        if not os.path.exists(p):
            return None
        h.update(open(p, "rb").read())
    return int(m_b.group(1)) if h.hexdigest()[:16] == m_h.group(1) else None


def flops_per_pixel_sample(cfg, st, with_grid=True):
    """Algorithmic FP32 work per grid pixel-sample of the FFT path.

    transform: 5 N log2 N per complex N-point transform, per pol;
    gridding: 4 flops (complex x real weight, complex add) per tap per pol;
    products: XX and YY 3 flops each, XY 6 (YX is its conjugate); accumulation:
    one add per real component (4 for two pols, 1 for one)."""
    npix = st.nx * st.ny
    fft = cfg.n_pol * 5.0 * math.log2(npix)
    grid = 4.0 * st.n_elem * st.support ** 2 * cfg.n_pol / npix if with_grid else 0.0
    prod = 12.0 + 4.0 if cfg.n_pol == 2 else 3.0 + 1.0
    return fft + grid + prod


def split_mfma_flops(cfg):
    """Matrix-core flops of the fused split-precision kernel for one cadence
    (stations with square grids up to 64): per sample, pol and channel, each of
    the n/16 waves (16 output rows each) runs my*mx stage-1 and (n/16)*mx
    stage-2 16x16x32 tiles for the real and imaginary outputs, three split
    products each, where mx, my are the footprint box sides in 16-cell tiles.
    The box follows the element cells and kernel support exactly as the plan
    places them."""
    total = 0
    for st in cfg.stations:
        if st.nx != st.ny or st.nx > 64:
            continue
        h = (st.support - 1) // 2
        for lam in cfg.wavelengths_m:
            d = W.GRID_SPACING_WL * lam
            ci = np.floor(st.pos_m[:, 0] / d + st.nx // 2 + 0.5)
            cj = np.floor(st.pos_m[:, 1] / d + st.ny // 2 + 0.5)
            bw = int(ci.max() - ci.min()) + 2 * h + 1
            bh = int(cj.max() - cj.min()) + 2 * h + 1
            mx, my = -(-bw // 16), -(-bh // 16)
            tiles = (st.nx // 16) * 2 * 3 * (my * mx + (st.nx // 16) * mx)
            total += tiles * 16 * 16 * 32 * 2 * cfg.n_time * cfg.n_pol
    return total


def tiles128_mfma_flops(cfg):
    """Matrix-core flops of the 128 x 128 split-precision plane transform for
    one cadence (stations with 128 x 128 grids): per sample, pol and channel,
    16 M-tiles (16 output rows each) times ka x cb tiles in the first pass and
    cb x 8 in the second, three split products of 16x16x32 each, where ka >= cb
    are the footprint box's sides in 16-cell tiles counted from its first cell
    (the longer side is transformed first).  The box follows the element cells and kernel support
    exactly as the plan places them."""
    total = 0
    for st in cfg.stations:
        if st.nx != 128 or st.ny != 128:
            continue
        h = (st.support - 1) // 2
        for lam in cfg.wavelengths_m:
            d = W.GRID_SPACING_WL * lam
            ci = np.floor(st.pos_m[:, 0] / d + st.nx // 2 + 0.5)
            cj = np.floor(st.pos_m[:, 1] / d + st.ny // 2 + 0.5)
            bw = int(ci.max() - ci.min()) + 2 * h + 1
            bh = int(cj.max() - cj.min()) + 2 * h + 1
            sx, sy = -(-bw // 16), -(-bh // 16)
            ka, cb = max(sx, sy), min(sx, sy)
            total += 3 * 16 * 16 * 32 * 2 * 16 * cb * (ka + 8) * cfg.n_time * cfg.n_pol
    return total


def pass_mfma_flops(cfg):
    """Matrix-core flops of the two-pass split-precision transform for one
    cadence (square grids of 256): per sample, pol and channel, the first pass
    (along y) runs 2N/16 M-tiles x 2 column tiles x (the footprint's 16-row
    tiles) for each 32-column block that meets the footprint, the second
    (along x) the same M-tiles x 2 column tiles x (the footprint's 16-column
    tiles) for all N/32 blocks; three split products of 16x16x32 each.  Tiles
    are aligned to the grid, as the passes read them."""
    total = 0
    for st in cfg.stations:
        if st.nx != 256 or st.ny != 256:
            continue
        n, h = st.nx, (st.support - 1) // 2
        for lam in cfg.wavelengths_m:
            d = W.GRID_SPACING_WL * lam
            ci = np.floor(st.pos_m[:, 0] / d + n // 2 + 0.5)
            cj = np.floor(st.pos_m[:, 1] / d + n // 2 + 0.5)
            x0, x1 = int(ci.min()) - h, int(ci.max()) + h
            y0, y1 = int(cj.min()) - h, int(cj.max()) + h
            ks_y, ks_x = (y1 >> 4) - (y0 >> 4) + 1, (x1 >> 4) - (x0 >> 4) + 1
            nblk_x = (x1 >> 5) - (x0 >> 5) + 1
            mt = 2 * n // 16
            mfma = 3 * mt * 2 * (ks_y * nblk_x + ks_x * (n // 32))
            total += mfma * 16 * 16 * 32 * 2 * cfg.n_time * cfg.n_pol
    return total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--precision", choices=sorted(PREC_NAMES), default="fp32")
    ap.add_argument("--n-chan", type=int, default=None, help="shrink the band (testing)")
    ap.add_argument("--n-time", type=int, default=None, help="shrink the cadence (testing)")
    ap.add_argument("--cpu-channels", type=int, default=192,
                    help="channels of the workload the CPU oracle is timed on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default time-chunk length of the fused kernels")
    ap.add_argument("--no-stages", action="store_true",
                    help="skip the per-stage (unfused) roofline measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (to scale the HBM "
                         "byte counters of a profiler run)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = 1 << 28                       # 2^28 float32 = 1 GiB
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": 4 * n, "launches": 3}))
        return

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only: the path would shard "
                          "by channel with no exchange between GPUs, and only the single-GPU "
                          "throughput is measured", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2411_17804_amd import epic

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    epic.load()

    cfg = W.make_config(args.config, n_chan=args.n_chan, n_time=args.n_time,
                        precision=PREC_NAMES[args.precision])
    log(f"workload C{cfg.index}: {len(cfg.stations)} station(s), {cfg.n_chan} channels x "
        f"{cfg.n_time} samples, precision {args.precision}")
    t_gen = time.time()
    stations = []
    host_volts = []
    for s, st in enumerate(cfg.stations):
        v = W.station_volts(cfg, s, threads=16)
        host_volts.append(v if not args.no_cpu_baseline else None)
        if v.dtype == np.int8:
            vd = torch.from_numpy(v).to(dev)
        else:
            vd = torch.from_numpy(v.view(np.float32)).to(dev)
        img = torch.zeros((cfg.n_chan, cfg.n_pol * cfg.n_pol, st.ny, st.nx, 2),
                          dtype=torch.float32, device=dev)
        stations.append(epic.Station(st.pos_m, st.nx, st.ny, st.kernel_type, st.support,
                                     st.sigma_cells, volts=vd, image=img))
    common = epic.Common(cfg.n_pol, cfg.wavelengths_m, W.GRID_SPACING_WL, cfg.n_time,
                         cfg.volt_type, cfg.precision)
    torch.cuda.synchronize()
    log(f"inputs generated and resident in HBM ({cfg.volt_bytes() / 1e9:.2f} GB) "
        f"in {time.time() - t_gen:.1f} s")

    # the tuned chunk lengths come back through the library's tune-cache file
    # ("class chunk" lines); without autotuning every class uses 32
    tune_file = os.environ.get("EPIC_TUNE_CACHE")
    if not tune_file:
        import tempfile
        tune_file = os.path.join(tempfile.mkdtemp(prefix="epic_bench_"), "tune.txt")
        os.environ["EPIC_TUNE_CACHE"] = tune_file
    chunks = {}
    if not args.no_autotune:
        t_tune = time.time()
        epic.autotune(common, stations)
        log(f"autotune done in {time.time() - t_tune:.1f} s")
        if os.path.exists(tune_file):
            for line in open(tune_file):
                parts = line.split()
                if len(parts) == 2:
                    chunks[parts[0]] = int(parts[1])
        log(f"tuned chunks {chunks}")
    for i in range(args.warmup):
        epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")

    # timed region: the cadence as the library runs it (graph replays)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # the same steps again with every kernel bracketed by HIP events on its
    # own stream (eager launches), for the per-kernel durations
    epic.timing_reset()
    epic.timing_enable(True)
    for i in range(args.steps):
        epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    epic.timing_enable(False)
    kern = epic.timing_report()
    pix = cfg.pixel_samples()
    value = pix / (ms_per_step / 1e3)
    log(f"{args.steps} steps: {ms_per_step:.2f} ms/step, {value:.3e} px-samples/s; kernels {kern}")

    # dominant kernel and its roofline
    dom_name, (dom_count, dom_ms) = max(kern.items(), key=lambda kv: kv[1][1])
    prefix = {"fused_fft_cadence": "fft_", "fused_dft_cadence": "dft_",
              "fused_fft128_cadence": "fft128_"}.get(dom_name)
    cls = sorted(v for k, v in chunks.items() if prefix and k.startswith(prefix))
    dom_chunk = cls[0] if len(set(cls)) == 1 else (32 if args.no_autotune else None)
    dom_avg_ms = dom_ms / dom_count
    launches_per_step = dom_count / args.steps
    st0 = cfg.stations[0]
    if args.precision == "fp32" and dom_name != "grid_gather":
        # the stations the dominant kernel serves (grids up to 64: the fused
        # FFT kernels with their gridding; 128: the 128 x 128 transform kernel,
        # whose gridding runs in k_grid_box)
        served = [s for s in cfg.stations if (s.nx == 128) == (dom_name == "fused_fft128_cadence")]
        served = served or cfg.stations
        with_grid = dom_name != "fused_fft128_cadence"
        work_step = sum(flops_per_pixel_sample(cfg, s, with_grid) * s.nx * s.ny * cfg.n_chan * cfg.n_time
                        for s in served)
        flop_px = work_step / sum(s.nx * s.ny * cfg.n_chan * cfg.n_time for s in served)
        work = work_step / launches_per_step
        achieved = work / (dom_avg_ms / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3),
                "peak": round(PEAK_FP32_VALU_TFLOPS, 1), "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 4),
                "traffic": measured_traffic(dom_name, f"C{cfg.index}", dom_chunk)
                if cfg.n_chan == W.make_config(cfg.index).n_chan and args.n_time is None else None,
                "kernel": dom_name, "avg_launch_ms": round(dom_avg_ms, 4), "chunk": dom_chunk,
                "flop_per_pixel_sample": round(flop_px, 2)}
    elif dom_name == "grid_gather" and args.precision == "fp32":
        # the composed path's gather gridding: HBM-bound; the voltages read
        # once and every written cell once per sample (on the two-pass grids,
        # 256 wide or 128 x 128, only the footprint box's rows are written)
        bv = 2 if cfg.volt_type == W.CI8 else 8
        bytes_step = 0
        for s in cfg.stations:
            two_pass = s.ny == 256 or (s.ny == 128 and s.nx >= 128)
            h = (s.support - 1) // 2
            for lam in cfg.wavelengths_m:
                rows = s.ny
                if two_pass:
                    cj = np.floor(s.pos_m[:, 1] / (W.GRID_SPACING_WL * lam) + s.ny // 2 + 0.5)
                    rows = int(cj.max() - cj.min()) + 2 * h + 1
                bytes_step += cfg.n_time * cfg.n_pol * (s.n_elem * bv + s.nx * rows * 8)
        achieved = bytes_step / launches_per_step / (dom_avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                "kernel": dom_name, "avg_launch_ms": round(dom_avg_ms, 4), "chunk": None,
                "bytes_per_step": int(bytes_step)}
    elif dom_name == "square_accumulate":
        # the composed path's squaring and compensated accumulation: HBM-bound;
        # per launch it reads a chunk of transformed planes and reads and
        # writes the (sum, compensation) accumulators, and the last launch of
        # each station writes its image
        acc_b = sum(cfg.n_chan * cfg.n_pol ** 2 * s.nx * s.ny * 8 for s in cfg.stations)
        field_b = sum(cfg.n_chan * cfg.n_time * cfg.n_pol * s.nx * s.ny * 8 for s in cfg.stations)
        bytes_step = field_b + launches_per_step * 4 * acc_b / len(cfg.stations) + acc_b
        achieved = bytes_step / launches_per_step / (dom_avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                "kernel": dom_name, "avg_launch_ms": round(dom_avg_ms, 4), "chunk": None,
                "bytes_per_step": int(bytes_step)}
    else:
        fl = {"fused_dft_cadence": split_mfma_flops,
              "dft2_tiles128": tiles128_mfma_flops,
              "dft_gemm_pass": pass_mfma_flops}.get(dom_name, lambda c: None)(cfg)
        achieved = fl / launches_per_step / (dom_avg_ms / 1e3) / 1e12 if fl else None
        roof = {"bound": "mfma", "achieved": round(achieved, 2) if achieved else None,
                "peak": PEAK_FP16_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP16_MFMA_TFLOPS, 4) if achieved else None,
                "traffic": measured_traffic(dom_name, f"C{cfg.index}", dom_chunk)
                if cfg.n_chan == W.make_config(cfg.index).n_chan and args.n_time is None else None,
                "kernel": dom_name, "avg_launch_ms": round(dom_avg_ms, 4), "chunk": dom_chunk,
                "flop_per_step": fl}

    out = {
        "metric": "grid pixel-samples/s per GPU",
        "value": value,
        "unit": "pixel-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16x3+f32acc", "bf16": "bf16x3+f32acc"}[args.precision],
        "data": "synthetic (seeded layouts and voltages shaped like the paper's arrays)",
        "config": {"workload": f"C{cfg.index}: " + {
            1: "64 el, 32x32 grid, nearest, 1 pol, cf32",
            2: "station: 256 el in 38 m circle, 64x64 grid, 3x3 Gaussian, 2 pols, ci8",
            3: "dense 64x32 lattice, 128x128 grid, 3x3 Gaussian, 2 pols, cf32",
            4: "96 stations of 64-1024 el, 32/64/128 grids, 2 pols, ci8",
            5: "128x128 lattice -5%, 256x256 grid, 5x5 Gaussian, 2 pols, cf32"}[cfg.index],
            "n_chan": cfg.n_chan, "n_time": cfg.n_time, "n_stations": len(cfg.stations),
            "precision": args.precision, "pixel_samples_per_step": pix,
            "realtime_factor": (cfg.n_time * 25e-6) / (ms_per_step / 1e3)},
        "roofline": roof,
        "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in kern.items()},
    }

    if not args.no_stages:
        c0 = epic.Common(cfg.n_pol, cfg.wavelengths_m, W.GRID_SPACING_WL, cfg.n_time,
                         cfg.volt_type, cfg.precision)
        out["stages"] = stage_rooflines(cfg, c0, stations[0])
        if len(cfg.stations) == 1:
            out["stages"]["inter_station_epic"] = array_stage(cfg)
        log(f"stages: {out['stages']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, stations, host_volts, args.cpu_channels)
    print(json.dumps(out), flush=True)


def stage_rooflines(cfg, common, station, nt=64, reps=3):
    """Each unfused stage on a block of nt samples of every channel of the
    first station, timed with events on the current stream, against the
    roofline that bounds it (algorithmic bytes for HBM-bound stages,
    algorithmic matrix-core flops for the DFT-matrix products)."""
    import torch
    from paper_2411_17804_amd import epic
    st = cfg.stations[0]
    npix = st.nx * st.ny
    nt = min(nt, cfg.n_time)
    batch = cfg.n_chan * nt * cfg.n_pol
    field_bytes = batch * npix * 8
    grid = torch.empty((cfg.n_chan, nt, cfg.n_pol, st.ny, st.nx, 2), dtype=torch.float32,
                       device="cuda:0")
    out = torch.empty_like(grid)
    acc = torch.zeros((2, cfg.n_chan, cfg.n_pol ** 2, st.ny, st.nx, 2), dtype=torch.float32,
                      device="cuda:0")
    img = torch.empty_like(acc[0])
    bv = 2 if cfg.volt_type == W.CI8 else 8

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = 1e30
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    res = {}
    ms = timed(lambda: epic.grid_voltages(common, station, 0, nt, grid))
    b = cfg.n_chan * nt * st.n_elem * cfg.n_pol * bv + field_bytes
    res["grid_voltages"] = {"ms": round(ms, 3), "bound": "hbm", "bytes": b,
                            "achieved": round(b / ms / 1e6, 1), "unit": "GB/s",
                            "frac": round(b / ms / 1e6 / PEAK_HBM_GBS, 4)}
    ms = timed(lambda: epic.fft2_batched(st.nx, st.ny, batch, epic.FP32_FFT, grid, out))
    b = 2 * field_bytes
    res["fft2_batched_fp32"] = {"ms": round(ms, 3), "bound": "hbm", "bytes": b,
                                "achieved": round(b / ms / 1e6, 1), "unit": "GB/s",
                                "frac": round(b / ms / 1e6 / PEAK_HBM_GBS, 4)}
    # the dense DFT-matrix products: planes non-zero everywhere (the gridded
    # planes are zero outside the footprint, and the 128 x 128 transform skips
    # all-zero tiles, which the dense flop count would not reflect)
    dense = torch.randn_like(grid)
    for name, p in (("fp16", epic.FP16_SPLIT), ("bf16", epic.BF16_SPLIT)):
        ms = timed(lambda: epic.fft2_batched(st.nx, st.ny, batch, p, dense, out))
        fl = batch * 3 * 8 * (st.ny ** 2 * st.nx + st.nx ** 2 * st.ny)
        res[f"fft2_batched_{name}_split"] = {
            "ms": round(ms, 3), "bound": "mfma", "flops": fl,
            "achieved": round(fl / ms / 1e9, 1), "unit": "TFLOP/s",
            "frac": round(fl / ms / 1e9 / PEAK_FP16_MFMA_TFLOPS, 4)}
    del dense
    ms = timed(lambda: epic.accumulate_power(cfg.n_pol, st.nx, st.ny, cfg.n_chan, nt, out, acc[0],
                                             acc[1], nt, img))
    b = field_bytes + 5 * cfg.n_chan * cfg.n_pol ** 2 * npix * 8
    res["accumulate_power"] = {"ms": round(ms, 3), "bound": "hbm", "bytes": b,
                               "achieved": round(b / ms / 1e6, 1), "unit": "GB/s",
                               "frac": round(b / ms / 1e6 / PEAK_HBM_GBS, 4)}
    # the FFT-correlator output of the accumulated images (one inverse transform
    # per channel and product, once per cadence)
    ms = timed(lambda: epic.image_to_visibilities(cfg.n_pol, st.nx, st.ny, cfg.n_chan, img, acc[1]))
    b = 2 * cfg.n_chan * cfg.n_pol ** 2 * npix * 8
    res["image_to_visibilities"] = {"ms": round(ms, 3), "bound": "hbm", "bytes": b,
                                    "achieved": round(b / ms / 1e6, 1), "unit": "GB/s",
                                    "frac": round(b / ms / 1e6 / PEAK_HBM_GBS, 4)}
    # incoherent combination (Eq. 7) of 8 station images on this sky grid,
    # with per-pixel weights (8 distinct copies of the image stand in for the
    # stations, so that every byte comes from HBM)
    n_st = 8
    copies = img.unsqueeze(0).repeat(n_st, *([1] * img.dim()))
    wts = torch.ones((n_st, cfg.n_pol ** 2, st.ny, st.nx), dtype=torch.float32, device="cuda:0")
    ms = timed(lambda: epic.combine_incoherent(cfg.n_pol, st.nx, st.ny, cfg.n_chan,
                                               [copies[m] for m in range(n_st)], acc[1], wts))
    plane = cfg.n_pol ** 2 * npix
    b = (n_st + 1) * cfg.n_chan * plane * 8 + n_st * plane * 4
    res["combine_incoherent_8"] = {"ms": round(ms, 3), "bound": "hbm", "bytes": b,
                                   "achieved": round(b / ms / 1e6, 1), "unit": "GB/s",
                                   "frac": round(b / ms / 1e6 / PEAK_HBM_GBS, 4)}
    del wts, copies
    # gridding with full polarimetric complex kernels (seeded random 2x2 pol
    # mixing on the K x K cells; algorithmic bytes: voltages, kernel table and
    # grid, each once)
    K = st.support
    kern = torch.randn((cfg.n_chan, st.n_elem, cfg.n_pol, cfg.n_pol, K, K, 2), device="cuda:0",
                       generator=torch.Generator(device="cuda:0").manual_seed(cfg.seed))
    ms = timed(lambda: epic.grid_voltages_pol(common, station, kern, 0, nt, grid))
    b = cfg.n_chan * nt * st.n_elem * cfg.n_pol * bv + kern.numel() * 4 + field_bytes
    res["grid_voltages_pol"] = {"ms": round(ms, 3), "bound": "hbm", "bytes": b,
                                "achieved": round(b / ms / 1e6, 1), "unit": "GB/s",
                                "frac": round(b / ms / 1e6 / PEAK_HBM_GBS, 4)}
    del kern
    res.update(xfft_stages(cfg, common, station, timed))
    res["_block"] = f"{cfg.n_chan} channels x {nt} samples x {cfg.n_pol} pols of {st.nx}x{st.ny}"
    del grid, out, acc, img
    torch.cuda.empty_cache()
    return res


def xfft_stages(cfg, common, station, timed):
    """The XFFT route (Sec. 5.4) on the whole cadence of the first station:
    the correlator of Eq. 4 against the matrix-core roofline of its dtype
    (algorithmic ops: 8 per complex product, over the R (R + 1) / 2 distinct
    entries of each channel's Hermitian matrix, R = n_elem * n_pol), the
    gridding of Eq. 6 plus the transform against HBM (algorithmic bytes: the
    visibilities read once and the image written once), and the route's
    image rate in the headline's unit (it returns the same image)."""
    import torch
    from paper_2411_17804_amd import epic
    st = cfg.stations[0]
    R = st.n_elem * cfg.n_pol
    vis_bytes = cfg.n_chan * R * R * 8
    if vis_bytes > (64 << 30):
        return {"xfft": f"skipped: the visibility matrices take {vis_bytes / 2**30:.0f} GiB"}
    vis = torch.empty((cfg.n_chan, st.n_elem, cfg.n_pol, st.n_elem, cfg.n_pol, 2),
                      dtype=torch.float32, device="cuda:0")
    ms_c = timed(lambda: epic.xfft_correlate(common, station, vis))
    ms_i = timed(lambda: epic.xfft_image(common, station, vis))
    ops = cfg.n_chan * R * (R + 1) // 2 * cfg.n_time * 8
    i8 = cfg.volt_type == W.CI8
    peak = PEAK_INT8_MFMA_TOPS if i8 else PEAK_FP32_MFMA_TFLOPS
    img_bytes = cfg.n_chan * cfg.n_pol ** 2 * st.nx * st.ny * 8
    out = {
        "xfft_correlate": {"ms": round(ms_c, 3), "bound": "mfma", "dtype": "i8" if i8 else "f32",
                           "ops": ops, "achieved": round(ops / ms_c / 1e9, 1),
                           "unit": "TOP/s" if i8 else "TFLOP/s",
                           "frac": round(ops / ms_c / 1e9 / peak, 4)},
        "xfft_image": {"ms": round(ms_i, 3), "bound": "hbm", "bytes": vis_bytes + img_bytes,
                       "achieved": round((vis_bytes + img_bytes) / ms_i / 1e6, 1), "unit": "GB/s",
                       "frac": round((vis_bytes + img_bytes) / ms_i / 1e6 / PEAK_HBM_GBS, 4)},
        "xfft_route": {"ms": round(ms_c + ms_i, 3),
                       "pixel_samples_per_s": cfg.n_chan * cfg.n_time * st.nx * st.ny / (ms_c + ms_i) * 1e3,
                       "cadence": f"{cfg.n_chan} channels x {cfg.n_time} samples"},
    }
    del vis
    torch.cuda.empty_cache()
    return out


def array_stage(cfg, reps=2):
    """Coherent inter-station EPIC (Eq. 10 then Eq. 9) on a synthetic array of
    16 copies of the first station (centres in a 300 m circle, 45 m apart):
    4 channels x 256 samples, every beam pixel, array grid 32 x 32 at half the
    station diameter, nearest-cell gridding.  Station fields come from
    grid_voltages + fft2_batched (timed as beam formation); array_cadence (the
    EPIC route at array scale) and array_xfft (the XFFT route) are timed on
    their own; the rate is array-grid pixel-samples per second of the EPIC
    route."""
    import torch
    from paper_2411_17804_amd import epic
    st = cfg.stations[0]
    n_st, n_ch, nt = 16, 4, 256
    lams = cfg.wavelengths_m[:n_ch]
    cen = W.array_centres(n_st, 300.0, 45.0, cfg.seed)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(cfg.seed)
    common_s = epic.Common(cfg.n_pol, lams, W.GRID_SPACING_WL, nt, cfg.volt_type, epic.FP32_FFT)
    bv = 2 if cfg.volt_type == W.CI8 else 8
    beams, volts = [], []
    for m in range(n_st):
        if cfg.volt_type == W.CI8:
            v = torch.randint(-48, 48, (n_ch, nt, st.n_elem, cfg.n_pol, 2), dtype=torch.int8,
                              device="cuda:0", generator=gen)
        else:
            v = torch.randn((n_ch, nt, st.n_elem, cfg.n_pol, 2), device="cuda:0", generator=gen)
        volts.append(v)
        beams.append(torch.empty((n_ch, nt, cfg.n_pol, st.ny, st.nx, 2), dtype=torch.float32,
                                 device="cuda:0"))

    def form():
        for m in range(n_st):
            s_m = epic.Station(st.pos_m, st.nx, st.ny, st.kernel_type, st.support, st.sigma_cells,
                               volts=volts[m])
            epic.grid_voltages(common_s, s_m, 0, nt, beams[m])
            epic.fft2_batched(st.nx, st.ny, n_ch * nt * cfg.n_pol, epic.FP32_FFT, beams[m], beams[m])

    na = 32
    dA = 0.5 * 2.0 * float(np.max(np.linalg.norm(st.pos_m, axis=1))) / float(lams.max())
    pix = np.arange(st.nx * st.ny, dtype=np.int32)
    img = torch.empty((n_ch, pix.size, cfg.n_pol ** 2, na, na, 2), dtype=torch.float32, device="cuda:0")
    common_a = epic.Common(cfg.n_pol, lams, dA, nt, W.CF32, epic.FP32_FFT)
    arr = epic.Station(cen, na, na, W.KERNEL_NEAREST, 1, 0.0, image=img)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    ms_b = timed(form)
    ms_a = timed(lambda: epic.array_cadence(common_a, arr, beams, st.nx, st.ny, pix))
    ms_x = timed(lambda: epic.array_xfft(common_a, arr, beams, st.nx, st.ny, pix))
    problems = n_ch * pix.size
    out = {"stations": n_st, "channels": n_ch, "samples": nt, "beam_pixels": int(pix.size),
           "array_grid": na, "array_spacing_wl": round(dA, 3),
           "beam_formation_ms": round(ms_b, 3), "array_cadence_ms": round(ms_a, 3),
           "array_pixel_samples_per_s": problems * nt * na * na / ms_a * 1e3,
           "array_xfft_ms": round(ms_x, 3),
           "voltage_bytes": n_st * n_ch * nt * st.n_elem * cfg.n_pol * bv}
    del beams, volts, img
    torch.cuda.empty_cache()
    return out


def cpu_baseline(cfg, stations, host_volts, n_sample_chan):
    """Time the FP64 oracle on a bounded sample (the first station, a spread of
    channels, every sample of the cadence) and check the GPU images there."""
    import oracle
    import torch
    threads = min(16, os.cpu_count() or 1)
    s = 0
    st = cfg.stations[s]
    n = min(n_sample_chan, cfg.n_chan)
    chans = np.unique(np.linspace(0, cfg.n_chan - 1, n).astype(int))
    v = host_volts[s][chans]
    log(f"cpu_baseline: oracle on {len(chans)} channels x {cfg.n_time} samples, {threads} threads")
    t0 = time.perf_counter()
    ref = oracle.image(st.pos_m, cfg.wavelengths_m[chans], W.GRID_SPACING_WL, st.nx, st.ny,
                       st.kernel_type, st.support, st.sigma_cells, v, n_threads=threads)
    dt = time.perf_counter() - t0
    a = stations[s].image[torch.as_tensor(chans, device=stations[s].image.device)].cpu().numpy()
    got = a[..., 0].astype(np.float64) + 1j * a[..., 1]
    err = oracle.image_error(got, ref, cfg.n_pol)
    px = st.nx * st.ny * len(chans) * cfg.n_time
    log(f"cpu_baseline: {dt:.1f} s, worst GPU error on the sample {err.max():.2e}")
    return {"value": px / dt, "unit": "pixel-samples/s", "cores": threads, "kind": "oracle",
            "sample": f"station 0, {len(chans)} of {cfg.n_chan} channels (evenly spread), all "
                      f"{cfg.n_time} samples; C99 FP64 oracle, OpenMP over channels",
            "seconds": round(dt, 2), "gpu_max_error_on_sample": float(err.max())}


if __name__ == "__main__":
    main()
