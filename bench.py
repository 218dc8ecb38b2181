#!/usr/bin/env python3
"""Throughput of the EPIC imager hot path on one MI355X.

A step is one whole cadence through image_cadence: every station, channel and
time sample of the workload is gridded, transformed, squared and averaged
(Eq. 3 then Eq. 2).  The default workload is the hierarchical layout, the
largest that fits one GPU: 96 stations of 64-1024 elements (uniform counts)
at the density of an SKA-low-like station, each on a 32x32, 64x64 or 128x128
grid chosen by its footprint, 3x3 Gaussian kernel, 2 pols, 64 channels, 1024
samples per cadence, int8 complex voltages (sigma 16).  It is timed with the
FP16-split DFT-GEMM transform (its own precision) and with the FP32 FFT, in
the same run, on the same resident voltages.  Inputs are seeded, synthetic
and already resident in HBM when the timed region starts.

Prints one JSON line: grid pixel-samples/s (sum over stations of
nx*ny*n_chan*n_time per cadence, divided by the cadence time) of the first
precision, the other under "precisions", the roofline of each precision's
dominant kernel (algorithmic work per launch over its launch duration, timed
live with HIP events on its launch stream), the worst error of each against
the FP64 CPU oracle on a bounded sample, and that oracle's own throughput.
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
_PERSISTENT = ["accum.hpp", "queue.hpp", "lds_sync.hpp", "volts.hpp"]
KERNEL_SOURCES = {
    "fused_fft_cadence": ["k_fused.hip", "fft_lds.hpp"] + _PERSISTENT,
    "fused_fft128_cadence": ["k_fused128.hip", "fft_lds.hpp"] + _PERSISTENT,
    "fused_dft_cadence": ["k_fused_dft.hip", "mfma_split.hpp"] + _PERSISTENT,
    "fused_dft128_cadence": ["k_fused_dft128.hip", "mfma_split.hpp"] + _PERSISTENT,
    "dft2_tiles128": ["k_dft.hip", "mfma_split.hpp"],
    "grid_gather": ["k_grid.hip", "volts.hpp"],
    "fft_rows": ["k_fft.hip", "fft_lds.hpp"],
    "fft_cols": ["k_fft.hip", "fft_lds.hpp"],
}


def source_hash(kernel: str):
    """First 16 hex digits of the SHA-256 of a timed kernel's source files."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        p = os.path.join(ROOT, "paper_2411_17804_amd", "csrc", f)
        if not os.path.exists(p):
            return None
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, flush):
    """HBM bytes per launch from profiles/<kernel>_<workload>_hbm_bytes.md, or
    None if there is no summary, the kernel changed since it was taken, or it
    was taken with another flush interval (the FP64 running-sum updates scale
    with 1/flush)."""
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_bytes.md")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    text = open(path).read()
    m_b = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    m_h = re.search(r"source_sha256_16: ([0-9a-f]+)", text)
    m_f = re.search(r"flush: (\d+|none)", text)
    if not (m_b and m_h and m_f):
        return None
    if m_f.group(1) != "none" and (flush is None or int(m_f.group(1)) != flush):
        return None
    return int(m_b.group(1)) if source_hash(kernel) == m_h.group(1) else None


def box_sides(cfg, st):
    """Footprint box sides (bw, bh) in cells of one station at every channel,
    placed exactly as the plan places them: nearest cell floor(u + 1/2) of
    every element, widened by the kernel's half support."""
    h = (st.support - 1) // 2
    out = []
    for lam in cfg.wavelengths_m:
        d = W.GRID_SPACING_WL * lam
        ci = np.floor(st.pos_m[:, 0] / d + st.nx // 2 + 0.5)
        cj = np.floor(st.pos_m[:, 1] / d + st.ny // 2 + 0.5)
        out.append((int(ci.max() - ci.min()) + 2 * h + 1, int(cj.max() - cj.min()) + 2 * h + 1))
    return out


def fft_flops_per_pixel_sample(cfg, st, with_grid=True):
    """Algorithmic FP32 work per grid pixel-sample of the FFT path, with the
    paper's FLOP constants (a complex multiply 6, a complex add 2, Sec. 3):
    transform 5 log2(N^2) per pol (5 N log2 N per N-point transform), squaring
    6 n_p^2 and accumulation 2 n_p^2 per pixel (Table 2), gridding 4 per tap
    and pol (complex value times real weight, added).  C2: 156.5."""
    npix = st.nx * st.ny
    fft = cfg.n_pol * 5.0 * math.log2(npix)
    grid = 4.0 * st.n_elem * st.support ** 2 * cfg.n_pol / npix if with_grid else 0.0
    return fft + grid + 8.0 * cfg.n_pol ** 2


def split_flops_per_sample_pol(cfg, st):
    """Algorithmic matrix-core work of the split-precision 2-D DFT-GEMM of one
    station, per (sample, pol), summed over the channels: Z = F_y X F_x^T
    pruned to the footprint (the y stage reads the f_y footprint rows, the x
    stage the f_x columns), complex entries as 2 x 2 real blocks (8 flop per
    complex multiply-add), three split products per stage:
    24 N f_x (f_y + N) for an N x N grid (48 N^3 dense)."""
    n = st.nx
    return sum(24.0 * n * bw * (bh + n) for bw, bh in box_sides(cfg, st))


# Kernels the bench can put on a roofline: timer name -> (bound, stations the
# kernel serves, algorithmic work of one cadence over those stations).
def _fft_work(cfg, stations, with_grid=True):
    return sum(fft_flops_per_pixel_sample(cfg, s, with_grid) * s.nx * s.ny * cfg.n_chan * cfg.n_time
               for s in stations)


def _split_work(cfg, stations):
    return sum(split_flops_per_sample_pol(cfg, s) * cfg.n_time * cfg.n_pol for s in stations)


def _grid_bytes(cfg, stations, rows_only=False):
    """Gridding: voltages read once, every written cell once per (sample, pol)."""
    bv = 2 if cfg.volt_type == W.CI8 else 8
    total = 0
    for s in stations:
        for bw, bh in box_sides(cfg, s):
            cells = s.nx * bh if rows_only else s.nx * s.ny
            total += cfg.n_time * cfg.n_pol * (s.n_elem * bv + cells * 8)
    return total


def _plane_pass_bytes(cfg, stations, cols):
    """One pass of the composed FP32 transform (FP32 complex values): the row
    pass reads and writes the footprint box's rows of every plane (the rest
    is zero and stays untouched), the column pass reads those rows and writes
    whole planes."""
    total = 0
    for s in stations:
        for bw, bh in box_sides(cfg, s):
            rows = min(bh, s.ny)
            total += cfg.n_time * cfg.n_pol * 8 * s.nx * (rows + (s.ny if cols else rows))
    return total


def _power_bytes(cfg, stations, launches):
    acc = sum(cfg.n_chan * cfg.n_pol ** 2 * s.nx * s.ny * 8 for s in stations)
    field = sum(cfg.n_chan * cfg.n_time * cfg.n_pol * s.nx * s.ny * 8 for s in stations)
    return field + launches * 4 * acc / max(1, len(stations)) + acc


ROOFLINE_KERNELS = {
    # FP32 path, fused: gridding, transform, products and accumulation in one kernel
    "fused_fft_cadence": ("alu", lambda s: s.nx <= 64, lambda c, st, n: _fft_work(c, st)),
    "fused_cadence": ("alu", lambda s: s.nx <= 128, lambda c, st, n: _fft_work(c, st)),
    # FP32 128 x 128: gridding into footprint boxes, transform, products
    "fused_fft128_cadence": ("alu", lambda s: s.nx == 128, lambda c, st, n: _fft_work(c, st)),
    # split precision, fused (N <= 64) and the 128 x 128 plane transform
    "fused_dft_cadence": ("mfma", lambda s: s.nx <= 64, lambda c, st, n: _split_work(c, st)),
    "fused_dft128_cadence": ("mfma", lambda s: s.nx == 128, lambda c, st, n: _split_work(c, st)),
    "dft2_tiles128": ("mfma", lambda s: s.nx == 128, lambda c, st, n: _split_work(c, st)),
    "dft_gemm_pass": ("mfma", lambda s: s.nx == 256, lambda c, st, n: _split_work(c, st)),
    # HBM-bound stages of the composed path
    "grid_gather": ("hbm", lambda s: True,
                    lambda c, st, n: _grid_bytes(c, st, rows_only=all(s.nx >= 128 for s in st))),
    "square_accumulate": ("hbm", lambda s: True, lambda c, st, n: _power_bytes(c, st, n)),
    # the composed FP32 path's row and column passes (256 x 256 planes)
    "fft_rows": ("hbm", lambda s: s.nx > 128, lambda c, st, n: _plane_pass_bytes(c, st, False)),
    "fft_cols": ("hbm", lambda s: s.nx > 128, lambda c, st, n: _plane_pass_bytes(c, st, True)),
}

PEAKS = {"alu": (PEAK_FP32_VALU_TFLOPS, "TFLOP/s"), "mfma": (PEAK_FP16_MFMA_TFLOPS, "TFLOP/s"),
         "hbm": (PEAK_HBM_GBS, "GB/s")}


def roofline(cfg, kern, steps, prec, tuned, traffic_ok):
    """Roofline of the kernel that takes the most time per step: its
    algorithmic work per launch (the work of the stations it serves per
    cadence, divided by its launches per cadence) over its average launch
    duration, both measured with HIP events on its launch stream."""
    dom_name, (dom_count, dom_ms) = max(kern.items(), key=lambda kv: kv[1][1])
    avg_ms = dom_ms / dom_count
    per_step = dom_count / steps
    out = {"kernel": dom_name, "avg_launch_ms": round(avg_ms, 4),
           "launches_per_step": round(per_step, 2)}
    if dom_name not in ROOFLINE_KERNELS:
        out.update({"bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                    "traffic": None})
        return out
    bound, serves, work_fn = ROOFLINE_KERNELS[dom_name]
    served = [s for s in cfg.stations if serves(s)] or cfg.stations
    work = work_fn(cfg, served, per_step) / per_step
    peak, unit = PEAKS[bound]
    scale = 1e9 if unit == "GB/s" else 1e12
    achieved = work / (avg_ms / 1e3) / scale
    # the flush interval of the kernel's classes (the tuned value, else the default 16)
    prefix = {"fused_fft_cadence": "fft_n", "fused_fft128_cadence": "fft128_",
              "fused_dft_cadence": "dft_n", "fused_dft128_cadence": "dft_n128"}.get(dom_name)
    fl = sorted({v for k, v in tuned.items() if prefix and k.startswith(prefix) and ":" not in k
                 and (dom_name != "fused_dft_cadence" or not k.startswith("dft_n128"))})
    flush = fl[0] if len(fl) == 1 else (16 if not fl else None)
    out.update({"bound": bound, "achieved": round(achieved, 3), "peak": round(peak, 1), "unit": unit,
                "frac": round(achieved / peak, 4),
                "traffic": measured_traffic(dom_name, f"C{cfg.index}", flush) if traffic_ok else None,
                "work_per_launch": work, "flush": flush if prefix else None})
    if bound == "alu":
        out["flop_per_pixel_sample"] = round(
            work * per_step / sum(s.nx * s.ny * cfg.n_chan * cfg.n_time for s in served), 2)
        out["peak_note"] = ("FP32 vector FMA without packed FP32 (256 CU x 64 lanes x 2 flop x "
                            "2.4 GHz); the published 157.3 TFLOP/s counts packed FP32, which "
                            "this library is built without")
        out["frac_of_157_3"] = round(achieved / 157.3, 4)
    return out


def time_precision(cfg, prec_name, common, stations, steps, warmup, autotune):
    """Autotune, warm up, then time `steps` whole cadences (graph replays as
    the library runs them); then the same steps again with every kernel
    bracketed by HIP events on its launch stream, for per-kernel durations."""
    import torch
    from paper_2411_17804_amd import epic
    tune_file = os.environ["EPIC_TUNE_CACHE"]
    tuned = {}
    if autotune:
        t_tune = time.time()
        epic.autotune(common, stations)
        log(f"{prec_name}: autotune done in {time.time() - t_tune:.1f} s")
        if os.path.exists(tune_file):
            # "class variant flush" lines
            for line in open(tune_file):
                parts = line.split()
                if len(parts) == 3:
                    tuned[parts[0]] = int(parts[2])
                    tuned[parts[0] + ":variant"] = int(parts[1])
    for _ in range(warmup):
        epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    epic.timing_reset()
    epic.timing_enable(True)
    for _ in range(steps):
        epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    epic.timing_enable(False)
    kern = epic.timing_report()
    log(f"{prec_name}: {ms:.2f} ms/step; tuned {tuned}; kernels {kern}")
    return ms, kern, tuned


def cpu_sample(cfg):
    """The bounded sample the oracle is timed and checked on: for one station,
    a spread of channels sized to ~10-30 s of host work; for a hierarchical
    layout, 8 stations spanning its grid sizes and element counts, 8 channels
    each.  Every sample of the cadence is kept (the image is its mean)."""
    if len(cfg.stations) == 1:
        n = {1: 4, 2: 192, 3: 12, 5: 4}.get(cfg.index, 4)
        chans = np.unique(np.linspace(0, cfg.n_chan - 1, min(n, cfg.n_chan)).astype(int))
        return [(0, chans)]
    picks = []
    for grid, k in ((128, 3), (64, 3), (32, 2)):
        idx = sorted((i for i, s in enumerate(cfg.stations) if s.nx == grid),
                     key=lambda i: cfg.stations[i].n_elem)
        if idx:
            picks += [idx[int(round(j))] for j in np.linspace(0, len(idx) - 1, min(k, len(idx)))]
    chans = np.unique(np.linspace(0, cfg.n_chan - 1, min(8, cfg.n_chan)).astype(int))
    return [(s, chans) for s in dict.fromkeys(picks)]


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = min(aff, int(omp)) if omp and omp.isdigit() and int(omp) > 0 else aff
    return {"nproc": os.cpu_count(), "affinity_cpus": aff, "omp_num_threads": omp,
            "cpu_model": model, "threads": threads}


def source_info():
    import hashlib
    import subprocess
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_17804_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    try:
        git = subprocess.run(["git", "-C", ROOT, "rev-parse", "HEAD"], capture_output=True,
                             text=True, timeout=10).stdout.strip() or None
    except (OSError, subprocess.SubprocessError):
        git = None
    return {"git_head": git, "csrc_sha256_16": h.hexdigest()[:16]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=4,
                    help="workload C1..C5 (default C4, the hierarchical layout: the largest "
                         "that fits one GPU)")
    ap.add_argument("--precision", choices=sorted(PREC_NAMES) + ["both", "all"], default="both",
                    help="both: the workload's own precision and the other of fp32/fp16-split "
                         "(the metric's comparison); all: fp32, fp16 and bf16 split")
    ap.add_argument("--n-chan", type=int, default=None, help="shrink the band (testing)")
    ap.add_argument("--n-time", type=int, default=None, help="shrink the cadence (testing)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile parameters of the fused kernels")
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

    cfg = W.make_config(args.config, n_chan=args.n_chan, n_time=args.n_time)
    own = {W.FP32_FFT: "fp32", W.FP16_SPLIT: "fp16", W.BF16_SPLIT: "bf16"}[cfg.precision]
    if args.precision == "both":
        precs = [own, "fp16" if own == "fp32" else "fp32"]
    elif args.precision == "all":
        precs = [own] + [p for p in ("fp32", "fp16", "bf16") if p != own]
    else:
        precs = [args.precision]
    log(f"workload C{cfg.index}: {len(cfg.stations)} station(s), {cfg.n_chan} channels x "
        f"{cfg.n_time} samples, precisions {precs}")
    t_gen = time.time()
    vdev = []
    sample = cpu_sample(cfg) if not args.no_cpu_baseline else []
    host_volts = {}
    want = {s for s, _ in sample}
    hi = host_info()
    for s in range(len(cfg.stations)):
        v = W.station_volts(cfg, s, threads=hi["threads"])
        if s in want:
            host_volts[s] = v
        vdev.append(torch.from_numpy(v if v.dtype == np.int8 else v.view(np.float32)).to(dev))
        del v
    torch.cuda.synchronize()
    log(f"inputs generated and resident in HBM ({cfg.volt_bytes() / 1e9:.2f} GB) "
        f"in {time.time() - t_gen:.1f} s")

    tune_file = os.environ.get("EPIC_TUNE_CACHE")
    if not tune_file:
        import tempfile
        tune_file = os.path.join(tempfile.mkdtemp(prefix="epic_bench_"), "tune.txt")
        os.environ["EPIC_TUNE_CACHE"] = tune_file

    pix = cfg.pixel_samples()
    full = cfg.n_chan == W.make_config(cfg.index).n_chan and args.n_time is None
    results = {}
    images = {}
    for p in precs:
        common = epic.Common(cfg.n_pol, cfg.wavelengths_m, W.GRID_SPACING_WL, cfg.n_time,
                             cfg.volt_type, PREC_NAMES[p])
        stations = []
        for s, st in enumerate(cfg.stations):
            img = torch.zeros((cfg.n_chan, cfg.n_pol * cfg.n_pol, st.ny, st.nx, 2),
                              dtype=torch.float32, device=dev)
            stations.append(epic.Station(st.pos_m, st.nx, st.ny, st.kernel_type, st.support,
                                         st.sigma_cells, volts=vdev[s], image=img))
        ms, kern, tuned = time_precision(cfg, p, common, stations, args.steps, args.warmup,
                                         not args.no_autotune)
        value = pix / (ms / 1e3)
        results[p] = {
            "value": value, "ms_per_step": ms,
            "realtime_factor": (cfg.n_time * 25e-6) / (ms / 1e3),
            "roofline": roofline(cfg, kern, args.steps, p, tuned, full),
            "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in kern.items()},
            "launches_per_step": round(sum(v[0] for v in kern.values()) / args.steps, 1),
            "tuned": tuned,
        }
        # keep the sampled stations' images for the error check; free the rest
        images[p] = {s: stations[s].image[torch.as_tensor(ch, device=dev)].cpu().numpy()
                     for s, ch in sample}
        del stations
        epic.cache_clear()
        torch.cuda.empty_cache()

    dtype_name = {"fp32": "f32", "fp16": "f16x3+f32acc", "bf16": "bf16x3+f32acc"}
    head = results[precs[0]]
    workload = {
        1: "C1: 64 el in a 16 m square, 32x32 grid, nearest, 1 pol, cf32, 4 ch x 256",
        2: "C2: station of 256 el in a 38 m circle, 64x64 grid, 3x3 Gaussian, 2 pols, ci8, 1024 ch x 2048",
        3: "C3: dense 64x32 lattice, 128x128 grid, 3x3 Gaussian, 2 pols, cf32, 256 ch x 4096",
        4: "C4: 96 stations of 64-1024 el, 32/64/128 grids by footprint, 3x3 Gaussian, 2 pols, ci8, 64 ch x 1024",
        5: "C5: 128x128 lattice less 5%, 256x256 grid, 5x5 Gaussian, 2 pols, cf32, 128 ch x 512"}[cfg.index]
    out = {
        "metric": "grid pixel-samples/s per GPU",
        "value": head["value"],
        "unit": "pixel-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name[precs[0]],
        "data": "synthetic (seeded layouts and voltages shaped like the paper's arrays)",
        "config": {"workload": workload, "n_chan": cfg.n_chan, "n_time": cfg.n_time,
                   "n_stations": len(cfg.stations), "precision": precs[0],
                   "pixel_samples_per_step": pix, "realtime_factor": head["realtime_factor"],
                   "seed": cfg.seed},
        "roofline": head["roofline"],
        "precisions": {p: {k: v for k, v in r.items()} for p, r in results.items()},
    }
    if "fp16" in results and "fp32" in results:
        out["fp16_split_vs_fp32"] = round(results["fp16"]["value"] / results["fp32"]["value"], 4)

    if not args.no_stages:
        s0 = next(i for i, s in enumerate(cfg.stations) if s.nx <= 128)
        st0 = cfg.stations[s0]
        c0 = epic.Common(cfg.n_pol, cfg.wavelengths_m, W.GRID_SPACING_WL, cfg.n_time,
                         cfg.volt_type, cfg.precision)
        img0 = torch.zeros((cfg.n_chan, cfg.n_pol * cfg.n_pol, st0.ny, st0.nx, 2),
                           dtype=torch.float32, device=dev)
        station = epic.Station(st0.pos_m, st0.nx, st0.ny, st0.kernel_type, st0.support,
                               st0.sigma_cells, volts=vdev[s0], image=img0)
        out["stages"] = stage_rooflines(cfg, c0, station, s0)
        if len(cfg.stations) == 1:
            out["stages"]["inter_station_epic"] = array_stage(cfg)
        log(f"stages: {out['stages']}")
    if sample:
        out["cpu_baseline"], errs = cpu_baseline(cfg, sample, host_volts, images, hi)
        for p, e in errs.items():
            out["precisions"][p]["worst_error_on_cpu_sample"] = e
    out["host"] = hi
    out["source"] = source_info()
    print(json.dumps(out), flush=True)


def stage_rooflines(cfg, common, station, s_idx=0, nt=64, reps=3):
    """Each unfused stage on a block of nt samples of every channel of one
    station (index s_idx), timed with events on the current stream, against
    the roofline that bounds it (algorithmic bytes for HBM-bound stages,
    algorithmic matrix-core flops for the DFT-matrix products)."""
    import torch
    from paper_2411_17804_amd import epic
    st = cfg.stations[s_idx]
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
    res.update(xfft_stages(cfg, common, station, timed, s_idx))
    res["_block"] = (f"station {s_idx}: {cfg.n_chan} channels x {nt} samples x {cfg.n_pol} pols "
                     f"of {st.nx}x{st.ny}")
    del grid, out, acc, img
    torch.cuda.empty_cache()
    return res


def xfft_stages(cfg, common, station, timed, s_idx=0):
    """The XFFT route (Sec. 5.4) on the whole cadence of the first station:
    the correlator of Eq. 4 against the matrix-core roofline of its dtype
    (algorithmic ops: 8 per complex product, over the R (R + 1) / 2 distinct
    entries of each channel's Hermitian matrix, R = n_elem * n_pol), the
    gridding of Eq. 6 plus the transform against HBM (algorithmic bytes: the
    visibilities read once and the image written once), and the route's
    image rate in the headline's unit (it returns the same image)."""
    import torch
    from paper_2411_17804_amd import epic
    st = cfg.stations[s_idx]
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
    grid_voltages + fft2_batched (timed as beam formation); array_cadence is
    timed on its own; the rate is array-grid pixel-samples per second."""
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
    problems = n_ch * pix.size
    out = {"stations": n_st, "channels": n_ch, "samples": nt, "beam_pixels": int(pix.size),
           "array_grid": na, "array_spacing_wl": round(dA, 3),
           "beam_formation_ms": round(ms_b, 3), "array_cadence_ms": round(ms_a, 3),
           "array_pixel_samples_per_s": problems * nt * na * na / ms_a * 1e3,
           "voltage_bytes": n_st * n_ch * nt * st.n_elem * cfg.n_pol * bv}
    del beams, volts, img
    torch.cuda.empty_cache()
    return out


def cpu_baseline(cfg, sample, host_volts, images, hi):
    """Time the FP64 oracle on the bounded sample (sample: [(station, channels)],
    every sample of the cadence) with every thread the process may use, and
    once more on one channel of the first sampled station with one thread;
    check every precision's GPU images on the sample against it."""
    import oracle
    threads = hi["threads"]
    errs = {p: 0.0 for p in images}
    px = 0
    dt = 0.0
    desc = []
    for s, chans in sample:
        st = cfg.stations[s]
        v = host_volts[s][chans]
        t0 = time.perf_counter()
        ref = oracle.image(st.pos_m, cfg.wavelengths_m[chans], W.GRID_SPACING_WL, st.nx, st.ny,
                           st.kernel_type, st.support, st.sigma_cells, v, n_threads=threads)
        dt += time.perf_counter() - t0
        px += st.nx * st.ny * len(chans) * cfg.n_time
        desc.append(f"{s}({st.nx}x{st.ny}, {st.n_elem} el)")
        for p, imgs in images.items():
            a = imgs[s]
            got = a[..., 0].astype(np.float64) + 1j * a[..., 1]
            errs[p] = max(errs[p], float(oracle.image_error(got, ref, cfg.n_pol).max()))
    s0, ch0 = sample[0]
    st = cfg.stations[s0]
    t0 = time.perf_counter()
    oracle.image(st.pos_m, cfg.wavelengths_m[ch0[:1]], W.GRID_SPACING_WL, st.nx, st.ny,
                 st.kernel_type, st.support, st.sigma_cells, host_volts[s0][ch0[:1]], n_threads=1)
    dt1 = time.perf_counter() - t0
    px1 = st.nx * st.ny * cfg.n_time
    log(f"cpu_baseline: {dt:.1f} s on {threads} threads ({px / dt:.3e} px-samples/s), 1 thread "
        f"{px1 / dt1:.3e}; worst GPU error on the sample {errs}")
    n_ch = len(sample[0][1])
    return ({"value": px / dt, "unit": "pixel-samples/s", "cores": threads, "kind": "oracle",
             "sample": f"stations {', '.join(desc)} x {n_ch} of {cfg.n_chan} channels (evenly "
                       f"spread) x all {cfg.n_time} samples; C99 FP64 oracle, OpenMP over "
                       f"channels",
             "seconds": round(dt, 2),
             "one_thread": {"value": px1 / dt1, "seconds": round(dt1, 2),
                            "sample": f"station {s0}, channel {int(ch0[0])}, all samples"},
             "nproc": hi["nproc"], "affinity_cpus": hi["affinity_cpus"],
             "cpu_model": hi["cpu_model"]}, errs)


if __name__ == "__main__":
    main()
