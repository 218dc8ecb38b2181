"""GPU parity: every ABI call against the FP64 oracle on the same seeded inputs.

Tolerances (per image, the max-abs error over pixels divided by the image
scale: max |I^{aa}| for auto products, sqrt(max XX max YY) for cross products):
FP32 transform path <= 1e-5.  Stage tests use max-abs error over the max
magnitude of the oracle's result.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import (from_complex, say, station_objects, to_complex, to_device_volts,
                            torch_cuda)

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    t = torch_cuda()
    from paper_2411_17804_amd import epic
    epic.load()
    return t


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# ------------------------------------------------------------------ grid ----
@pytest.mark.parametrize("case", ["C1", "C2", "C2-nearest-ci8", "C3", "C5"])
def test_grid_voltages(torch, case):
    from paper_2411_17804_amd import epic
    say(f"grid_voltages {case}")
    if case == "C1":
        cfg = W.make_config(1, n_time=6)
    elif case.startswith("C2"):
        cfg = W.make_config(2, chan_subset=[0, 17, 1023], n_time=6)
    elif case == "C3":
        cfg = W.make_config(3, chan_subset=[5, 200], n_time=5)
    else:
        cfg = W.make_config(5, chan_subset=[127], n_time=4)
    st = cfg.stations[0]
    ktype, K, sig = st.kernel_type, st.support, st.sigma_cells
    if case == "C2-nearest-ci8":
        ktype, K, sig = W.KERNEL_NEAREST, 1, 0.0
    v = W.station_volts(cfg, 0)
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    station.kernel_type, station.support, station.sigma_cells = ktype, K, sig
    t0, nt = 2, cfg.n_time - 3
    grid = torch.zeros((cfg.n_chan, nt, cfg.n_pol, st.ny, st.nx, 2), dtype=torch.float32,
                       device="cuda")
    epic.grid_voltages(common, station, t0, nt, grid)
    torch.cuda.synchronize()
    got = to_complex(grid)
    for c in range(cfg.n_chan):
        ref = oracle.grid(st.pos_m, cfg.wavelengths_m[c], W.GRID_SPACING_WL, st.nx, st.ny, ktype,
                          K, sig, v[c], t0=t0, nt=nt)
        if case == "C2-nearest-ci8":
            assert np.array_equal(got[c], ref), "integer sums must be exact"
        else:
            assert _rel(got[c], ref) <= 1e-6, (case, c, _rel(got[c], ref))


# ------------------------------------------------------------------- fft ----
FFT_SHAPES = [(16, 16), (32, 32), (64, 64), (128, 128), (256, 256), (32, 16), (16, 64),
              (128, 64), (64, 256), (256, 32), (256, 128)]


@pytest.mark.parametrize("nx,ny", FFT_SHAPES)
def test_fft2_batched_fp32(torch, nx, ny):
    from paper_2411_17804_amd import epic
    say(f"fft2_batched fp32 {nx}x{ny}")
    rng = np.random.default_rng([17804, nx, ny])
    batch = 3
    x = (rng.standard_normal((batch, ny, nx)) + 1j * rng.standard_normal((batch, ny, nx)))
    x = x.astype(np.complex64).astype(np.complex128)
    xin = from_complex(x)
    out = torch.empty_like(xin)
    epic.fft2_batched(nx, ny, batch, epic.FP32_FFT, xin, out)
    torch.cuda.synchronize()
    ref = oracle.fft2(x)
    err = _rel(to_complex(out), ref)
    assert err <= 2e-6, err
    # in place gives the same bits
    epic.fft2_batched(nx, ny, batch, epic.FP32_FFT, xin, xin)
    torch.cuda.synchronize()
    assert torch.equal(xin, out)


# ---------------------------------------------- FFT-correlator output ----
@pytest.mark.parametrize("nx,ny", [(16, 16), (64, 32), (64, 64), (128, 128), (256, 256), (256, 64)])
def test_image_to_visibilities_transform(torch, nx, ny):
    # the inverse transform: (1/N) sum_k x[k] exp(-2 pi i k.j/N) = conj(F(conj x)) / N
    # with F the oracle's + sign transform
    from paper_2411_17804_amd import epic
    say(f"image_to_visibilities {nx}x{ny}")
    rng = np.random.default_rng([17804, 91, nx, ny])
    n_pol, n_chan = 2, 2
    shape = (n_chan, n_pol * n_pol, ny, nx)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    x = x.astype(np.complex128)
    xin = from_complex(x)
    out = torch.empty_like(xin)
    epic.image_to_visibilities(n_pol, nx, ny, n_chan, xin, out)
    torch.cuda.synchronize()
    ref = np.conj(oracle.fft2(np.conj(x).reshape(-1, ny, nx))).reshape(shape) / (nx * ny)
    err = _rel(to_complex(out), ref)
    assert err <= 2e-6, err
    epic.image_to_visibilities(n_pol, nx, ny, n_chan, xin, xin)      # in place: same bits
    torch.cuda.synchronize()
    assert torch.equal(xin, out)


@pytest.mark.parametrize("case", ["C1-full", "C2-2ch"])
def test_fft_correlator_output(torch, case):
    # image_cadence then image_to_visibilities against the visibilities of
    # Eq. 4 gridded directly as in Eq. 6 (no transform on the oracle side)
    from paper_2411_17804_amd import epic
    say(f"FFT-correlator output {case}")
    if case == "C1-full":
        cfg = W.make_config(1, precision=W.FP32_FFT)
    else:
        cfg = W.make_config(2, chan_subset=[5, 900], n_time=24, precision=W.FP32_FFT)
    volts, _, (common, stations) = run_cadence(cfg)
    st, s0 = cfg.stations[0], stations[0]
    vis = torch.empty_like(s0.image)
    epic.image_to_visibilities(cfg.n_pol, st.nx, st.ny, cfg.n_chan, s0.image, vis)
    torch.cuda.synchronize()
    ref = oracle.grid_visibilities(st.pos_m, cfg.wavelengths_m, W.GRID_SPACING_WL, st.nx, st.ny,
                                   st.kernel_type, st.support, st.sigma_cells, volts[0])
    err = oracle.image_error(to_complex(vis), ref, cfg.n_pol)
    say(f"  worst error {err.max():.2e}")
    assert err.max() <= FP32_TOL, err


# ---------------------------------------------- incoherent combination ----
def test_combine_incoherent_weighted(torch):
    from paper_2411_17804_amd import epic
    say("combine_incoherent: 5 stations, per-pixel weights with zeros")
    rng = np.random.default_rng([17804, 93])
    n_st, n_pol, n_chan, ny, nx = 5, 2, 3, 32, 64
    shape = (n_chan, n_pol * n_pol, ny, nx)
    imgs = [(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
            for _ in range(n_st)]
    w = rng.uniform(0.0, 2.0, (n_st, n_pol * n_pol, ny, nx)).astype(np.float32)
    w[:, :, 5, 7] = 0.0                      # a pixel no station sees
    w[1:, 2, :, :] = 0.0                     # one product from station 0 alone
    dev = [from_complex(i.astype(np.complex128)) for i in imgs]
    wd = torch.from_numpy(w).to("cuda:0")
    out = torch.empty_like(dev[0])
    epic.combine_incoherent(n_pol, nx, ny, n_chan, dev, out, wd)
    torch.cuda.synchronize()
    ref = oracle.combine_incoherent([i.astype(np.complex128) for i in imgs], w.astype(np.float64))
    got = to_complex(out)
    assert _rel(got, ref) <= 2e-6, _rel(got, ref)
    assert np.all(got[:, :, 5, 7] == 0)
    # equal weights (NULL), written over the first station's image
    epic.combine_incoherent(n_pol, nx, ny, n_chan, dev, dev[0])
    torch.cuda.synchronize()
    ref = oracle.combine_incoherent([i.astype(np.complex128) for i in imgs])
    assert _rel(to_complex(dev[0]), ref) <= 2e-6


def test_combine_incoherent_after_cadence(torch):
    # three stations imaged on one 64 x 64 sky grid, combined with beam-like
    # weights, against the oracle's images combined in FP64
    from paper_2411_17804_amd import epic
    say("combine_incoherent after image_cadence (C4, three 64x64 stations)")
    cfg = W.make_config(4, chan_subset=[0, 40], n_time=16, n_stations=12, precision=W.FP32_FFT)
    cfg.stations = [s for s in cfg.stations if s.nx == 64][:3]
    assert len(cfg.stations) == 3
    volts, _, (common, stations) = run_cadence(cfg)
    st = cfg.stations[0]
    ky, kx = np.meshgrid(np.fft.fftfreq(st.ny), np.fft.fftfreq(st.nx), indexing="ij")
    w = np.stack([np.broadcast_to(np.exp(-(kx ** 2 + ky ** 2) / (0.1 * (m + 1))), (4, st.ny, st.nx))
                  for m in range(3)]).astype(np.float32)
    out = torch.empty_like(stations[0].image)
    epic.combine_incoherent(2, st.nx, st.ny, cfg.n_chan, [s.image for s in stations], out,
                            torch.from_numpy(np.ascontiguousarray(w)).to("cuda:0"))
    torch.cuda.synchronize()
    ref = oracle.combine_incoherent([oracle_image(cfg, m, volts[m]) for m in range(3)],
                                    w.astype(np.float64))
    err = oracle.image_error(to_complex(out), ref, 2)
    say(f"  worst error {err.max():.2e}")
    assert err.max() <= FP32_TOL, err


# ----------------------------------------------------------------- power ----
@pytest.mark.parametrize("n_pol", [1, 2])
def test_accumulate_power(torch, n_pol):
    from paper_2411_17804_amd import epic
    say(f"accumulate_power n_pol={n_pol}")
    rng = np.random.default_rng([17804, 77, n_pol])
    n_chan, nt, ny, nx = 3, 37, 32, 16
    f = rng.standard_normal((n_chan, nt, n_pol, ny, nx)) + 1j * rng.standard_normal(
        (n_chan, nt, n_pol, ny, nx))
    f = (f * 50).astype(np.complex64).astype(np.complex128)
    fd = from_complex(f)
    shape = (n_chan, n_pol * n_pol, ny, nx, 2)
    s1, c1, img1 = (torch.zeros(shape, device="cuda") for _ in range(3))
    epic.accumulate_power(n_pol, nx, ny, n_chan, nt, fd, s1, c1, nt, img1)
    # the same cadence split over two calls: bit-identical
    s2, c2, img2 = (torch.zeros(shape, device="cuda") for _ in range(3))
    a = 20
    epic.accumulate_power(n_pol, nx, ny, n_chan, a, from_complex(f[:, :a]), s2, c2, 0, None)
    epic.accumulate_power(n_pol, nx, ny, n_chan, nt - a, from_complex(f[:, a:]), s2, c2, nt, img2)
    torch.cuda.synchronize()
    assert torch.equal(img1, img2)
    got = to_complex(img1)
    for c in range(n_chan):
        ref = oracle.power_mean(f[c])
        err = oracle.image_error(got[c], ref, n_pol)
        assert err.max() <= 1e-6, err
    if n_pol == 2:
        assert np.array_equal(got[:, 2], np.conj(got[:, 1]))
        assert np.all(got[:, 0].imag == 0) and np.all(got[:, 3].imag == 0)


# ---------------------------------------------------------- image_cadence ----
def run_cadence(cfg, precision=None):
    from paper_2411_17804_amd import epic
    torch = torch_cuda()
    volts = [W.station_volts(cfg, s) for s in range(len(cfg.stations))]
    common, stations = station_objects(cfg, [to_device_volts(v) for v in volts], precision)
    epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    return volts, [to_complex(s.image) for s in stations], (common, stations)


def oracle_image(cfg, s, v):
    st = cfg.stations[s]
    return oracle.image(st.pos_m, cfg.wavelengths_m, W.GRID_SPACING_WL, st.nx, st.ny,
                        st.kernel_type, st.support, st.sigma_cells, v)


CADENCE_CASES = {
    # name: (config, channel subset, n_time)
    "C1-full": (1, None, None),
    "C2-3ch": (2, [0, 600, 1023], 96),
    "C2-ragged-time": (2, [3], 37),
    "C3-2ch": (3, [0, 255], 12),
    "C3-ragged-blocks": (3, [5, 130, 250], 70),
    "C5-1ch": (5, [64], 3),
}


@pytest.mark.parametrize("case", sorted(CADENCE_CASES))
def test_image_cadence_fp32(torch, case):
    idx, chans, nt = CADENCE_CASES[case]
    say(f"image_cadence fp32 {case}")
    cfg = W.make_config(idx, chan_subset=chans, n_time=nt, precision=W.FP32_FFT)
    volts, imgs, _ = run_cadence(cfg)
    for s in range(len(cfg.stations)):
        ref = oracle_image(cfg, s, volts[s])
        err = oracle.image_error(imgs[s], ref, cfg.n_pol)
        say(f"  {case} station {s}: worst error {err.max():.2e}")
        assert err.max() <= FP32_TOL, err
        if cfg.n_pol == 2:
            assert np.array_equal(imgs[s][:, 2], np.conj(imgs[s][:, 1]))
            assert np.all(imgs[s][:, 0].imag == 0) and np.all(imgs[s][:, 3].imag == 0)


def test_image_cadence_deterministic(torch):
    say("image_cadence determinism C2")
    cfg = W.make_config(2, chan_subset=[1, 2], n_time=64)
    _, a, (common, stations) = run_cadence(cfg)
    from paper_2411_17804_amd import epic
    epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    assert np.array_equal(a[0], to_complex(stations[0].image))


def test_point_source_through_the_gpu_path(torch):
    # a plane wave from pixel (kx', ky') = (5, -3) must peak there (sign pin)
    from paper_2411_17804_amd import epic
    say("image_cadence point source")
    cfg = W.make_config(2, chan_subset=[512], n_time=8)
    st = cfg.stations[0]
    lam = cfg.wavelengths_m[0]
    l, m = 5 / (st.nx * W.GRID_SPACING_WL), -3 / (st.ny * W.GRID_SPACING_WL)
    ph = np.exp(-2j * np.pi * (l * st.pos_m[:, 0] + m * st.pos_m[:, 1]) / lam)
    rng = np.random.default_rng(5)
    A = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    v = (A[:, None, None] * ph[None, :, None] * np.ones((1, 1, 2))).astype(np.complex64)[None]
    cfg.volt_type = W.CF32
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    epic.image_cadence(common, [station])
    torch.cuda.synchronize()
    img = to_complex(station.image)[0, 0].real
    assert np.unravel_index(np.argmax(img), img.shape) == (-3 % st.ny, 5 % st.nx)
    ref = oracle.image(st.pos_m, cfg.wavelengths_m, 0.5, st.nx, st.ny, st.kernel_type, st.support,
                       st.sigma_cells, v)
    assert oracle.image_error(to_complex(station.image), ref, 2).max() <= FP32_TOL


# ------------------------------------------------- split-precision DFT-GEMM ----
SPLIT_TOL = {"fp16": 1e-4, "bf16": 2e-3}   # fp16 is the gate; bf16 is reported with a bound


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("nx,ny", [(16, 16), (32, 64), (64, 64), (128, 128), (256, 256),
                                   (256, 32), (16, 128)])
def test_fft2_batched_split(torch, prec, nx, ny):
    from paper_2411_17804_amd import epic
    say(f"fft2_batched {prec} {nx}x{ny}")
    p = epic.FP16_SPLIT if prec == "fp16" else epic.BF16_SPLIT
    rng = np.random.default_rng([17804, nx, ny, 9])
    batch = 3
    x = rng.standard_normal((batch, ny, nx)) + 1j * rng.standard_normal((batch, ny, nx))
    x[1] *= 3e6            # beyond FP16 range: the per-block power-of-two scale must handle it
    x[2] *= 1e-6
    x = x.astype(np.complex64).astype(np.complex128)
    xin = from_complex(x)
    out = torch.empty_like(xin)
    epic.fft2_batched(nx, ny, batch, p, xin, out)
    torch.cuda.synchronize()
    got = to_complex(out)
    ref = oracle.fft2(x)
    errs = [_rel(got[b], ref[b]) for b in range(batch)]
    say(f"  {prec} {nx}x{ny}: errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= SPLIT_TOL[prec], errs
    # in place
    epic.fft2_batched(nx, ny, batch, p, xin, xin)
    torch.cuda.synchronize()
    assert torch.equal(xin, out)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_fft2_batched_split_sparse_planes(torch, prec):
    # 128 x 128 planes that are zero outside a box: the transform finds the
    # box of non-zero 16 x 16 tiles itself and sums over it only (wide, tall,
    # single-tile, corner-cell, full and all-zero planes in one batch)
    from paper_2411_17804_amd import epic
    say(f"fft2_batched {prec} 128x128 sparse planes")
    p = epic.FP16_SPLIT if prec == "fp16" else epic.BF16_SPLIT
    rng = np.random.default_rng([17804, 128, 21])
    boxes = [(30, 68, 46, 36), (40, 36, 20, 68), (17, 9, 100, 5), (127, 1, 127, 1), (0, 128, 0, 128),
             None]
    x = np.zeros((len(boxes), 128, 128), np.complex128)
    for i, bx in enumerate(boxes):
        if bx is not None:
            x0, bw, y0, bh = bx
            x[i, y0:y0 + bh, x0:x0 + bw] = rng.standard_normal((bh, bw)) + 1j * rng.standard_normal((bh, bw))
    x = x.astype(np.complex64).astype(np.complex128)
    xin = from_complex(x)
    out = torch.empty_like(xin)
    epic.fft2_batched(128, 128, len(boxes), p, xin, out)
    torch.cuda.synchronize()
    got = to_complex(out)
    ref = oracle.fft2(x)
    errs = [_rel(got[b], ref[b]) for b in range(len(boxes) - 1)]
    say(f"  {prec}: errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= SPLIT_TOL[prec], errs
    assert not np.any(got[-1]), "an all-zero plane transforms to zeros"


SPLIT_CASES = {
    "C2-fp16-2ch": (2, [0, 1023], 40, "fp16"),
    "C3-fp16-2ch": (3, [0, 255], 12, "fp16"),
    "C3-bf16-1ch": (3, [100], 8, "bf16"),
    "C5-fp16-1ch": (5, [0], 3, "fp16"),
    "C5-bf16-1ch": (5, [127], 3, "bf16"),
}


@pytest.mark.parametrize("case", sorted(SPLIT_CASES))
def test_image_cadence_split(torch, case):
    idx, chans, nt, prec = SPLIT_CASES[case]
    say(f"image_cadence {case}")
    p = W.FP16_SPLIT if prec == "fp16" else W.BF16_SPLIT
    cfg = W.make_config(idx, chan_subset=chans, n_time=nt, precision=p)
    volts, imgs, _ = run_cadence(cfg)
    for s in range(len(cfg.stations)):
        ref = oracle_image(cfg, s, volts[s])
        err = oracle.image_error(imgs[s], ref, cfg.n_pol)
        say(f"  {case} station {s}: worst error {err.max():.2e}")
        assert err.max() <= SPLIT_TOL[prec], err
        assert np.array_equal(imgs[s][:, 2], np.conj(imgs[s][:, 1]))


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_image_cadence_split_wide_box(torch, prec):
    # C3's lattice stretched to twice its extent along y: the footprint box
    # (about 68 x 70 cells) spans 5 tiles on both sides, the largest box the
    # fused 128 x 128 split kernel takes
    p = W.FP16_SPLIT if prec == "fp16" else W.BF16_SPLIT
    cfg = W.make_config(3, chan_subset=[0, 255], n_time=6, precision=p)
    st = cfg.stations[0]
    st.pos_m = st.pos_m * np.array([1.0, 2.0])
    bw = bh = 0                                  # the largest box over the channels
    for lam in cfg.wavelengths_m:
        cj = np.floor(st.pos_m[:, 1] / (W.GRID_SPACING_WL * lam) + st.ny // 2 + 0.5)
        ci = np.floor(st.pos_m[:, 0] / (W.GRID_SPACING_WL * lam) + st.nx // 2 + 0.5)
        bw = max(bw, int(np.ptp(ci)) + st.support)
        bh = max(bh, int(np.ptp(cj)) + st.support)
    assert min(-(-bw // 16), -(-bh // 16)) > 4 and max(bw, bh) < st.nx, (bw, bh)
    say(f"image_cadence C3 {prec}, largest footprint {bw} x {bh} cells")
    volts, imgs, _ = run_cadence(cfg)
    err = oracle.image_error(imgs[0], oracle_image(cfg, 0, volts[0]), cfg.n_pol)
    say(f"  worst error {err.max():.2e}")
    assert err.max() <= SPLIT_TOL[prec], err


def test_fp32_footprint_rows_small_station(torch, monkeypatch):
    # every 20th element of the C5 lattice (under 1024 elements: the per-row
    # gather) on the 256 x 256 grid, in chunks of 2 samples: only the
    # footprint box's rows are gridded and transformed, and the rows outside
    # it hold the previous chunk's output, which nothing may read
    from paper_2411_17804_amd import epic
    cfg = W.make_config(5, chan_subset=[64], n_time=5, precision=W.FP32_FFT)
    st = cfg.stations[0]
    st.pos_m = st.pos_m[::20]
    assert st.n_elem < 1024
    say(f"image_cadence fp32 256x256, {st.n_elem} elements, chunks of 2 samples")
    v = W.station_volts(cfg, 0)
    monkeypatch.setenv("EPIC_FIELD_BUDGET_MB", "2")
    epic.cache_clear()
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    epic.image_cadence(common, (station,))
    torch.cuda.synchronize()
    err = oracle.image_error(to_complex(station.image), oracle_image(cfg, 0, v), cfg.n_pol)
    say(f"  worst error {err.max():.2e}")
    assert err.max() <= FP32_TOL, err
    monkeypatch.delenv("EPIC_FIELD_BUDGET_MB")
    epic.cache_clear()


def test_fp32_row_pass_in_band_gather_128(torch):
    # the C5 lattice shrunk onto a 128 x 128 grid (15565 elements, a footprint
    # of 106 cells, about 35 taps per cell: row-band tables, more taps per
    # cell than the gather holds in registers, far too many for the fused
    # 128 x 128 kernel, so the composed path): the row-band gather does the
    # row pass of the 128-wide transform itself and only the column pass
    # follows; 13 samples leave a ragged last block of its 8-sample runs
    import bench
    from paper_2411_17804_amd import epic
    cfg = W.make_config(5, chan_subset=[9], n_time=13, precision=W.FP32_FFT)
    st = cfg.stations[0]
    st.pos_m = st.pos_m * 0.8
    st.nx = st.ny = 128
    bw, bh = bench.box_sides(cfg, st)[0]
    assert st.n_elem >= 8192 and max(bw, bh) < 128, (st.n_elem, bw, bh)
    say(f"image_cadence fp32 128x128 composed, {st.n_elem} elements, footprint {bw} x {bh}")
    v = W.station_volts(cfg, 0)
    epic.cache_clear()
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    epic.timing_reset()
    epic.timing_enable(True)
    epic.image_cadence(common, (station,))
    torch.cuda.synchronize()
    epic.timing_enable(False)
    kern = epic.timing_report()
    assert "fft_cols" in kern and "fft_rows" not in kern, kern
    err = oracle.image_error(to_complex(station.image), oracle_image(cfg, 0, v), cfg.n_pol)
    say(f"  worst error {err.max():.2e}")
    assert err.max() <= FP32_TOL, err
    epic.cache_clear()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_one_pol_row_band_station(torch, prec):
    # the C5 station with one pol: the row-band gather with 16-byte slots of
    # one pol (grid_voltages, every row of the plane) and the composed
    # cadence (FP32: the gather does the row pass; FP16-split: the dense
    # DFT-matrix passes), 13 samples for a ragged last run
    import dataclasses
    from paper_2411_17804_amd import epic
    p = W.FP32_FFT if prec == "fp32" else W.FP16_SPLIT
    cfg = dataclasses.replace(W.make_config(5, chan_subset=[40], n_time=13, precision=p), n_pol=1)
    st = cfg.stations[0]
    say(f"one-pol C5 station ({st.n_elem} elements), {prec}")
    v = W.station_volts(cfg, 0)
    epic.cache_clear()
    common, (station,) = station_objects(cfg, [to_device_volts(v)], p)
    grid = torch.zeros((cfg.n_chan, cfg.n_time, 1, st.ny, st.nx, 2), dtype=torch.float32, device="cuda")
    epic.grid_voltages(common, station, 0, cfg.n_time, grid)
    epic.image_cadence(common, (station,))
    torch.cuda.synchronize()
    ref = oracle.grid(st.pos_m, cfg.wavelengths_m[0], W.GRID_SPACING_WL, st.nx, st.ny, st.kernel_type,
                      st.support, st.sigma_cells, v[0], t0=0, nt=cfg.n_time)
    assert _rel(to_complex(grid)[0], ref) <= 1e-6
    err = oracle.image_error(to_complex(station.image), oracle_image(cfg, 0, v), cfg.n_pol)
    say(f"  worst error {err.max():.2e}")
    assert err.max() <= (FP32_TOL if prec == "fp32" else SPLIT_TOL["fp16"]), err
    epic.cache_clear()


@pytest.mark.parametrize("idx,prec", [(3, "fp16"), (5, "bf16"), (5, "fp32")])
def test_composed_cadence_in_chunks(torch, monkeypatch, idx, prec):
    # a field budget of 2 MB splits the composed cadence into chunks of a few
    # samples: the accumulators carry across chunks, and each chunk grids only
    # what its transform reads (the tile region of the split 128 x 128
    # transform, the footprint rows of the two-pass FP32 transform) while the
    # rest of the buffer still holds the previous chunk's transform
    from paper_2411_17804_amd import epic
    p = {"fp16": W.FP16_SPLIT, "bf16": W.BF16_SPLIT, "fp32": W.FP32_FFT}[prec]
    cfg = W.make_config(idx, chan_subset=[3, 200] if idx == 3 else [9], n_time=11, precision=p)
    st = cfg.stations[0]
    if idx == 3:
        # stretched along y to a footprint of about 100 rows: beyond the fused
        # 128 x 128 split kernel, so the composed path runs
        st.pos_m = st.pos_m * np.array([1.0, 3.0])
    per_sample = cfg.n_chan * cfg.n_pol * st.nx * st.ny * 8
    say(f"image_cadence C{idx} {prec} in chunks of {max(1, (2 << 20) // per_sample)} samples")
    v = W.station_volts(cfg, 0)
    monkeypatch.setenv("EPIC_FIELD_BUDGET_MB", "2")
    epic.cache_clear()
    common, (station,) = station_objects(cfg, [to_device_volts(v)], p)
    epic.image_cadence(common, (station,))
    torch.cuda.synchronize()
    got = to_complex(station.image)
    err = oracle.image_error(got, oracle_image(cfg, 0, v), cfg.n_pol)
    say(f"  worst error {err.max():.2e}")
    assert err.max() <= (FP32_TOL if prec == "fp32" else SPLIT_TOL[prec]), err
    monkeypatch.delenv("EPIC_FIELD_BUDGET_MB")
    epic.cache_clear()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_footprint_pruned_transform_matches_dense(torch, prec):
    # the composed cadence's split transform (256 x 256 grids take that path)
    # sums only the footprint's tiles; the dense transform of the same gridded
    # planes (zero outside the footprint) must give the same images bit for bit
    from paper_2411_17804_amd import epic
    say(f"pruned split transform vs dense, C5 {prec}")
    p = W.FP16_SPLIT if prec == "fp16" else W.BF16_SPLIT
    cfg = W.make_config(5, chan_subset=[0, 127], n_time=3, precision=p)
    st = cfg.stations[0]
    v = W.station_volts(cfg, 0)
    common, (station,) = station_objects(cfg, [to_device_volts(v)], p)
    epic.image_cadence(common, (station,))
    torch.cuda.synchronize()
    nt, npol = cfg.n_time, cfg.n_pol
    grid = torch.zeros((cfg.n_chan, nt, npol, st.ny, st.nx, 2), dtype=torch.float32,
                       device="cuda")
    epic.grid_voltages(common, station, 0, nt, grid)
    epic.fft2_batched(st.nx, st.ny, cfg.n_chan * nt * npol, p, grid, grid)
    shape = (cfg.n_chan, npol * npol, st.ny, st.nx, 2)
    acc, comp, img = (torch.zeros(shape, device="cuda") for _ in range(3))
    epic.accumulate_power(npol, st.nx, st.ny, cfg.n_chan, nt, grid, acc, comp, nt, img)
    torch.cuda.synchronize()
    assert torch.equal(img, station.image)


# ------------------------------------------- hierarchical batch, graphs, tuning ----
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_image_cadence_hierarchical_batch(torch, prec):
    # 12 stations of uneven size (grids 32/64/128) in one call; ragged cadence
    p = W.FP32_FFT if prec == "fp32" else W.FP16_SPLIT
    cfg = W.make_config(4, chan_subset=[0, 63], n_time=40, n_stations=12, precision=p)
    sizes = sorted({s.nx for s in cfg.stations})
    say(f"image_cadence C4 {prec}: 12 stations, grids {sizes}")
    assert len(sizes) >= 2
    volts, imgs, _ = run_cadence(cfg)
    tol = FP32_TOL if prec == "fp32" else SPLIT_TOL["fp16"]
    worst = 0.0
    for s in range(len(cfg.stations)):
        err = oracle.image_error(imgs[s], oracle_image(cfg, s, volts[s]), cfg.n_pol)
        worst = max(worst, float(err.max()))
        assert err.max() <= tol, (s, cfg.stations[s].nx, err)
    say(f"  worst error over stations {worst:.2e}")


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_graph_replays_match_eager(torch, prec):
    # the first call runs eagerly, later calls replay a captured graph; eager
    # work and synchronisations sit between the replays
    from paper_2411_17804_amd import epic
    say(f"image_cadence graph replays {prec}")
    p = W.FP16_SPLIT if prec == "fp16" else W.FP32_FFT
    cfg = W.make_config(4, chan_subset=[1, 2], n_time=33, n_stations=8, precision=p)
    # keep only stations the fused kernels cover: grids up to 64 for the split
    # path, every grid size (32, 64 and 128) for FP32
    cfg.stations = [s for s in cfg.stations if prec == "fp32" or s.nx <= 64][:4]
    if prec == "fp32":
        assert any(s.nx == 128 for s in cfg.stations)
    volts = [W.station_volts(cfg, s) for s in range(len(cfg.stations))]
    common, stations = station_objects(cfg, [to_device_volts(v) for v in volts])
    epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    ref = [s.image.clone() for s in stations]
    for rep in range(4):
        for s in stations:
            s.image.fill_(float("nan"))          # eager work between replays
        torch.cuda.synchronize()
        epic.image_cadence(common, stations)
        torch.cuda.synchronize()
        for a, b in zip(ref, stations):
            assert torch.equal(a, b.image), f"replay {rep} differs from the eager result"


def test_cadence128_mixed_supports(torch):
    # 128 x 128 FP32 stations of three kernel supports in one call: the C3
    # lattice (2048 elements, support 3), a 512-element subset with support 5
    # and a 1024-element subset with the nearest-cell kernel.  Together their
    # taps overflow the LDS, so the class splits into persistent launches;
    # n_time = 37 leaves a ragged last block of samples and of gridding.
    import dataclasses
    from paper_2411_17804_amd import epic
    say("image_cadence fp32, 128 x 128 stations of supports 3, 5 and 1")
    cfg = W.make_config(3, chan_subset=[7, 100, 201], n_time=37, precision=W.FP32_FFT)
    base = cfg.stations[0]
    rng = np.random.default_rng(5)
    sub5 = np.sort(rng.choice(base.n_elem, 512, replace=False))
    sub1 = np.sort(rng.choice(base.n_elem, 1024, replace=False))
    cfg.stations = [base,
                    dataclasses.replace(base, pos_m=base.pos_m[sub5], support=5, sigma_cells=5.0 / 6.0),
                    dataclasses.replace(base, pos_m=base.pos_m[sub1], kernel_type=W.KERNEL_NEAREST,
                                        support=1, sigma_cells=0.0)]
    volts = [W.station_volts(cfg, s) for s in range(3)]
    common, stations = station_objects(cfg, [to_device_volts(v) for v in volts])
    epic.cache_clear()
    epic.timing_reset()
    epic.timing_enable(True)
    epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    epic.timing_enable(False)
    used = epic.timing_report()
    launches = used.get("fused_fft128_cadence", (0, 0.0))[0]
    say(f"  launches {used}")
    assert 2 <= launches <= 3, used                # every station in the 128 x 128 class
    assert set(used) == {"fused_fft128_cadence"}, used
    first = [s.image.clone() for s in stations]
    for s in range(3):
        err = oracle.image_error(to_complex(first[s]), oracle_image(cfg, s, volts[s]), 2)
        say(f"  station {s} (support {cfg.stations[s].support}) worst error {err.max():.2e}")
        assert err.max() <= FP32_TOL
    for rep in range(3):                         # graph replays
        for s in stations:
            s.image.fill_(float("nan"))
        torch.cuda.synchronize()
        epic.image_cadence(common, stations)
        torch.cuda.synchronize()
        for a, b in zip(first, stations):
            assert torch.equal(a, b.image), f"replay {rep} differs"
    epic.cache_clear()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_split128_one_launch_mixed_supports(torch, prec):
    # 128 x 128 split-precision stations of supports 3, 5 and 1 (the C3
    # lattice and two subsets of it) in one persistent launch; n_time = 20
    # ends on a partial block of samples
    import dataclasses
    from paper_2411_17804_amd import epic
    p = W.FP16_SPLIT if prec == "fp16" else W.BF16_SPLIT
    say(f"image_cadence {prec}, 128 x 128 stations of supports 3, 5 and 1")
    cfg = W.make_config(3, chan_subset=[0, 131, 255], n_time=20, precision=p)
    base = cfg.stations[0]
    rng = np.random.default_rng(7)
    sub5 = np.sort(rng.choice(base.n_elem, 512, replace=False))
    sub1 = np.sort(rng.choice(base.n_elem, 1024, replace=False))
    cfg.stations = [base,
                    dataclasses.replace(base, pos_m=base.pos_m[sub5], support=5, sigma_cells=5.0 / 6.0),
                    dataclasses.replace(base, pos_m=base.pos_m[sub1], kernel_type=W.KERNEL_NEAREST,
                                        support=1, sigma_cells=0.0)]
    volts = [W.station_volts(cfg, s) for s in range(3)]
    common, stations = station_objects(cfg, [to_device_volts(v) for v in volts], p)
    epic.cache_clear()
    epic.timing_reset()
    epic.timing_enable(True)
    epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    epic.timing_enable(False)
    used = epic.timing_report()
    say(f"  launches {used}")
    assert set(used) == {"fused_dft128_cadence"} and used["fused_dft128_cadence"][0] == 1, used
    first = [s.image.clone() for s in stations]
    for s in range(3):
        err = oracle.image_error(to_complex(first[s]), oracle_image(cfg, s, volts[s]), 2)
        say(f"  station {s} (support {cfg.stations[s].support}) worst error {err.max():.2e}")
        assert err.max() <= SPLIT_TOL[prec]
    for rep in range(3):                         # graph replays
        for s in stations:
            s.image.fill_(float("nan"))
        torch.cuda.synchronize()
        epic.image_cadence(common, stations)
        torch.cuda.synchronize()
        for a, b in zip(first, stations):
            assert torch.equal(a, b.image), f"replay {rep} differs"
    epic.cache_clear()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_autotune_small_cadence(torch, prec):
    # C1 (4 channels of one small station): the tuner weighs the persistent
    # 32 x 32 kernel, which keeps 4 work-groups busy, against the composed
    # path; whichever it keeps must match the oracle
    from paper_2411_17804_amd import epic
    p = W.FP32_FFT if prec == "fp32" else W.FP16_SPLIT
    cfg = W.make_config(1, precision=p)
    v = W.station_volts(cfg, 0)
    epic.cache_clear()
    common, stations = station_objects(cfg, [to_device_volts(v)], p)
    epic.autotune(common, stations)
    epic.timing_reset()
    epic.timing_enable(True)
    epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    epic.timing_enable(False)
    say(f"C1 {prec} after autotune: {sorted(epic.timing_report())}")
    err = oracle.image_error(to_complex(stations[0].image), oracle_image(cfg, 0, v), cfg.n_pol)
    say(f"  worst error {err.max():.2e}")
    assert err.max() <= (FP32_TOL if prec == "fp32" else SPLIT_TOL["fp16"]), err
    epic.cache_clear()


def test_autotune_then_cadence(torch, tmp_path, monkeypatch):
    from paper_2411_17804_amd import epic
    say("autotune + image_cadence")
    cfg = W.make_config(2, chan_subset=[0, 700], n_time=96, precision=W.FP32_FFT)
    volts = [W.station_volts(cfg, 0)]
    common, stations = station_objects(cfg, [to_device_volts(volts[0])])
    epic.autotune(common, stations)
    epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    err = oracle.image_error(to_complex(stations[0].image), oracle_image(cfg, 0, volts[0]), 2)
    assert err.max() <= FP32_TOL
