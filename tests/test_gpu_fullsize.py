"""GPU parity at full size: whole cadences run as the benchmark runs them
(image_cadence over the full set of samples: the fused kernels, replayed
from the captured graph on the second call), checked against the FP64 oracle
on sampled stations and channels that it images one by one.

* C2: the station cadence (256 elements in a 38 m circle, 64 x 64 grid, 3 x 3
  Gaussian, 2 pols, ci8), all 1024 channels x 2048 samples, five channels
  checked.
* C4: the hierarchical layout, all 96 stations (64-1024 elements on 32 x 32,
  64 x 64 and 128 x 128 grids) x 64 channels x 1024 samples, eight stations
  spanning the three grid sizes and their element counts x three channels
  checked.
* C3: the dense 64 x 32 lattice on a 128 x 128 grid, two channels (the band
  edges) x all 4096 samples.
* C5: the 128 x 128 lattice less 5 % on a 256 x 256 grid with a 5 x 5 kernel,
  two channels (the band edges) x all 512 samples.

Tolerances (c-14 metric): FP32 1e-5, FP16-split 1e-4; BF16-split is reported
with a loose bound.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import say, station_objects, to_complex, to_device_volts, torch_cuda

pytestmark = pytest.mark.gpu

SAMPLED = [0, 257, 514, 771, 1023]
TOL = {W.FP32_FFT: 1e-5, W.FP16_SPLIT: 1e-4, W.BF16_SPLIT: 2e-3}
NAME = {W.FP32_FFT: "fp32", W.FP16_SPLIT: "fp16-split", W.BF16_SPLIT: "bf16-split"}


def _run_twice(torch, common, stations, check):
    """image_cadence twice (the second call replays the captured graph): the
    checked images must be bit-identical between the calls."""
    from paper_2411_17804_amd import epic
    epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    first = [stations[s].image[ch].clone() for s, ch in check]
    for st in stations:
        st.image.zero_()
    epic.image_cadence(common, stations)
    torch.cuda.synchronize()
    for (s, ch), f in zip(check, first):
        assert torch.equal(stations[s].image[ch], f), f"replay differs from the first call (station {s})"


def _hermitian_and_finite(torch, img):
    assert bool(torch.isfinite(img).all())
    assert torch.equal(img[:, 2, ..., 0], img[:, 1, ..., 0])
    assert torch.equal(img[:, 2, ..., 1], -img[:, 1, ..., 1])


# ------------------------------------------------------------------- C2 ----
@pytest.fixture(scope="module")
def c2_full():
    torch = torch_cuda()
    from paper_2411_17804_amd import epic
    epic.load()
    cfg = W.make_config(2)
    assert cfg.n_chan == 1024 and cfg.n_time == 2048
    say("C2 full cadence: generating 1024 x 2048 samples of 256 elements")
    v = W.station_volts(cfg, 0, threads=16)
    st = cfg.stations[0]
    say("C2 full cadence: oracle on the sampled channels")
    ref = oracle.image(st.pos_m, cfg.wavelengths_m[SAMPLED], W.GRID_SPACING_WL, st.nx, st.ny,
                       st.kernel_type, st.support, st.sigma_cells, v[SAMPLED], n_threads=16)
    dev = to_device_volts(v)
    del v
    yield torch, cfg, dev, ref
    del dev
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", [W.FP32_FFT, W.FP16_SPLIT])
def test_c2_full_cadence_sampled_channels(c2_full, prec):
    torch, cfg, dev, ref = c2_full
    say(f"C2 full cadence {NAME[prec]}: image_cadence twice (the second call replays the graph)")
    common, stations = station_objects(cfg, [dev], prec)
    _run_twice(torch, common, stations, [(0, SAMPLED)])
    got = to_complex(stations[0].image[SAMPLED])
    err = oracle.image_error(got, ref, cfg.n_pol)
    say(f"  {NAME[prec]}: worst error over channels {SAMPLED}: {err.max():.2e}")
    assert err.max() <= TOL[prec], err
    _hermitian_and_finite(torch, stations[0].image)


# ------------------------------------------------------------------- C4 ----
C4_CHANNELS = [0, 31, 63]


def _c4_sample(cfg):
    """Eight stations: the smallest, median and largest 128 x 128 and 64 x 64
    stations by element count, and the smallest and largest 32 x 32 ones."""
    picks = []
    for grid, k in ((128, 3), (64, 3), (32, 2)):
        idx = sorted((i for i, s in enumerate(cfg.stations) if s.nx == grid),
                     key=lambda i: cfg.stations[i].n_elem)
        picks += [idx[int(round(j))] for j in np.linspace(0, len(idx) - 1, min(k, len(idx)))]
    return list(dict.fromkeys(picks))


@pytest.fixture(scope="module")
def c4_full():
    torch = torch_cuda()
    from paper_2411_17804_amd import epic
    epic.load()
    cfg = W.make_config(4)
    assert len(cfg.stations) == 96 and cfg.n_chan == 64 and cfg.n_time == 1024
    sample = _c4_sample(cfg)
    assert {cfg.stations[s].nx for s in sample} == {32, 64, 128}
    say(f"C4 full cadence: generating 96 stations x 64 channels x 1024 samples; oracle on "
        f"stations {sample} x channels {C4_CHANNELS}")
    devs, refs = [], {}
    for s, st in enumerate(cfg.stations):
        v = W.station_volts(cfg, s, threads=16)
        if s in sample:
            refs[s] = oracle.image(st.pos_m, cfg.wavelengths_m[C4_CHANNELS], W.GRID_SPACING_WL,
                                   st.nx, st.ny, st.kernel_type, st.support, st.sigma_cells,
                                   v[C4_CHANNELS], n_threads=16)
        devs.append(to_device_volts(v))
        del v
    say("C4 full cadence: inputs resident")
    yield torch, cfg, devs, refs
    del devs
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", [W.FP32_FFT, W.FP16_SPLIT, W.BF16_SPLIT])
def test_c4_full_cadence_sampled_stations(c4_full, prec):
    from paper_2411_17804_amd import epic
    torch, cfg, devs, refs = c4_full
    say(f"C4 full cadence {NAME[prec]}: 96 stations, image_cadence twice")
    common, stations = station_objects(cfg, devs, prec)
    check = [(s, C4_CHANNELS) for s in refs]
    _run_twice(torch, common, stations, check)
    worst = 0.0
    for s, ref in refs.items():
        got = to_complex(stations[s].image[C4_CHANNELS])
        err = oracle.image_error(got, ref, cfg.n_pol)
        st = cfg.stations[s]
        say(f"  {NAME[prec]}: station {s} ({st.nx}x{st.ny}, {st.n_elem} el): {err.max():.2e}")
        worst = max(worst, float(err.max()))
        assert err.max() <= TOL[prec], (s, err)
    say(f"  {NAME[prec]}: worst error over the sample {worst:.2e}")
    for st in stations:
        _hermitian_and_finite(torch, st.image)
    del stations
    epic.cache_clear()
    torch.cuda.empty_cache()


# -------------------------------------------------------------- C3, C5 ----
_EDGES = {}


def _band_edges(idx):
    """Config idx restricted to its first and last channel (full cadence),
    its voltages and the oracle's images of them (computed once per config)."""
    if idx not in _EDGES:
        full = W.make_config(idx)
        cfg = W.make_config(idx, chan_subset=[0, full.n_chan - 1])
        assert cfg.n_time == full.n_time
        st = cfg.stations[0]
        v = W.station_volts(cfg, 0, threads=16)
        say(f"C{idx}: oracle on 2 channels x {cfg.n_time} samples of {st.n_elem} elements "
            f"on {st.nx}x{st.ny}")
        ref = oracle.image(st.pos_m, cfg.wavelengths_m, W.GRID_SPACING_WL, st.nx, st.ny,
                           st.kernel_type, st.support, st.sigma_cells, v, n_threads=16)
        _EDGES.clear()
        _EDGES[idx] = (cfg, v, ref)
    return _EDGES[idx]


@pytest.mark.parametrize("prec", [W.FP32_FFT, W.FP16_SPLIT, W.BF16_SPLIT])
@pytest.mark.parametrize("idx", [3, 5])
def test_band_edges_full_cadence(idx, prec):
    torch = torch_cuda()
    from paper_2411_17804_amd import epic
    epic.load()
    cfg, v, ref = _band_edges(idx)
    say(f"C{idx} full cadence {NAME[prec]}: 2 channels x {cfg.n_time} samples")
    common, stations = station_objects(cfg, [to_device_volts(v)], prec)
    _run_twice(torch, common, stations, [(0, [0, 1])])
    err = oracle.image_error(to_complex(stations[0].image), ref, cfg.n_pol)
    say(f"  C{idx} {NAME[prec]}: worst error {err.max():.2e}")
    assert err.max() <= TOL[prec], err
    _hermitian_and_finite(torch, stations[0].image)
