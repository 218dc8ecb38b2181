"""GPU parity of the XFFT route (Sec. 5.4): the correlator of Eq. 4
(xfft_correlate) and the gridding of Eq. 6 plus the transform (xfft_image),
against the FP64 oracle on the same seeded inputs.

Tolerances: ci8 visibilities are exact integer sums scaled once in FP32, so a
power-of-two cadence (the scale is exact) must match the oracle bit for bit
and any other cadence to 2^-23 of the largest visibility; cf32 visibilities
are FP32 sums of n_time products (<= 2e-6 of the largest at these sizes);
images use the c-14 metric with the FP32 gate 1e-5; gridded visibilities
<= 1e-6 of their largest value.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import from_complex, say, station_objects, to_complex, to_device_volts, torch_cuda

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


def _station_cfg(idx, chans, nt, n_elem=None, support=None):
    cfg = W.make_config(idx, chan_subset=chans, n_time=nt)
    st = cfg.stations[0]
    if n_elem is not None:
        st.pos_m = st.pos_m[:n_elem]
    if support is not None:
        st.support, st.sigma_cells = support, support / 6.0
    return cfg


def run_xfft(cfg, v, s=0, gridded=True):
    from paper_2411_17804_amd import epic
    torch = torch_cuda()
    st = cfg.stations[s]
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    station.pos_m, station.nx, station.ny = st.pos_m, st.nx, st.ny
    station.kernel_type, station.support, station.sigma_cells = st.kernel_type, st.support, st.sigma_cells
    vis = torch.zeros((cfg.n_chan, st.n_elem, cfg.n_pol, st.n_elem, cfg.n_pol, 2),
                      dtype=torch.float32, device="cuda")
    epic.xfft_correlate(common, station, vis)
    grid = None
    if gridded:
        grid = torch.zeros((cfg.n_chan, cfg.n_pol ** 2, st.ny, st.nx, 2), dtype=torch.float32,
                           device="cuda")
    epic.xfft_image(common, station, vis, grid)
    torch.cuda.synchronize()
    return (to_complex(vis), None if grid is None else to_complex(grid),
            to_complex(station.image), (common, station, vis))


# ------------------------------------------------------------- correlator ----
CORR_CASES = {
    # name: (config, channels, n_time, n_elem)
    "C2-ci8-pow2": (2, [0, 777], 64, None),
    "C2-ci8-ragged-time": (2, [5], 70, None),
    "C2-ci8-ragged-rows": (2, [300], 100, 37),       # R = 74: rows not a multiple of 8
    "C1-cf32": (1, [0, 3], 256, None),
    "C1-cf32-odd-rows": (1, [1], 45, 37),            # R = 37
    "C3-cf32-1ch": (3, [100], 8, None),              # R = 4096
}


@pytest.mark.parametrize("case", sorted(CORR_CASES))
def test_xfft_correlate(torch, case):
    from paper_2411_17804_amd import epic
    idx, chans, nt, ne = CORR_CASES[case]
    say(f"xfft_correlate {case}")
    cfg = _station_cfg(idx, chans, nt, ne)
    v = W.station_volts(cfg, 0)
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    station.pos_m = cfg.stations[0].pos_m
    n_el = cfg.stations[0].n_elem
    vis = torch.zeros((cfg.n_chan, n_el, cfg.n_pol, n_el, cfg.n_pol, 2), dtype=torch.float32,
                      device="cuda")
    epic.xfft_correlate(common, station, vis)
    torch.cuda.synchronize()
    got = to_complex(vis)
    ref = oracle.visibilities(v)
    if cfg.volt_type == W.CI8 and nt & (nt - 1) == 0:
        assert np.array_equal(got, ref), "exact integer sums scaled by a power of two"
        say(f"  {case}: bit-exact")
        return
    err = _rel(got, ref)
    say(f"  {case}: error {err:.2e}")
    assert err <= (2.0 ** -23 if cfg.volt_type == W.CI8 else 2e-6), err
    R = n_el * cfg.n_pol
    m = got.reshape(cfg.n_chan, R, R)
    assert np.array_equal(m, np.conj(np.transpose(m, (0, 2, 1)))), "Hermitian by construction"


def test_xfft_correlate_long_cadence(torch):
    # more than 65408 ci8 samples: the correlator sums in segments (exact int32
    # within each) and adds them in FP32; 64 elements, one pol
    from paper_2411_17804_amd import epic
    say("xfft_correlate ci8, 70000 samples (two segments)")
    cfg = W.make_config(1, chan_subset=[2], n_time=70000)
    cfg.volt_type = W.CI8
    st = cfg.stations[0]
    rng = np.random.default_rng([17804, 30])
    v = np.clip(np.rint(rng.standard_normal((1, cfg.n_time, st.n_elem, 1, 2)) * 40), -128, 127).astype(np.int8)
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    vis = torch.zeros((1, st.n_elem, 1, st.n_elem, 1, 2), dtype=torch.float32, device="cuda")
    epic.xfft_correlate(common, station, vis)
    torch.cuda.synchronize()
    got, ref = to_complex(vis), oracle.visibilities(v)
    err = _rel(got, ref)
    say(f"  error {err:.2e}")
    assert err <= 2.0 ** -22, err


# ------------------------------------------------------- gridding + image ----
IMAGE_CASES = {
    # name: (config, channels, n_time, n_elem, support, check gridded against the oracle)
    "C1-nearest": (1, [0, 2], 64, None, None, True),
    "C2-2ch": (2, [0, 1023], 40, None, None, True),
    "C2-K5": (2, [512], 24, None, 5, False),
    "C2-K7-ragged": (2, [3], 30, 101, 7, False),
    "C3-1ch": (3, [100], 8, None, None, False),
}


@pytest.mark.parametrize("case", sorted(IMAGE_CASES))
def test_xfft_image(torch, case):
    idx, chans, nt, ne, K, check_grid = IMAGE_CASES[case]
    say(f"xfft_image {case}")
    cfg = _station_cfg(idx, chans, nt, ne, K)
    st = cfg.stations[0]
    v = W.station_volts(cfg, 0)
    vis, grid, img, _ = run_xfft(cfg, v)
    ref = oracle.image(st.pos_m, cfg.wavelengths_m, W.GRID_SPACING_WL, st.nx, st.ny,
                       st.kernel_type, st.support, st.sigma_cells, v)
    err = oracle.image_error(img, ref, cfg.n_pol)
    say(f"  {case}: image error {err.max():.2e}")
    assert err.max() <= FP32_TOL, err
    if check_grid:
        gref = oracle.grid_visibility_matrix(oracle.visibilities(v), st.pos_m, cfg.wavelengths_m,
                                             W.GRID_SPACING_WL, st.nx, st.ny, st.kernel_type,
                                             st.support, st.sigma_cells)
        gerr = _rel(grid, gref)
        say(f"  {case}: gridded error {gerr:.2e}")
        assert gerr <= 1e-6, gerr


def test_xfft_hierarchical_stations(torch):
    # stations of uneven size (grids 32 / 64 / 128) from the batched layout
    cfg = W.make_config(4, chan_subset=[0, 63], n_time=16)
    picks = {}
    for s, st in enumerate(cfg.stations):
        picks.setdefault(st.nx, s)
    say(f"xfft_image C4 stations {sorted(picks.items())}")
    for n, s in sorted(picks.items()):
        st = cfg.stations[s]
        one = W.make_config(4, chan_subset=[0, 63], n_time=16)
        one.stations = [st]
        v = W.station_volts(cfg, s)
        _, _, img, _ = run_xfft(one, v, gridded=False)
        ref = oracle.image(st.pos_m, cfg.wavelengths_m, W.GRID_SPACING_WL, st.nx, st.ny,
                           st.kernel_type, st.support, st.sigma_cells, v)
        err = oracle.image_error(img, ref, cfg.n_pol)
        say(f"  station {s} ({n}x{n}, {st.n_elem} elements): image error {err.max():.2e}")
        assert err.max() <= FP32_TOL, err


def test_xfft_matches_epic_and_fft_correlator(torch):
    # the two routes on the GPU: the XFFT image against image_cadence's, and the
    # gridded visibilities against image_to_visibilities of the EPIC image
    from paper_2411_17804_amd import epic
    say("xfft vs image_cadence, C2")
    cfg = W.make_config(2, chan_subset=[100, 900], n_time=48)
    v = W.station_volts(cfg, 0)
    _, grid, img, _ = run_xfft(cfg, v)
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    epic.image_cadence(common, (station,))
    vis2 = torch.empty_like(station.image)
    epic.image_to_visibilities(cfg.n_pol, 64, 64, cfg.n_chan, station.image, vis2)
    torch.cuda.synchronize()
    err = oracle.image_error(img, to_complex(station.image), cfg.n_pol)
    say(f"  image difference {err.max():.2e}")
    assert err.max() <= 2 * FP32_TOL
    gerr = _rel(grid, to_complex(vis2))
    say(f"  gridded visibility difference {gerr:.2e}")
    assert gerr <= 2e-5


def test_xfft_deterministic(torch):
    say("xfft determinism C2")
    cfg = W.make_config(2, chan_subset=[7], n_time=33)
    v = W.station_volts(cfg, 0)
    a = run_xfft(cfg, v)
    b = run_xfft(cfg, v)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
