"""GPU parity of gridding with full polarimetric complex kernels (Sec. 5.2,
Eq. 3 in general form: grid_voltages_pol, image_cadence_pol) against the FP64
oracle (oracle.grid_pol, oracle.image_pol) on the same seeded inputs.
Tolerances: gridded fields 1e-6 of their largest value; images the c-14
metric, 1e-5 (FP32 transform) and 1e-4 (FP16-split)."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import from_complex, say, station_objects, to_complex, to_device_volts, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = torch_cuda()
    from paper_2411_17804_amd import epic
    epic.load()
    return t


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _kernels(cfg, K, kind, seed):
    """Seeded complex kernels [n_chan][n_elem][n_pol][n_pol][K][K]: "random"
    (a leaky pol response with random complex taps) or "wproj" (a Gaussian
    illumination times a per-element quadratic phase screen, as w-projection
    kernels are, with a small cross-pol leakage)."""
    st = cfg.stations[0]
    rng = np.random.default_rng([17804, 20, seed])
    shape = (cfg.n_chan, st.n_elem, cfg.n_pol, cfg.n_pol, K, K)
    if kind == "random":
        k = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    else:
        d = np.arange(K) - (K - 1) / 2
        g = np.exp(-0.5 * (d / (K / 6.0)) ** 2)
        w = rng.uniform(-0.3, 0.3, (cfg.n_chan, st.n_elem))
        ph = np.exp(-1j * np.pi * w[:, :, None, None] * (d[None, None, :, None] ** 2 + d[None, None, None, :] ** 2))
        base = (g[:, None] * g[None, :])[None, None] * ph
        k = np.zeros(shape, np.complex128)
        for a in range(cfg.n_pol):
            for p in range(cfg.n_pol):
                k[:, :, a, p] = base * (1.0 if a == p else 0.05 * np.exp(0.7j * (a - p)))
    return k.astype(np.complex64).astype(np.complex128)


GRID_CASES = {
    # name: (config, channels, n_time, K, kind)
    "C2-ci8-random-K3": (2, [0, 700], 10, 3, "random"),
    "C1-cf32-1pol-K1": (1, [0, 3], 12, 1, "random"),
    "C2-ci8-wproj-K7": (2, [40], 9, 7, "wproj"),
}


@pytest.mark.parametrize("case", sorted(GRID_CASES))
def test_grid_voltages_pol(torch, case):
    from paper_2411_17804_amd import epic
    idx, chans, nt, K, kind = GRID_CASES[case]
    say(f"grid_voltages_pol {case}")
    cfg = W.make_config(idx, chan_subset=chans, n_time=nt)
    st = cfg.stations[0]
    st.support = K
    st.kernel_type = W.KERNEL_GAUSSIAN if K > 1 else W.KERNEL_NEAREST
    st.sigma_cells = K / 6.0
    v = W.station_volts(cfg, 0)
    kern = _kernels(cfg, K, kind, len(case))
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    grid = torch.zeros((cfg.n_chan, nt, cfg.n_pol, st.ny, st.nx, 2), dtype=torch.float32,
                       device="cuda")
    epic.grid_voltages_pol(common, station, from_complex(kern), 0, nt, grid)
    torch.cuda.synchronize()
    got = to_complex(grid)
    for c in range(cfg.n_chan):
        ref = oracle.grid_pol(st.pos_m, cfg.wavelengths_m[c], W.GRID_SPACING_WL, st.nx, st.ny, K,
                              kern[c], v[c])
        err = _rel(got[c], ref)
        say(f"  {case} channel {c}: error {err:.2e}")
        assert err <= 1e-6, err


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_image_cadence_pol(torch, prec):
    from paper_2411_17804_amd import epic
    say(f"image_cadence_pol C2 {prec}")
    p = W.FP32_FFT if prec == "fp32" else W.FP16_SPLIT
    cfg = W.make_config(2, chan_subset=[3, 901], n_time=40, precision=p)
    st = cfg.stations[0]
    v = W.station_volts(cfg, 0)
    kern = _kernels(cfg, 3, "wproj", 7)
    common, (station,) = station_objects(cfg, [to_device_volts(v)])
    epic.image_cadence_pol(common, station, from_complex(kern))
    torch.cuda.synchronize()
    got = to_complex(station.image)
    ref = oracle.image_pol(st.pos_m, cfg.wavelengths_m, W.GRID_SPACING_WL, st.nx, st.ny, 3, kern, v)
    err = max(float(oracle.image_error(got[c], ref[c], cfg.n_pol).max()) for c in range(cfg.n_chan))
    say(f"  {prec}: image error {err:.2e}")
    assert err <= (1e-5 if prec == "fp32" else 1e-4)


def test_diagonal_pol_kernels_match_image_cadence(torch):
    # real diagonal kernels from the separable weights: the same image as
    # image_cadence (up to FP32 rounding of the weights)
    from paper_2411_17804_amd import epic
    say("image_cadence_pol with diagonal kernels vs image_cadence, C2")
    cfg = W.make_config(2, chan_subset=[11, 512], n_time=32)
    st = cfg.stations[0]
    v = W.station_volts(cfg, 0)
    kern = np.zeros((cfg.n_chan, st.n_elem, 2, 2, 3, 3), np.complex128)
    for c, lam in enumerate(cfg.wavelengths_m):
        _, _, wx, wy = oracle.plan(st.pos_m, lam, W.GRID_SPACING_WL, st.nx, st.ny, st.kernel_type,
                                   st.support, st.sigma_cells)
        for p in range(2):
            kern[c, :, p, p] = wy[:, :, None] * wx[:, None, :]
    common, (s1,) = station_objects(cfg, [to_device_volts(v)])
    epic.image_cadence_pol(common, s1, from_complex(kern))
    common, (s2,) = station_objects(cfg, [to_device_volts(v)])
    epic.image_cadence(common, (s2,))
    torch.cuda.synchronize()
    a, b = to_complex(s1.image), to_complex(s2.image)
    err = max(float(oracle.image_error(a[c], b[c], 2).max()) for c in range(cfg.n_chan))
    say(f"  difference {err:.2e}")
    assert err <= 2e-6
