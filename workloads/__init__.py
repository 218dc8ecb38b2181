"""Seeded synthetic workloads shaped like the arrays the imager is studied for.

This module only draws inputs: layouts, wavelengths and voltages.  It holds none
of the imaging arithmetic (no gridding, transform or products), so both the GPU
tests and the CPU oracle can consume what it produces without sharing code.

Five configurations:

* ``C1`` plain FP32, CPU-sized: 64 elements uniform in a 16 m square, 32x32 grid,
  nearest-cell gridding, 1 pol, 4 channels, 256 samples, complex64 N(0,1)
  voltages plus 3 point sources at SNR 10.
* ``C2`` station scale (an SKA-low-like station, D_s/lambda = 17.5, D_e/lambda
  = 1, Table 1): 256 elements uniform in a 38 m circle with 1.5 m minimum
  spacing, 150 MHz, 64x64 grid at lambda/2, 3x3 Gaussian kernel, 2 pols,
  1024 channels, 2048 samples, int8 complex Gaussian voltages (sigma 16).
* ``C3`` dense compact array: 64x32 lattice at 1 m, lambda = 2 m, 128x128 grid,
  3x3 kernel, 2 pols, 256 channels, 4096 samples, complex64 noise plus 20
  power-law sources (integral counts N(>S) ~ S^-1.5).
* ``C4`` hierarchical: 96 stations with uniform element counts in [64, 1024] at
  the C2 density, each on a 32/64/128 grid chosen by its footprint, 2 pols,
  64 channels, 1024 samples, int8 voltages.
* ``C5`` large dense layout: 128x128 lattice at 0.75 m with 5 % of the sites
  dropped (15565 elements), lambda = 1.5 m, 256x256 grid, 5x5 kernel, 2 pols,
  128 channels, 512 samples, complex64 noise plus 20 power-law sources.

Channels are centred on the nominal frequency with 40 kHz spacing
(delta_nu = 1/delta_t, delta_t = 25 us, Sec. 4).  The grid spacing is lambda/2
at every channel.  Random streams: ``default_rng([seed, station, channel])``
per (station, channel) for voltages, ``default_rng([seed, 0xC0FFEE])`` for
layouts and sources, seed = 17804 + config number.
"""
from __future__ import annotations

import dataclasses
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

C_LIGHT = 299792458.0
DELTA_NU_HZ = 40e3          # 1 / 25 us
GRID_SPACING_WL = 0.5       # lambda / 2

KERNEL_NEAREST = 0
KERNEL_GAUSSIAN = 1
CI8 = 0
CF32 = 1
FP32_FFT = 0
FP16_SPLIT = 1
BF16_SPLIT = 2


@dataclasses.dataclass(frozen=True)
class Source:
    kx: int            # pixel (signed, natural-order index kx' in [-nx/2, nx/2))
    ky: int
    flux: float        # S: per-pol signal variance scale
    xy_corr: float     # correlation of the X and Y signals (0 = unpolarised)


@dataclasses.dataclass
class Station:
    pos_m: np.ndarray            # [n_elem, 2] float64, metres from the phase centre
    nx: int
    ny: int
    kernel_type: int
    support: int
    sigma_cells: float
    sources: tuple = ()

    @property
    def n_elem(self) -> int:
        return int(self.pos_m.shape[0])


@dataclasses.dataclass
class Config:
    name: str
    index: int
    seed: int
    n_pol: int
    wavelengths_m: np.ndarray    # [n_chan]
    chan_ids: np.ndarray         # global channel numbers (for the random streams)
    n_time: int
    volt_type: int
    precision: int
    noise_sigma: float
    stations: list

    @property
    def n_chan(self) -> int:
        return int(self.wavelengths_m.shape[0])

    def pixel_samples(self) -> int:
        """Grid pixel-samples per cadence: sum over stations of nx*ny*n_chan*n_time."""
        return sum(s.nx * s.ny for s in self.stations) * self.n_chan * self.n_time

    def volt_bytes(self) -> int:
        b = 2 if self.volt_type == CI8 else 8
        return sum(s.n_elem for s in self.stations) * self.n_pol * self.n_chan * self.n_time * b


def wavelengths(nu0_hz: float, n_chan: int) -> np.ndarray:
    c = np.arange(n_chan, dtype=np.float64)
    nu = nu0_hz + (c - n_chan // 2) * DELTA_NU_HZ
    return C_LIGHT / nu


def _dart_circle(rng, n, diameter, min_spacing, max_tries=1_000_000):
    """n points uniform in a circle with a minimum spacing (dart throwing)."""
    r = diameter / 2.0
    pts = np.zeros((n, 2))
    k = 0
    tries = 0
    batch = 256
    while k < n:
        if tries > max_tries:
            raise RuntimeError("dart throwing did not converge")
        rad = r * np.sqrt(rng.random(batch))
        ang = 2 * np.pi * rng.random(batch)
        cand = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
        for p in cand:
            tries += 1
            if k == 0 or np.min(np.sum((pts[:k] - p) ** 2, axis=1)) >= min_spacing ** 2:
                pts[k] = p
                k += 1
                if k == n:
                    break
    return pts


def _distinct_pixels(rng, n, nx, ny, dwl, lmax=0.5):
    """n distinct pixel centres (kx', ky') with |l|, |m| <= lmax."""
    kxmax = int(math.floor(lmax * nx * dwl))
    kymax = int(math.floor(lmax * ny * dwl))
    seen = set()
    out = []
    while len(out) < n:
        kx = int(rng.integers(-kxmax, kxmax + 1))
        ky = int(rng.integers(-kymax, kymax + 1))
        if (kx, ky) in seen or (kx, ky) == (0, 0):
            continue
        seen.add((kx, ky))
        out.append((kx, ky))
    return out


def _power_law_sources(rng, n, s_min, nx, ny):
    u = rng.random(n)
    flux = np.minimum(s_min * u ** (-1.0 / 1.5), 100.0 * s_min)
    pix = _distinct_pixels(rng, n, nx, ny, GRID_SPACING_WL)
    order = np.argsort(-flux)
    srcs = []
    for rank, i in enumerate(order):
        srcs.append(Source(pix[i][0], pix[i][1], float(flux[i]), 0.5 if rank == 0 else 0.0))
    return tuple(srcs)


def _snr_flux(snr, sigma_n, n_elem, n_time):
    # coherent peak n_e^2 * 2S over a noise floor n_e * 2 sigma^2 / sqrt(n_time)
    return snr * sigma_n ** 2 / (n_elem * math.sqrt(n_time))


def _grid_size_for(diameter, lam_min, K):
    need = math.ceil(diameter / (GRID_SPACING_WL * lam_min)) + K + 1
    for n in (32, 64, 128):
        if n >= need:
            return n
    raise ValueError("station too large for a 128 grid")


def make_config(index: int, n_chan: int | None = None, n_time: int | None = None,
                chan_subset=None, n_stations: int | None = None,
                precision: int | None = None) -> Config:
    """Build configuration C<index>.  n_chan/n_time shrink the cadence (the first
    n_chan channels of the full band keep their true frequencies);
    chan_subset picks explicit channel numbers of the full band instead."""
    seed = 17804 + index
    lrng = np.random.default_rng([seed, 0xC0FFEE])
    if index == 1:
        full_chan, full_time, nu0 = 4, 256, C_LIGHT / 2.0
        pos = np.stack([lrng.uniform(-8, 8, 64), lrng.uniform(-8, 8, 64)], axis=1)
        st = Station(pos, 32, 32, KERNEL_NEAREST, 1, 0.0)
        nt_full = full_time
        srcs = tuple(Source(kx, ky, _snr_flux(10.0, 1.0, 64, nt_full), 0.0)
                     for kx, ky in _distinct_pixels(lrng, 3, 32, 32, GRID_SPACING_WL))
        st.sources = srcs
        stations, n_pol, vt, prec, sig = [st], 1, CF32, FP32_FFT, 1.0
    elif index == 2:
        full_chan, full_time, nu0 = 1024, 2048, 150e6
        pos = _dart_circle(lrng, 256, 38.0, 1.5)
        stations = [Station(pos, 64, 64, KERNEL_GAUSSIAN, 3, 0.5)]
        n_pol, vt, prec, sig = 2, CI8, FP32_FFT, 16.0
    elif index == 3:
        full_chan, full_time, nu0 = 256, 4096, C_LIGHT / 2.0
        ii, jj = np.meshgrid(np.arange(64), np.arange(32), indexing="ij")
        pos = np.stack([(ii.ravel() - 32) * 1.0, (jj.ravel() - 16) * 1.0], axis=1)
        st = Station(pos, 128, 128, KERNEL_GAUSSIAN, 3, 0.5)
        s_min = _snr_flux(5.0, 1.0, pos.shape[0], full_time)
        st.sources = _power_law_sources(lrng, 20, s_min, 128, 128)
        stations, n_pol, vt, prec, sig = [st], 2, CF32, FP16_SPLIT, 1.0
    elif index == 4:
        full_chan, full_time, nu0 = 64, 1024, C_LIGHT / 2.0
        lam_min = float(wavelengths(nu0, full_chan).min())
        stations = []
        n_st = 96
        counts = lrng.integers(64, 1025, n_st)
        for ne in counts:
            d = 38.0 * math.sqrt(ne / 256.0)
            pos = _dart_circle(lrng, int(ne), d, 1.5)
            span = 2.0 * float(np.max(np.abs(pos))) if ne > 0 else d
            n = _grid_size_for(max(span, 1e-9), lam_min, 3)
            stations.append(Station(pos, n, n, KERNEL_GAUSSIAN, 3, 0.5))
        n_pol, vt, prec, sig = 2, CI8, FP16_SPLIT, 16.0
    elif index == 5:
        full_chan, full_time, nu0 = 128, 512, C_LIGHT / 1.5
        ii, jj = np.meshgrid(np.arange(128), np.arange(128), indexing="ij")
        pos = np.stack([(ii.ravel() - 64) * 0.75, (jj.ravel() - 64) * 0.75], axis=1)
        drop = lrng.choice(pos.shape[0], 819, replace=False)
        keep = np.setdiff1d(np.arange(pos.shape[0]), drop)
        pos = pos[keep]
        st = Station(pos, 256, 256, KERNEL_GAUSSIAN, 5, 5.0 / 6.0)
        s_min = _snr_flux(5.0, 1.0, pos.shape[0], full_time)
        st.sources = _power_law_sources(lrng, 20, s_min, 256, 256)
        stations, n_pol, vt, prec, sig = [st], 2, CF32, FP16_SPLIT, 1.0
    else:
        raise ValueError(f"no configuration C{index}")

    lam_full = wavelengths(nu0, full_chan)
    if chan_subset is not None:
        ids = np.asarray(chan_subset, np.int64)
    else:
        ids = np.arange(full_chan if n_chan is None else n_chan, dtype=np.int64)
    if n_stations is not None:
        stations = stations[:n_stations]
    return Config(name=f"C{index}", index=index, seed=seed, n_pol=n_pol,
                  wavelengths_m=lam_full[ids], chan_ids=ids,
                  n_time=full_time if n_time is None else n_time, volt_type=vt,
                  precision=prec if precision is None else precision, noise_sigma=sig,
                  stations=stations)


def array_centres(n_stations: int, diameter_m: float, min_spacing_m: float, seed: int) -> np.ndarray:
    """Station centres of a synthetic array (metres, array frame): uniform in a
    circle with a minimum spacing, for the inter-station (Eq. 10) workload."""
    return _dart_circle(np.random.default_rng([seed, 0xA77A]), n_stations, diameter_m, min_spacing_m)


def channel_volts(cfg: Config, station_idx: int, chan_pos: int) -> np.ndarray:
    """Voltages of one station at one channel of cfg: [n_time, n_elem, n_pol].

    complex64 for cf32 configs, int8 [..., 2] (re, im) for ci8 configs.  The
    stream depends on (seed, station, global channel number) only, so any
    channel can be regenerated on its own."""
    st = cfg.stations[station_idx]
    cid = int(cfg.chan_ids[chan_pos])
    lam = float(cfg.wavelengths_m[chan_pos])
    rng = np.random.default_rng([cfg.seed, station_idx, cid])
    shape = (cfg.n_time, st.n_elem, cfg.n_pol)
    if cfg.volt_type == CI8:
        x = rng.standard_normal(shape + (2,), dtype=np.float32) * np.float32(cfg.noise_sigma)
        return np.clip(np.rint(x), -127, 127).astype(np.int8)
    re = rng.standard_normal(shape, dtype=np.float32)
    im = rng.standard_normal(shape, dtype=np.float32)
    v = (re * np.float32(cfg.noise_sigma)).astype(np.complex64)
    v.imag = im * np.float32(cfg.noise_sigma)
    if st.sources:
        v = v.astype(np.complex128)
        x = st.pos_m[:, 0]
        y = st.pos_m[:, 1]
        for s in st.sources:
            l = s.kx / (st.nx * GRID_SPACING_WL)
            m = s.ky / (st.ny * GRID_SPACING_WL)
            # a source at direction (l, m) reaches element a with phase
            # exp(-i 2 pi (l x_a + m y_a) / lambda)
            phase = np.exp(-2j * np.pi * (l * x + m * y) / lam)          # [n_elem]
            gx = rng.standard_normal(cfg.n_time) + 1j * rng.standard_normal(cfg.n_time)
            gy_ind = rng.standard_normal(cfg.n_time) + 1j * rng.standard_normal(cfg.n_time)
            rho = s.xy_corr
            gy = rho * gx + math.sqrt(1.0 - rho * rho) * gy_ind
            amp = math.sqrt(s.flux)
            v[:, :, 0] += amp * gx[:, None] * phase[None, :]
            if cfg.n_pol == 2:
                v[:, :, 1] += amp * gy[:, None] * phase[None, :]
        v = v.astype(np.complex64)
    return v


def station_volts(cfg: Config, station_idx: int, chan_positions=None, threads: int = 8):
    """All (or the listed) channels of one station: [n_chan, n_time, n_elem, n_pol](, 2)."""
    chans = range(cfg.n_chan) if chan_positions is None else list(chan_positions)
    chans = list(chans)
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        parts = list(ex.map(lambda c: channel_volts(cfg, station_idx, c), chans))
    return np.stack(parts)
