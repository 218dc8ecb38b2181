"""Second, independently written FP64 oracle in numpy -- TEST INFRASTRUCTURE ONLY.

It exists to cross-check the C oracle (``epic_oracle.c``): it recomputes the
element cells and weights with vectorised numpy, grids with ``np.add.at`` and
transforms with ``numpy.fft`` (``ifft2`` times the cell count has the + sign and
no normalisation of Eq. 3).  Sec. 5.2, Eq. 3 then Eq. 2.
"""
from __future__ import annotations

import numpy as np


def element_weights(pos_m, wavelength_m, grid_spacing_wl, nx, ny, K, sigma_cells, nearest):
    """Nearest cell and normalised separable Gaussian (or unit) weights per element."""
    pos = np.asarray(pos_m, np.float64)
    delta = grid_spacing_wl * wavelength_m
    u = pos[:, 0] / delta + nx // 2
    v = pos[:, 1] / delta + ny // 2
    i = np.floor(u + 0.5)
    j = np.floor(v + 0.5)
    h = (K - 1) // 2
    if np.any(i - h < 0) or np.any(i + h > nx - 1) or np.any(j - h < 0) or np.any(j + h > ny - 1):
        raise ValueError("kernel footprint leaves the grid")
    if nearest:
        wx = np.ones((pos.shape[0], 1))
        wy = np.ones((pos.shape[0], 1))
    else:
        d = np.arange(-h, h + 1, dtype=np.float64)
        wx = np.exp(-0.5 * ((d[None, :] - (u - i)[:, None]) / sigma_cells) ** 2)
        wy = np.exp(-0.5 * ((d[None, :] - (v - j)[:, None]) / sigma_cells) ** 2)
        wx /= wx.sum(axis=1, keepdims=True)
        wy /= wy.sum(axis=1, keepdims=True)
    return i.astype(np.int64), j.astype(np.int64), wx, wy


def to_complex(volts):
    v = np.asarray(volts)
    if v.dtype == np.int8:
        return v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)
    return v.astype(np.complex128)


def grid(pos_m, wavelength_m, grid_spacing_wl, nx, ny, K, sigma_cells, nearest, volts):
    """volts: [n_time, n_elem, n_pol] -> G complex128 [n_time, n_pol, ny, nx]."""
    E = to_complex(volts)
    n_time, n_elem, n_pol = E.shape
    i, j, wx, wy = element_weights(pos_m, wavelength_m, grid_spacing_wl, nx, ny, K,
                                   sigma_cells, nearest)
    h = (K - 1) // 2
    G = np.zeros((n_time, n_pol, ny, nx), np.complex128)
    for dy in range(-h, h + 1):
        for dx in range(-h, h + 1):
            w = wx[:, dx + h] * wy[:, dy + h]                      # [n_elem]
            contrib = E * w[None, :, None]                           # [t, a, p]
            for p in range(n_pol):
                np.add.at(G[:, p], (slice(None), j + dy, i + dx), contrib[:, :, p])
    return G


def image(pos_m, wavelengths_m, grid_spacing_wl, nx, ny, K, sigma_cells, nearest, volts):
    """volts: [n_chan, n_time, n_elem, n_pol] -> complex128 [n_chan, n_pol^2, ny, nx]."""
    out = []
    for c, lam in enumerate(np.asarray(wavelengths_m, np.float64)):
        G = grid(pos_m, lam, grid_spacing_wl, nx, ny, K, sigma_cells, nearest, volts[c])
        F = np.fft.ifft2(G, axes=(-2, -1)) * (nx * ny)
        n_pol = F.shape[1]
        prods = [np.mean(F[:, a] * np.conj(F[:, b]), axis=0)
                 for a in range(n_pol) for b in range(n_pol)]
        out.append(np.stack(prods))
    return np.stack(out)
