"""FP64 CPU oracle for the EPIC direct imager -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never links, loads or
calls it, and it shares no code with the GPU library.

Two independent implementations live here:

* ``epic_oracle.c`` -- plain C99 in double precision (own radix-2 FFT and a
  direct DFT), wrapped by the functions below through ctypes;
* ``numpy_oracle.py`` -- a second, separately written numpy version (own plan,
  ``np.add.at`` gridding, ``numpy.fft``) used to cross-check the first.

Both follow Sec. 5.2, Eq. 3 (grid the element voltages with the element
kernel, then the 2-D transform with the + sign) and Eq. 2 (polarisation outer
product averaged over the cadence).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "epic_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "libepic_oracle.so")

KERNEL_NEAREST = 0
KERNEL_GAUSSIAN = 1
VOLT_CI8 = 0
VOLT_CF32 = 1
VOLT_CF64 = 2

ERR_ARG = -1
ERR_OFFGRID = -2

_lib = None


def build(src: str = _SRC, out: str = _LIB_PATH, extra_flags: tuple = ()) -> str:
    """Compile the C oracle with gcc (OpenMP, -O2, strict IEEE: no fast-math)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           *extra_flags, src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def load(path: str | None = None) -> ctypes.CDLL:
    """Load (building first if needed) the C oracle; cached for the default path."""
    global _lib
    if path is None:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        path = _LIB_PATH
    lib = ctypes.CDLL(path)
    _declare(lib)
    if path == _LIB_PATH:
        _lib = lib
    return lib


def _declare(lib):
    P = ctypes.c_void_p
    i32, f64 = ctypes.c_int, ctypes.c_double
    lib.eo_element_taps.argtypes = [f64, f64, f64, i32, i32, i32, i32, f64, P, P, P, P]
    lib.eo_element_taps.restype = i32
    lib.eo_plan.argtypes = [i32, P, f64, f64, i32, i32, i32, i32, f64, P, P, P, P]
    lib.eo_plan.restype = i32
    lib.eo_fft2_batched.argtypes = [P, ctypes.c_long, i32, i32]
    lib.eo_fft2_batched.restype = None
    lib.eo_dft2.argtypes = [P, P, i32, i32]
    lib.eo_dft2.restype = None
    lib.eo_power_mean.argtypes = [i32, i32, i32, i32, P, i32, P]
    lib.eo_power_mean.restype = None
    lib.eo_grid.argtypes = [i32, P, f64, f64, i32, i32, i32, i32, f64, i32, i32, P, i32, i32, P]
    lib.eo_grid.restype = i32
    lib.eo_image.argtypes = [i32, P, i32, P, f64, i32, i32, i32, i32, i32, i32, f64, i32, P,
                             i32, i32, P]
    lib.eo_image.restype = i32
    lib.eo_max_threads.argtypes = []
    lib.eo_max_threads.restype = i32


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


def _volt_type(volts: np.ndarray) -> tuple[int, np.ndarray]:
    """Map a voltage array to (type code, contiguous raw array).

    complex64 -> cf32, complex128 -> cf64, int8 with a trailing axis of 2
    (re, im) -> ci8."""
    if volts.dtype == np.complex64:
        return VOLT_CF32, np.ascontiguousarray(volts)
    if volts.dtype == np.complex128:
        return VOLT_CF64, np.ascontiguousarray(volts)
    if volts.dtype == np.int8:
        assert volts.shape[-1] == 2, "ci8 voltages carry a trailing (re, im) axis"
        return VOLT_CI8, np.ascontiguousarray(volts)
    raise TypeError(f"unsupported voltage dtype {volts.dtype}")


def plan(pos_m, wavelength_m, grid_spacing_wl, nx, ny, kernel_type, K, sigma_cells,
         lib=None):
    """Per-element nearest cells and separable kernel weights (Sec. 5.2, Eq. 3).

    Returns (ix, iy, wx, wy) with wx, wy of shape [n_elem, K]."""
    lib = lib or load()
    pos = np.ascontiguousarray(pos_m, dtype=np.float64)
    n = pos.shape[0]
    ix = np.zeros(n, np.int32)
    iy = np.zeros(n, np.int32)
    wx = np.zeros((n, K), np.float64)
    wy = np.zeros((n, K), np.float64)
    rc = lib.eo_plan(n, _ptr(pos), float(wavelength_m), float(grid_spacing_wl), nx, ny,
                     kernel_type, K, float(sigma_cells), _ptr(ix), _ptr(iy), _ptr(wx), _ptr(wy))
    if rc != 0:
        raise OracleError(rc)
    return ix, iy, wx, wy


def grid(pos_m, wavelength_m, grid_spacing_wl, nx, ny, kernel_type, K, sigma_cells, volts,
         t0=0, nt=None, lib=None):
    """Gridded field G (inner bracket of Eq. 3) of one channel.

    volts: [n_time, n_elem, n_pol] complex (or [..., 2] int8).  Returns
    complex128 [nt, n_pol, ny, nx]."""
    lib = lib or load()
    vt, v = _volt_type(volts)
    n_time, n_elem, n_pol = v.shape[:3]
    nt = n_time - t0 if nt is None else nt
    pos = np.ascontiguousarray(pos_m, dtype=np.float64)
    out = np.zeros((nt, n_pol, ny, nx), np.complex128)
    rc = lib.eo_grid(n_elem, _ptr(pos), float(wavelength_m), float(grid_spacing_wl), nx, ny,
                     kernel_type, K, float(sigma_cells), n_pol, vt, _ptr(v), t0, nt, _ptr(out))
    if rc != 0:
        raise OracleError(rc)
    return out


def fft2(data: np.ndarray, lib=None) -> np.ndarray:
    """Unnormalised 2-D transform with the + sign of Eq. 3 over the last two
    axes, by the oracle's own radix-2 FFT.  Returns complex128."""
    lib = lib or load()
    a = np.array(data, dtype=np.complex128, copy=True, order="C")
    ny, nx = a.shape[-2:]
    lib.eo_fft2_batched(_ptr(a), a.size // (nx * ny), nx, ny)
    return a


def dft2(data: np.ndarray, lib=None) -> np.ndarray:
    """The same transform as fft2, as a direct O(N^4) sum (small grids only)."""
    lib = lib or load()
    a = np.ascontiguousarray(data, dtype=np.complex128)
    ny, nx = a.shape[-2:]
    flat = a.reshape(-1, ny, nx)
    out = np.zeros_like(flat)
    for b in range(flat.shape[0]):
        lib.eo_dft2(_ptr(flat[b]), _ptr(out[b]), nx, ny)
    return out.reshape(a.shape)


def power_mean(field: np.ndarray, n_div: int = 0, lib=None) -> np.ndarray:
    """Eq. 2 on a per-sample field [nt, n_pol, ny, nx]: returns complex128
    [n_pol*n_pol, ny, nx] = sum_t F^a conj(F^b) / (n_div or nt)."""
    lib = lib or load()
    f = np.ascontiguousarray(field, dtype=np.complex128)
    nt, n_pol, ny, nx = f.shape
    out = np.zeros((n_pol * n_pol, ny, nx), np.complex128)
    lib.eo_power_mean(n_pol, nx, ny, nt, _ptr(f), int(n_div), _ptr(out))
    return out


def image(pos_m, wavelengths_m, grid_spacing_wl, nx, ny, kernel_type, K, sigma_cells,
          volts, use_dft=False, n_threads=0, lib=None):
    """EPIC image of one station (Eq. 3 then Eq. 2) for every channel.

    volts: [n_chan, n_time, n_elem, n_pol] complex64/complex128, or
    [n_chan, n_time, n_elem, n_pol, 2] int8.  Returns complex128
    [n_chan, n_pol*n_pol, ny, nx] (mean over n_time, products XX, XY, YX, YY)."""
    lib = lib or load()
    vt, v = _volt_type(volts)
    n_chan, n_time, n_elem, n_pol = v.shape[:4]
    lam = np.ascontiguousarray(wavelengths_m, dtype=np.float64)
    assert lam.shape == (n_chan,)
    pos = np.ascontiguousarray(pos_m, dtype=np.float64)
    assert pos.shape == (n_elem, 2)
    out = np.zeros((n_chan, n_pol * n_pol, ny, nx), np.complex128)
    rc = lib.eo_image(n_elem, _ptr(pos), n_chan, _ptr(lam), float(grid_spacing_wl), n_time,
                      n_pol, nx, ny, kernel_type, K, float(sigma_cells), vt, _ptr(v),
                      1 if use_dft else 0, int(n_threads), _ptr(out))
    if rc != 0:
        raise OracleError(rc)
    return out


def grid_pol(pos_m, wavelength_m, grid_spacing_wl, nx, ny, K, kernels, volts, lib=None):
    """Gridded field of one channel with full polarimetric complex kernels
    (Eq. 3, inner bracket, in general form):
        G^a[j] = sum_elem sum_p conj(W_elem^{ap}[j - c_elem + h]) E_elem^p
    on the K x K cells around each element's nearest cell c_elem (h = (K-1)/2;
    the cells are those of plan()).  kernels: complex [n_elem, n_pol (a),
    n_pol (p), K (dy), K (dx)], the caller's kernel values at those cells.
    volts: [n_time, n_elem, n_pol] complex (or [..., 2] int8).  Returns
    complex128 [n_time, n_pol, ny, nx]."""
    lib = lib or load()
    _, v = _volt_type(volts)
    if v.dtype == np.int8:
        v = v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)
    v = np.asarray(v, np.complex128)
    n_time, n_elem, n_pol = v.shape
    W = np.asarray(kernels, np.complex128)
    ix, iy, _, _ = plan(pos_m, wavelength_m, grid_spacing_wl, nx, ny, KERNEL_NEAREST if K == 1
                        else KERNEL_GAUSSIAN, K, 1.0, lib=lib)
    h = (K - 1) // 2
    out = np.zeros((n_time, n_pol, ny, nx), np.complex128)
    for a in range(n_elem):
        for dy in range(K):
            for dx in range(K):
                y, x = iy[a] - h + dy, ix[a] - h + dx
                for al in range(n_pol):
                    for p in range(n_pol):
                        out[:, al, y, x] += np.conj(W[a, al, p, dy, dx]) * v[:, a, p]
    return out


def image_pol(pos_m, wavelengths_m, grid_spacing_wl, nx, ny, K, kernels, volts, lib=None):
    """EPIC image (Eq. 3 with grid_pol(), then Eq. 2) for every channel;
    kernels: complex [n_chan, n_elem, n_pol, n_pol, K, K].  Returns complex128
    [n_chan, n_pol*n_pol, ny, nx]."""
    lib = lib or load()
    n_chan = len(wavelengths_m)
    out = []
    for c in range(n_chan):
        f = fft2(grid_pol(pos_m, wavelengths_m[c], grid_spacing_wl, nx, ny, K, kernels[c],
                          volts[c], lib=lib), lib=lib)
        out.append(power_mean(f, lib=lib))
    return np.stack(out)


def station_beams(pos_m, wavelengths_m, grid_spacing_wl, nx, ny, kernel_type, K, sigma_cells,
                  volts, lib=None):
    """The station-synthesised electric fields of Sec. 6.2: for every channel
    and sample, the Eq. 3 transform of the gridded voltages before any
    squaring, i.e. the station acting as a virtual telescope pointed at every
    pixel k of its sky grid.  volts as for image(); returns complex128
    [n_chan, n_time, n_pol, ny, nx]."""
    lib = lib or load()
    _, v = _volt_type(volts)
    n_chan, n_time, n_elem, n_pol = v.shape[:4]
    out = np.empty((n_chan, n_time, n_pol, ny, nx), np.complex128)
    for c in range(n_chan):
        out[c] = fft2(grid(pos_m, wavelengths_m[c], grid_spacing_wl, nx, ny, kernel_type, K,
                           sigma_cells, volts[c], lib=lib), lib=lib)
    return out


def array_image(beams, pixels, array_pos_m, wavelengths_m, array_spacing_wl, nx, ny,
                kernel_type, K, sigma_cells, lib=None):
    """Coherent inter-station EPIC (Sec. 6.2, Eq. 10 then Eq. 9): the M
    stations are the elements of an array-scale EPIC imager.  For every
    channel c and selected station pixel k (flat index ky * beam_nx + kx),
    the fields beams[m][c][t][p][k] of the stations (station_beams() of each)
    are gridded at the station positions array_pos_m on the array grid,
    transformed, squared and averaged over the cadence, exactly as image()
    does for elements.  Returns complex128 [n_chan, n_sel, n_pol^2, ny, nx]."""
    lib = lib or load()
    b = np.stack([np.asarray(x, np.complex128) for x in beams])      # [m, c, t, p, by, bx]
    n_st, n_chan, n_time, n_pol = b.shape[:4]
    flat = b.reshape(n_st, n_chan, n_time, n_pol, -1)
    pix = np.asarray(pixels, np.int64)
    # array-scale voltages of every (channel, pixel) problem: [c, s, t, m, p]
    v = np.transpose(flat[..., pix], (1, 4, 2, 0, 3))
    lam = np.repeat(np.asarray(wavelengths_m, np.float64), pix.size)
    img = image(array_pos_m, lam, array_spacing_wl, nx, ny, kernel_type, K, sigma_cells,
                np.ascontiguousarray(v.reshape(n_chan * pix.size, n_time, n_st, n_pol)), lib=lib)
    return img.reshape(n_chan, pix.size, n_pol * n_pol, ny, nx)


def visibilities(volts):
    """Eq. 4, the correlator of the XFFT architecture (Sec. 5.4): per channel the
    mean over the cadence of E_a^p(t) conj(E_b^q(t)) for every ordered element
    pair (autocorrelations included) and every pol pair, in FP64.  volts as for
    image(); returns complex128 [n_chan, n_elem, n_pol, n_elem, n_pol] (row
    (a, p), column (b, q)).  Each channel's matrix is X^T conj(X) / n_time for
    X = the [n_time, n_elem * n_pol] voltage matrix (one library matmul)."""
    if volts.dtype == np.int8:
        v = volts[..., 0].astype(np.float64) + 1j * volts[..., 1].astype(np.float64)
    else:
        v = volts.astype(np.complex128)
    n_chan, n_time, n_elem, n_pol = v.shape[:4]
    X = v.reshape(n_chan, n_time, n_elem * n_pol)
    out = np.empty((n_chan, n_elem * n_pol, n_elem * n_pol), np.complex128)
    for c in range(n_chan):
        out[c] = (X[c].T @ np.conj(X[c])) / n_time
    return out.reshape(n_chan, n_elem, n_pol, n_elem, n_pol)


def grid_visibility_matrix(vis, pos_m, wavelengths_m, grid_spacing_wl, nx, ny, kernel_type, K,
                           sigma_cells, lib=None):
    """Eq. 6 gridding (no transform) of given visibilities vis
    [n_chan, n_elem, n_pol, n_elem, n_pol] (as visibilities() returns): each
    V_ab^{pq} is placed at its baseline cell c_a - c_b with the
    cross-correlation of the two elements' kernels (extent 2K - 1 per axis),
        G^{pq}[j] = sum_{a,b} sum_{d1,d2} w_a(d1) w_b(d2) V_ab^{pq}
                    [j = (c_a + d1) - (c_b + d2) mod (nx, ny)].
    Cells and weights come from plan(); returns complex128
    [n_chan, n_pol*n_pol, ny, nx]."""
    lib = lib or load()
    n_chan, n_elem, n_pol = vis.shape[0], vis.shape[1], vis.shape[2]
    h = (K - 1) // 2
    out = np.zeros((n_chan, n_pol * n_pol, ny, nx), np.complex128)
    for c in range(n_chan):
        ix, iy, wx, wy = plan(pos_m, wavelengths_m[c], grid_spacing_wl, nx, ny, kernel_type, K,
                              sigma_cells, lib=lib)
        ix = ix.astype(np.int64)
        iy = iy.astype(np.int64)
        for d1y in range(-h, h + 1):
            for d1x in range(-h, h + 1):
                wa = wx[:, d1x + h] * wy[:, d1y + h]
                for d2y in range(-h, h + 1):
                    for d2x in range(-h, h + 1):
                        wb = wx[:, d2x + h] * wy[:, d2y + h]
                        cx = ((ix + d1x)[:, None] - (ix + d2x)[None, :]) % nx
                        cy = ((iy + d1y)[:, None] - (iy + d2y)[None, :]) % ny
                        wab = wa[:, None] * wb[None, :]
                        for p in range(n_pol):
                            for q in range(n_pol):
                                np.add.at(out[c, p * n_pol + q], (cy, cx),
                                          wab * vis[c, :, p, :, q])
    return out


def grid_visibilities(pos_m, wavelengths_m, grid_spacing_wl, nx, ny, kernel_type, K,
                      sigma_cells, volts, lib=None):
    """FFT-correlator output of one station written out directly, per channel:
    the visibilities of Eq. 4 (visibilities()) gridded as in Eq. 6
    (grid_visibility_matrix()).  No transform is involved; on the circular
    grid the result is the inverse transform of the EPIC image.  volts as for
    image(); returns complex128 [n_chan, n_pol*n_pol, ny, nx]."""
    return grid_visibility_matrix(visibilities(volts), pos_m, wavelengths_m, grid_spacing_wl, nx,
                                  ny, kernel_type, K, sigma_cells, lib=lib)


def combine_incoherent(images, weights=None):
    """Incoherent combination of station images (Sec. 6.1, Eq. 7), in FP64:
    per pixel, product and channel, sum_m w_m I_m / sum_m w_m, for stations on
    one sky pixel grid.  images: sequence of [n_chan, n_q, ny, nx] complex;
    weights: [n_stations, n_q, ny, nx] real (the same for every channel) or
    None for equal weights.  Pixels whose weights sum to 0 give 0."""
    imgs = np.stack([np.asarray(i, np.complex128) for i in images])      # [m, c, q, y, x]
    if weights is None:
        w = np.ones((imgs.shape[0],) + imgs.shape[2:], np.float64)
    else:
        w = np.asarray(weights, np.float64)
    num = np.einsum("mqyx,mcqyx->cqyx", w, imgs)
    den = w.sum(axis=0)
    out = np.zeros(num.shape, np.complex128)
    nz = den != 0
    out[:, nz] = num[:, nz] / den[nz]
    return out


def max_threads(lib=None) -> int:
    return (lib or load()).eo_max_threads()


def image_error(img: np.ndarray, ref: np.ndarray, n_pol: int) -> np.ndarray:
    """Per-image error: max |I - I_ref| over pixels divided by the image scale.

    The scale is max |I_ref^{aa}| for the auto products and
    sqrt(max I_ref^{XX} * max I_ref^{YY}) for the cross products (their
    Cauchy-Schwarz bound); a per-pixel relative error is meaningless where a
    cross product crosses zero.  img, ref: [..., n_pol*n_pol, ny, nx].
    Returns [..., n_pol*n_pol]."""
    img = np.asarray(img)
    ref = np.asarray(ref)
    diff = np.abs(img - ref).max(axis=(-1, -2))
    auto = np.stack([np.abs(ref[..., a * n_pol + a, :, :]).max(axis=(-1, -2))
                     for a in range(n_pol)], axis=-1)
    scale = np.empty(diff.shape, np.float64)
    for a in range(n_pol):
        for b in range(n_pol):
            scale[..., a * n_pol + b] = np.sqrt(auto[..., a] * auto[..., b])
    return diff / np.maximum(scale, np.finfo(np.float64).tiny)
