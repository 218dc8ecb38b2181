"""ctypes binding of the C ABI in include/epic.h (argument marshalling only).

Every step of the imager runs in the gfx950 kernels of libepic.so; this module
only turns Python objects into the ABI's structs and pointers.  Device buffers
are torch tensors (used for their memory and for the current HIP stream);
host arrays (positions, wavelengths) are numpy float64 arrays.  There is no
fallback: if the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libepic.so")

# enums of epic.h
EPIC_OK = 0
EPIC_ERR_INVALID_ARG = -1
EPIC_ERR_UNSUPPORTED = -2
EPIC_ERR_OUT_OF_MEMORY = -3
EPIC_ERR_DEVICE = -4
EPIC_ERR_INTERNAL = -5
CI8 = 0
CF32 = 1
FP32_FFT = 0
FP16_SPLIT = 1
BF16_SPLIT = 2
KERNEL_NEAREST = 0
KERNEL_GAUSSIAN = 1

# every function the header declares
ABI_FUNCTIONS = ("grid_voltages", "fft2_batched", "accumulate_power", "image_cadence",
                 "image_cadence_noalloc",
                 "image_to_visibilities", "combine_incoherent", "xfft_correlate", "xfft_image", "array_cadence", "array_xfft", "grid_voltages_pol", "image_cadence_pol",
                 "epic_autotune", "epic_validate", "epic_timing_enable", "epic_timing_report",
                 "epic_timing_reset", "epic_status_string", "epic_last_error",
                 "epic_cache_clear")


class _Kernel(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("support", ctypes.c_int32),
                ("sigma_cells", ctypes.c_double)]


class _Common(ctypes.Structure):
    _fields_ = [("n_pol", ctypes.c_int32), ("n_chan", ctypes.c_int32),
                ("wavelength_m", ctypes.c_void_p), ("grid_spacing_wl", ctypes.c_double),
                ("n_time", ctypes.c_int32), ("volt_type", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


class _Station(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int32), ("pos_m", ctypes.c_void_p),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("kernel", _Kernel),
                ("volts", ctypes.c_void_p), ("image", ctypes.c_void_p)]


class EpicError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{status_name(status)}: {detail}")
        self.status = status
        self.detail = detail


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libepic.so.  Import torch first in GPU processes so that the
    library binds to the same HIP runtime as torch's streams."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.grid_voltages.argtypes = [P, P, i32, i32, P, P]
    lib.grid_voltages.restype = i32
    lib.fft2_batched.argtypes = [i32, i32, i64, i32, P, P, P]
    lib.fft2_batched.restype = i32
    lib.accumulate_power.argtypes = [i32, i32, i32, i32, i32, P, P, P, i32, P, P]
    lib.accumulate_power.restype = i32
    lib.image_cadence.argtypes = [P, P, i32, P]
    lib.image_cadence.restype = i32
    lib.image_cadence_noalloc.argtypes = [P, P, i32, P]
    lib.image_cadence_noalloc.restype = i32
    lib.image_to_visibilities.argtypes = [i32, i32, i32, i32, P, P, P]
    lib.image_to_visibilities.restype = i32
    lib.combine_incoherent.argtypes = [i32, i32, i32, i32, i32, P, P, P, P]
    lib.combine_incoherent.restype = i32
    lib.xfft_correlate.argtypes = [P, P, P, P]
    lib.xfft_correlate.restype = i32
    lib.xfft_image.argtypes = [P, P, P, P, P]
    lib.xfft_image.restype = i32
    lib.grid_voltages_pol.argtypes = [P, P, P, i32, i32, P, P]
    lib.grid_voltages_pol.restype = i32
    lib.image_cadence_pol.argtypes = [P, P, P, P]
    lib.image_cadence_pol.restype = i32
    lib.array_cadence.argtypes = [P, P, P, i32, i32, i32, P, P]
    lib.array_cadence.restype = i32
    lib.array_xfft.argtypes = [P, P, P, i32, i32, i32, P, P]
    lib.array_xfft.restype = i32
    lib.epic_autotune.argtypes = [P, P, i32, P]
    lib.epic_autotune.restype = i32
    lib.epic_validate.argtypes = [P, P, i32]
    lib.epic_validate.restype = i32
    lib.epic_status_string.argtypes = [i32]
    lib.epic_status_string.restype = ctypes.c_char_p
    lib.epic_last_error.argtypes = []
    lib.epic_last_error.restype = ctypes.c_char_p
    lib.epic_timing_enable.argtypes = [i32]
    lib.epic_timing_enable.restype = None
    lib.epic_timing_report.argtypes = [ctypes.c_char_p, i32]
    lib.epic_timing_report.restype = i32
    lib.epic_timing_reset.argtypes = []
    lib.epic_timing_reset.restype = None
    lib.epic_cache_clear.argtypes = []
    lib.epic_cache_clear.restype = None
    _lib = lib
    return lib


def status_name(status: int) -> str:
    return load().epic_status_string(int(status)).decode()


def last_error() -> str:
    return load().epic_last_error().decode()


def cache_clear() -> None:
    load().epic_cache_clear()


def timing_enable(on: bool = True) -> None:
    load().epic_timing_enable(1 if on else 0)


def timing_reset() -> None:
    load().epic_timing_reset()


def timing_report() -> dict:
    """{kernel name: (launch count, total ms)} of the launches recorded while
    timing was enabled (waits for them to finish)."""
    buf = ctypes.create_string_buffer(1 << 16)
    load().epic_timing_report(buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        name, count, ms = line.split()
        out[name] = (int(count), float(ms))
    return out


def _check(status: int) -> None:
    if status != EPIC_OK:
        raise EpicError(status, last_error())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    """Device address of a torch tensor (or an int address, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


# dtypes a device buffer may have: complex float32 data as complex64 or as
# float32 (re, im) pairs; ci8 voltages as int8 (re, im) pairs
_CF32 = ("complex64", "float32")
_F32 = ("float32",)
_I8 = ("int8",)


def _dev(t, what: str, nbytes: int, dtypes=_CF32):
    """Device address of buffer t after checking it against the size and type
    the call implies.  The C ABI receives no device-buffer sizes, so this is
    the one place a wrong tensor can be caught: it must be a contiguous GPU
    tensor of one of the dtypes and exactly nbytes long.  Raw integer
    addresses and None are passed through unchecked (the ABI rejects a null
    pointer where one is required)."""
    if t is None or isinstance(t, int):
        return t
    dt = str(t.dtype).replace("torch.", "")
    if not t.is_cuda:
        raise ValueError(f"{what}: expected a GPU tensor, got one on {t.device}")
    if dt not in dtypes:
        raise ValueError(f"{what}: dtype {dt}, expected one of {', '.join(dtypes)}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor is not contiguous (the kernels read it densely)")
    got = t.numel() * t.element_size()
    if got != nbytes:
        raise ValueError(f"{what}: {got} bytes, the call implies {nbytes} "
                         f"(shape {tuple(t.shape)}, dtype {dt})")
    return t.data_ptr()


def _volts(common: "Common", station: "Station", what: str = "volts"):
    """Checked address of a station's voltages [n_chan][n_time][n_elem][n_pol]."""
    n = len(np.atleast_1d(common.wavelength_m)) * common.n_time * np.asarray(station.pos_m).shape[0] \
        * common.n_pol
    if common.volt_type == CI8:
        return _dev(station.volts, what, n * 2, _I8)
    return _dev(station.volts, what, n * 8, _CF32)


def _image(common: "Common", station: "Station", what: str = "image", planes: int = 1):
    """Checked address of a station's image [n_chan][planes][n_pol^2][ny][nx] cf32."""
    n = len(np.atleast_1d(common.wavelength_m)) * planes * common.n_pol ** 2 * station.nx * station.ny
    return _dev(station.image, what, n * 8)


@dataclasses.dataclass
class Common:
    """Parameters shared by the stations of a call (epic_common)."""
    n_pol: int
    wavelength_m: np.ndarray
    grid_spacing_wl: float
    n_time: int
    volt_type: int
    precision: int = FP32_FFT

    def to_c(self):
        lam = np.ascontiguousarray(self.wavelength_m, dtype=np.float64)
        c = _Common(self.n_pol, lam.shape[0], lam.ctypes.data, float(self.grid_spacing_wl),
                    self.n_time, self.volt_type, self.precision)
        return c, lam


@dataclasses.dataclass
class Station:
    """One station (epic_station): host positions, device voltages and image."""
    pos_m: np.ndarray
    nx: int
    ny: int
    kernel_type: int
    support: int
    sigma_cells: float
    volts: object = None       # torch tensor on the GPU
    image: object = None       # torch tensor on the GPU (complex64 or float32 pairs)

    def to_c(self, volts=None, image=None):
        """The epic_station struct; volts and image are the (checked) device
        addresses to put in it, by default the tensors' own unchecked ones."""
        pos = np.ascontiguousarray(self.pos_m, dtype=np.float64)
        s = _Station(pos.shape[0], pos.ctypes.data, self.nx, self.ny,
                     _Kernel(self.kernel_type, self.support, float(self.sigma_cells)),
                     _dptr(self.volts) if volts is None else volts,
                     _dptr(self.image) if image is None else image)
        return s, pos


def grid_voltages(common: Common, station: Station, t0: int, nt: int, grid, stream=None):
    lib = load()
    c, keep1 = common.to_c()
    s, keep2 = station.to_c(volts=_volts(common, station))
    n_chan = len(np.atleast_1d(common.wavelength_m))
    g = _dev(grid, "grid", n_chan * max(nt, 0) * common.n_pol * station.ny * station.nx * 8)
    _check(lib.grid_voltages(ctypes.byref(c), ctypes.byref(s), t0, nt, g, _stream(stream)))


def fft2_batched(nx: int, ny: int, batch: int, precision: int, inp, out, stream=None):
    lib = load()
    n = max(batch, 0) * nx * ny * 8
    _check(lib.fft2_batched(nx, ny, batch, precision, _dev(inp, "in", n), _dev(out, "out", n),
                            _stream(stream)))


def accumulate_power(n_pol: int, nx: int, ny: int, n_chan: int, nt: int, field, acc_sum,
                     acc_comp, finalize_n_time: int = 0, image=None, stream=None):
    lib = load()
    plane = max(n_chan, 0) * n_pol * n_pol * nx * ny * 8
    _check(lib.accumulate_power(n_pol, nx, ny, n_chan, nt,
                                _dev(field, "field", max(n_chan, 0) * max(nt, 0) * n_pol * nx * ny * 8),
                                _dev(acc_sum, "acc_sum", plane), _dev(acc_comp, "acc_comp", plane),
                                finalize_n_time, _dev(image, "image", plane), _stream(stream)))


def image_to_visibilities(n_pol: int, nx: int, ny: int, n_chan: int, image, vis, stream=None):
    """FFT-correlator output: the inverse transform of each product image
    (image, vis: device cf32 [n_chan][n_pol^2][ny][nx]; image is vis allowed)."""
    lib = load()
    n = max(n_chan, 0) * n_pol * n_pol * nx * ny * 8
    _check(lib.image_to_visibilities(n_pol, nx, ny, n_chan, _dev(image, "image", n),
                                     _dev(vis, "vis", n), _stream(stream)))


def combine_incoherent(n_pol: int, nx: int, ny: int, n_chan: int, images, out, weights=None,
                       stream=None):
    """Weighted mean of station images on one sky grid (images: sequence of
    device tensors cf32 [n_chan][n_pol^2][ny][nx]; weights: device float
    [n_stations][n_pol^2][ny][nx] or None for equal weights)."""
    lib = load()
    plane = n_pol * n_pol * nx * ny
    n = max(n_chan, 0) * plane * 8
    ptrs = (ctypes.c_void_p * max(1, len(images)))(
        *[_dev(t, f"images[{m}]", n) for m, t in enumerate(images)])
    _check(lib.combine_incoherent(n_pol, nx, ny, n_chan, len(images), ptrs if images else None,
                                  _dev(weights, "weights", len(images) * plane * 4, _F32),
                                  _dev(out, "out", n), _stream(stream)))


def grid_voltages_pol(common: Common, station: Station, kernels, t0: int, nt: int, grid,
                      stream=None):
    """Gridding with full polarimetric complex kernels (device cf32
    [n_chan][n_elem][n_pol][n_pol][K][K]) into grid [n_chan][nt][n_pol][ny][nx]."""
    lib = load()
    c, keep1 = common.to_c()
    s, keep2 = station.to_c(volts=_volts(common, station))
    n_chan = len(np.atleast_1d(common.wavelength_m))
    n_elem = np.asarray(station.pos_m).shape[0]
    kn = n_chan * n_elem * common.n_pol ** 2 * station.support ** 2 * 8
    g = _dev(grid, "grid", n_chan * max(nt, 0) * common.n_pol * station.ny * station.nx * 8)
    _check(lib.grid_voltages_pol(ctypes.byref(c), ctypes.byref(s), _dev(kernels, "kernels", kn),
                                 t0, nt, g, _stream(stream)))


def image_cadence_pol(common: Common, station: Station, kernels, stream=None):
    """The cadence of one station with full polarimetric kernels into station.image."""
    lib = load()
    c, keep1 = common.to_c()
    s, keep2 = station.to_c(volts=_volts(common, station), image=_image(common, station))
    n_chan = len(np.atleast_1d(common.wavelength_m))
    n_elem = np.asarray(station.pos_m).shape[0]
    kn = n_chan * n_elem * common.n_pol ** 2 * station.support ** 2 * 8
    _check(lib.image_cadence_pol(ctypes.byref(c), ctypes.byref(s), _dev(kernels, "kernels", kn),
                                 _stream(stream)))


def xfft_correlate(common: Common, station: Station, vis, stream=None):
    """Eq. 4 visibilities of one station into vis (device cf32
    [n_chan][n_elem][n_pol][n_elem][n_pol])."""
    lib = load()
    c, keep1 = common.to_c()
    s, keep2 = station.to_c(volts=_volts(common, station))
    n_chan = len(np.atleast_1d(common.wavelength_m))
    r = np.asarray(station.pos_m).shape[0] * common.n_pol
    _check(lib.xfft_correlate(ctypes.byref(c), ctypes.byref(s), _dev(vis, "vis", n_chan * r * r * 8),
                              _stream(stream)))


def xfft_image(common: Common, station: Station, vis, gridded=None, stream=None):
    """Eq. 6 gridding of vis and the transform into station.image; gridded
    (device cf32 [n_chan][n_pol^2][ny][nx] or None) receives the gridded
    visibilities."""
    lib = load()
    c, keep1 = common.to_c()
    s, keep2 = station.to_c(image=_image(common, station))
    n_chan = len(np.atleast_1d(common.wavelength_m))
    r = np.asarray(station.pos_m).shape[0] * common.n_pol
    gn = n_chan * common.n_pol ** 2 * station.nx * station.ny * 8
    _check(lib.xfft_image(ctypes.byref(c), ctypes.byref(s), _dev(vis, "vis", n_chan * r * r * 8),
                          _dev(gridded, "gridded", gn), _stream(stream)))


def array_cadence(common: Common, array: Station, beams, beam_nx: int, beam_ny: int, pixels,
                  stream=None):
    """Coherent inter-station EPIC: array.image (device cf32
    [n_chan][n_sel][n_pol^2][ny][nx]) from the stations' fields beams
    (sequence of device tensors cf32 [n_chan][n_time][n_pol][beam_ny][beam_nx])
    at the selected flat beam pixels."""
    lib = load()
    c, keep1 = common.to_c()
    pix = np.ascontiguousarray(pixels, dtype=np.int32)
    s, keep2 = array.to_c(image=_image(common, array, planes=pix.size))
    ptrs = _beam_ptrs(common, beams, beam_nx, beam_ny)
    _check(lib.array_cadence(ctypes.byref(c), ctypes.byref(s), ptrs if beams else None, beam_nx,
                             beam_ny, pix.size, pix.ctypes.data if pix.size else None,
                             _stream(stream)))


def array_xfft(common: Common, array: Station, beams, beam_nx: int, beam_ny: int, pixels,
               stream=None):
    """Coherent inter-station imaging by the XFFT route: arguments and output as
    array_cadence."""
    lib = load()
    c, keep1 = common.to_c()
    pix = np.ascontiguousarray(pixels, dtype=np.int32)
    s, keep2 = array.to_c(image=_image(common, array, planes=pix.size))
    ptrs = _beam_ptrs(common, beams, beam_nx, beam_ny)
    _check(lib.array_xfft(ctypes.byref(c), ctypes.byref(s), ptrs if beams else None, beam_nx,
                          beam_ny, pix.size, pix.ctypes.data if pix.size else None,
                          _stream(stream)))


def _beam_ptrs(common: Common, beams, beam_nx: int, beam_ny: int):
    """Checked addresses of the station fields [n_chan][n_time][n_pol][beam_ny][beam_nx]."""
    n = len(np.atleast_1d(common.wavelength_m)) * common.n_time * common.n_pol * beam_nx * beam_ny * 8
    return (ctypes.c_void_p * max(1, len(beams)))(
        *[_dev(t, f"beams[{m}]", n) for m, t in enumerate(beams)])


def _stations_c(stations, common: Common | None = None):
    """The epic_station array of a call; with common given, each station's
    voltages and image are checked against the shapes the call implies."""
    arr = (_Station * len(stations))()
    keep = []
    for i, st in enumerate(stations):
        if common is None:
            s, k = st.to_c()
        else:
            s, k = st.to_c(volts=_volts(common, st, f"stations[{i}].volts"),
                           image=_image(common, st, f"stations[{i}].image"))
        arr[i] = s
        keep.append(k)
    return arr, keep


def validate(common: Common, stations) -> None:
    """Host-only validation of an image_cadence call (no device work)."""
    lib = load()
    c, keep1 = common.to_c()
    arr, keep = _stations_c(stations)
    _check(lib.epic_validate(ctypes.byref(c), arr, len(stations)))


def image_cadence(common: Common, stations, stream=None):
    lib = load()
    c, keep1 = common.to_c()
    arr, keep = _stations_c(stations, common)
    _check(lib.image_cadence(ctypes.byref(c), arr, len(stations), _stream(stream)))


def image_cadence_noalloc(common: Common, stations, stream=None):
    """image_cadence without any device allocation (tables in the library's
    fixed scratch array; square grids up to 64 only)."""
    lib = load()
    c, keep1 = common.to_c()
    arr, keep = _stations_c(stations, common)
    _check(lib.image_cadence_noalloc(ctypes.byref(c), arr, len(stations), _stream(stream)))


def autotune(common: Common, stations, stream=None):
    """Time each kernel class's tiles (flush interval, kernel shape, persistent
    kernel or composed path) on these buffers and keep the fastest."""
    lib = load()
    c, keep1 = common.to_c()
    arr, keep = _stations_c(stations, common)
    _check(lib.epic_autotune(ctypes.byref(c), arr, len(stations), _stream(stream)))
