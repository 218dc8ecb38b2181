"""Host-side tests of the C ABI (no GPU): the library loads, exports every
function include/epic.h declares, and rejects bad arguments before any device
work (epic_validate runs all of image_cadence's checks on the host)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2411_17804_amd import epic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "epic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


def test_library_exports_every_declared_function():
    lib = epic.load()
    decl = declared_functions()
    assert set(decl) == set(epic.ABI_FUNCTIONS), decl
    for name in decl:
        assert hasattr(lib, name), name


def test_status_strings():
    assert epic.status_name(0) == "EPIC_OK"
    assert epic.status_name(-1) == "EPIC_ERR_INVALID_ARG"
    assert epic.status_name(-3) == "EPIC_ERR_OUT_OF_MEMORY"
    assert epic.status_name(-99) == "EPIC_ERR_UNKNOWN"


def _c2_like(n_chan=4, **over):
    cfg = W.make_config(2, n_chan=n_chan, n_time=8)
    st = cfg.stations[0]
    common = epic.Common(cfg.n_pol, cfg.wavelengths_m, W.GRID_SPACING_WL, cfg.n_time,
                         cfg.volt_type, epic.FP32_FFT)
    station = epic.Station(st.pos_m, st.nx, st.ny, st.kernel_type, st.support, st.sigma_cells,
                           volts=0x1000, image=0x2000)
    for k, v in over.items():
        setattr(common if hasattr(common, k) else station, k, v)
    return common, station


def test_validate_accepts_the_configs():
    for idx in (1, 2, 3, 5):
        cfg = W.make_config(idx, n_chan=None, n_time=4)
        common = epic.Common(cfg.n_pol, cfg.wavelengths_m, W.GRID_SPACING_WL, cfg.n_time,
                             cfg.volt_type, cfg.precision)
        sts = [epic.Station(s.pos_m, s.nx, s.ny, s.kernel_type, s.support, s.sigma_cells,
                            volts=0x1000, image=0x2000) for s in cfg.stations]
        epic.validate(common, sts)


@pytest.mark.parametrize("field,value", [
    ("n_pol", 3), ("n_time", 0), ("volt_type", 7), ("precision", 9), ("grid_spacing_wl", 0.0),
    ("grid_spacing_wl", float("nan")), ("nx", 48), ("ny", 512), ("nx", 8), ("support", 2),
    ("support", 9), ("kernel_type", 5), ("sigma_cells", -1.0), ("volts", None),
])
def test_validate_rejects(field, value):
    common, station = _c2_like(**{field: value})
    with pytest.raises(epic.EpicError) as e:
        epic.validate(common, [station])
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG


def test_validate_rejects_bad_wavelengths():
    for lam in (np.array([2.0, -1.0]), np.array([np.inf]), np.array([0.0])):
        common, station = _c2_like(wavelength_m=lam)
        with pytest.raises(epic.EpicError) as e:
            epic.validate(common, [station])
        assert e.value.status == epic.EPIC_ERR_INVALID_ARG


def test_validate_rejects_nearest_with_support():
    common, station = _c2_like(kernel_type=epic.KERNEL_NEAREST)
    with pytest.raises(epic.EpicError):
        epic.validate(common, [station])


def test_footprint_off_grid_at_some_channel_is_rejected():
    # the 38 m station fits a 64 grid at 150 MHz but not a 32 grid
    common, station = _c2_like(nx=32, ny=32)
    with pytest.raises(epic.EpicError) as e:
        epic.validate(common, [station])
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    assert "footprint" in e.value.detail
    # and a grid that only fails at the highest frequency channel of a wide band
    pos = np.array([[14.0, 0.0]])
    lam = np.array([2.2, 2.0, 1.8])          # cells: 12.7, 14.0, 15.6 from the centre
    common = epic.Common(1, lam, 0.5, 4, epic.CF32)
    st = epic.Station(pos, 32, 32, epic.KERNEL_GAUSSIAN, 3, 0.5, volts=0x1000, image=0x2000)
    with pytest.raises(epic.EpicError) as e:
        epic.validate(common, [st])
    assert "channel 2" in e.value.detail


def test_non_finite_position_rejected():
    common, station = _c2_like()
    pos = station.pos_m.copy()
    pos[3, 1] = np.nan
    station.pos_m = pos
    with pytest.raises(epic.EpicError):
        epic.validate(common, [station])


def test_unfused_calls_reject_bad_shapes_without_a_device():
    with pytest.raises(epic.EpicError) as e:
        epic.fft2_batched(48, 64, 1, epic.FP32_FFT, 0x1000, 0x1000, stream=0)
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    with pytest.raises(epic.EpicError):
        epic.fft2_batched(64, 64, 0, epic.FP32_FFT, 0x1000, 0x1000, stream=0)
    with pytest.raises(epic.EpicError):
        epic.fft2_batched(64, 64, 1, 5, 0x1000, 0x1000, stream=0)
    with pytest.raises(epic.EpicError):
        epic.accumulate_power(3, 64, 64, 1, 1, 0x1000, 0x1000, 0x1000, stream=0)
    with pytest.raises(epic.EpicError):
        epic.accumulate_power(2, 64, 64, 1, 1, 0x1000, 0x1000, 0x1000, finalize_n_time=4,
                              image=None, stream=0)
    for args in [(3, 64, 64, 1), (2, 48, 64, 1), (2, 64, 512, 1), (2, 64, 64, 0)]:
        with pytest.raises(epic.EpicError) as e:
            epic.image_to_visibilities(*args, 0x1000, 0x1000, stream=0)
        assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    with pytest.raises(epic.EpicError):
        epic.image_to_visibilities(2, 64, 64, 1, None, 0x1000, stream=0)
    for n_pol, nx, n_chan, imgs in [(3, 64, 1, [0x1000]), (2, 40, 1, [0x1000]), (2, 64, 0, [0x1000]),
                                    (2, 64, 1, []), (2, 64, 1, [0x1000] * 129),
                                    (2, 64, 1, [0x1000, None])]:
        with pytest.raises(epic.EpicError) as e:
            epic.combine_incoherent(n_pol, nx, 64, n_chan, imgs, 0x2000, stream=0)
        assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    common, station = _c2_like()
    with pytest.raises(epic.EpicError):
        epic.grid_voltages(common, station, 6, 4, 0x3000, stream=0)     # t0 + nt > n_time
    with pytest.raises(epic.EpicError):
        epic.grid_voltages(common, station, 0, 0, 0x3000, stream=0)


def test_xfft_calls_reject_bad_arguments_without_a_device():
    common, station = _c2_like()
    with pytest.raises(epic.EpicError) as e:
        epic.xfft_correlate(common, station, None, stream=0)
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    with pytest.raises(epic.EpicError) as e:
        epic.xfft_image(common, station, None, stream=0)
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    common, station = _c2_like(volts=None)
    with pytest.raises(epic.EpicError) as e:
        epic.xfft_correlate(common, station, 0x3000, stream=0)        # needs the voltages
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    common, station = _c2_like(image=None)
    with pytest.raises(epic.EpicError) as e:
        epic.xfft_image(common, station, 0x3000, stream=0)            # needs the image
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    common, station = _c2_like(n_pol=3)
    with pytest.raises(epic.EpicError) as e:
        epic.xfft_correlate(common, station, 0x3000, stream=0)
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    pos = np.zeros((70000, 2))
    common, station = _c2_like(pos_m=pos)
    with pytest.raises(epic.EpicError) as e:
        epic.xfft_correlate(common, station, 0x3000, stream=0)
    assert e.value.status == epic.EPIC_ERR_UNSUPPORTED


def test_array_cadence_rejects_bad_arguments_without_a_device():
    common, station = _c2_like()
    station.pos_m = station.pos_m[:8]
    station.nx = station.ny = 64
    ok = [0x1000] * 8
    for beams, nb, pix in [(None, 64, [0]), ([0x1000] * 7 + [None], 64, [0]), (ok, 48, [0]),
                           (ok, 64, []), (ok, 64, [64 * 64]), (ok, 64, [-1])]:
        for fn in (epic.array_cadence, epic.array_xfft):
            with pytest.raises(epic.EpicError) as e:
                fn(common, station, beams or [], nb, nb, pix, stream=0)
            assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    big = epic.Station(np.zeros((129, 2)), 64, 64, station.kernel_type, station.support,
                       station.sigma_cells, image=0x2000)
    with pytest.raises(epic.EpicError) as e:
        epic.array_cadence(common, big, [0x1000] * 129, 64, 64, [0], stream=0)
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG


def test_pol_calls_reject_bad_arguments_without_a_device():
    common, station = _c2_like()
    with pytest.raises(epic.EpicError) as e:
        epic.grid_voltages_pol(common, station, None, 0, 4, 0x3000, stream=0)
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    with pytest.raises(epic.EpicError) as e:
        epic.grid_voltages_pol(common, station, 0x4000, 6, 4, 0x3000, stream=0)
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    with pytest.raises(epic.EpicError) as e:
        epic.image_cadence_pol(common, station, None, stream=0)
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG
    common, station = _c2_like(image=None)
    with pytest.raises(epic.EpicError) as e:
        epic.image_cadence_pol(common, station, 0x4000, stream=0)
    assert e.value.status == epic.EPIC_ERR_INVALID_ARG


def test_struct_layout_matches_header():
    # epic_common: 2 x int32, pointer, double, 3 x int32 (+ pad) ; epic_station as declared
    assert ctypes.sizeof(epic._Common) == 40
    assert ctypes.sizeof(epic._Kernel) == 16
    assert ctypes.sizeof(epic._Station) == 56


class _FakeDeviceTensor:
    """Stands in for a GPU tensor on the host: the binding only looks at
    is_cuda, dtype, contiguity, size and address."""

    def __init__(self, shape, dtype="float32", contiguous=True, cuda=True):
        import torch
        self.shape = tuple(shape)
        self.dtype = getattr(torch, dtype)
        self._contig = contiguous
        self.is_cuda = cuda
        self.device = "cuda:0" if cuda else "cpu"
        self._es = torch.empty((), dtype=self.dtype).element_size()

    def is_contiguous(self):
        return self._contig

    def numel(self):
        return int(np.prod(self.shape))

    def element_size(self):
        return self._es

    def data_ptr(self):
        return 0x7000


def test_binding_checks_device_buffers_before_the_call():
    n_chan, nt, n_pol, ny, nx = 2, 3, 2, 64, 64
    good = (n_chan, nt, n_pol, ny, nx, 2)
    # a correctly shaped buffer passes the checks (and then fails in the
    # library only because no GPU is present: the fake address is never used)
    common, station = _c2_like(n_chan=n_chan)
    station.volts = _FakeDeviceTensor((n_chan, common.n_time, 256, 2, 2), "int8")
    cases = {
        "host tensor": _FakeDeviceTensor(good, cuda=False),
        "wrong dtype": _FakeDeviceTensor(good, "float64"),
        "not contiguous": _FakeDeviceTensor(good, contiguous=False),
        "too small": _FakeDeviceTensor((n_chan, nt, n_pol, ny, nx - 1, 2)),
        "too large": _FakeDeviceTensor((n_chan, nt + 1, n_pol, ny, nx, 2)),
    }
    for name, grid in cases.items():
        with pytest.raises(ValueError):
            epic.grid_voltages(common, station, 0, nt, grid, stream=0)
    # complex64 of the same bytes is accepted by the checks
    ok = _FakeDeviceTensor((n_chan, nt, n_pol, ny, nx), "complex64")
    with pytest.raises(epic.EpicError):
        epic.grid_voltages(common, station, 0, nt, ok, stream=0)


def test_binding_checks_voltage_type_and_size():
    common, station = _c2_like(n_chan=2)
    station.image = _FakeDeviceTensor((2, 4, 64, 64, 2))
    for v in (_FakeDeviceTensor((2, common.n_time, 256, 2, 2), "float32"),     # ci8 config
              _FakeDeviceTensor((2, common.n_time, 255, 2, 2), "int8"),
              _FakeDeviceTensor((2, common.n_time, 256, 2, 2), "int8", contiguous=False)):
        station.volts = v
        with pytest.raises(ValueError):
            epic.image_cadence(common, [station], stream=0)
    station.volts = _FakeDeviceTensor((2, common.n_time, 256, 2, 2), "int8")
    station.image = _FakeDeviceTensor((2, 1, 64, 64, 2))                       # n_pol 2 needs 4 products
    with pytest.raises(ValueError):
        epic.image_cadence(common, [station], stream=0)


def test_binding_checks_unfused_call_buffers():
    n = (3, 64, 64, 2)
    with pytest.raises(ValueError):
        epic.fft2_batched(64, 64, 3, epic.FP32_FFT, _FakeDeviceTensor(n), _FakeDeviceTensor((2, 64, 64, 2)),
                          stream=0)
    shape = (2, 4, 32, 16, 2)
    with pytest.raises(ValueError):
        epic.accumulate_power(2, 16, 32, 2, 5, _FakeDeviceTensor((2, 5, 2, 32, 16, 2)),
                              _FakeDeviceTensor(shape), _FakeDeviceTensor((2, 4, 32, 16)), 5,
                              _FakeDeviceTensor(shape), stream=0)
    with pytest.raises(ValueError):
        epic.combine_incoherent(2, 16, 32, 2, [_FakeDeviceTensor(shape)] * 2, _FakeDeviceTensor(shape),
                                _FakeDeviceTensor((2, 4, 32, 16), "float64"), stream=0)
