"""The allocation-free entry point, image_cadence_noalloc, against
image_cadence on the same inputs (the same kernels run, so the images must
be bit-identical), on two calls in a row, the second with a smaller input;
device memory must not change across a call; a call whose tables exceed the
fixed scratch array is refused before any launch."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import say, station_objects, to_device_volts, torch_cuda

pytestmark = pytest.mark.gpu


def _pair(cfg, prec):
    volts = [to_device_volts(W.station_volts(cfg, s)) for s in range(len(cfg.stations))]
    a = station_objects(cfg, volts, prec)
    b = station_objects(cfg, volts, prec)
    return a, b


@pytest.mark.parametrize("prec", [W.FP32_FFT, W.FP16_SPLIT])
def test_noalloc_matches_image_cadence(prec):
    torch = torch_cuda()
    from paper_2411_17804_amd import epic
    epic.load()
    # no tuned choices from earlier calls: a class tuned to its composed path
    # would run other kernels in image_cadence than the persistent ones here
    epic.cache_clear()
    name = "fp32" if prec == W.FP32_FFT else "fp16-split"
    # first call: a hierarchical batch (3 stations, 6 channels, ragged
    # cadence) of grids up to 64, and in split precision one 128 x 128 station
    # too (its persistent kernel); second call: smaller (one station, 2
    # channels, fewer samples)
    big = W.make_config(4, chan_subset=[0, 9, 20, 33, 47, 63], n_time=41, n_stations=24, precision=prec)
    small_grids = [s for s in big.stations if s.nx <= 64]
    big.stations = small_grids[:3] if prec == W.FP32_FFT else \
        small_grids[:2] + [s for s in big.stations if s.nx == 128][:1]
    small = W.make_config(2, chan_subset=[5, 600], n_time=23, precision=prec)
    free_after_first = None
    for k, cfg in enumerate((big, small)):
        say(f"noalloc {name} call {k}: {len(cfg.stations)} station(s), {cfg.n_chan} channels x {cfg.n_time}")
        (ca, sa), (cb, sb) = _pair(cfg, prec)
        epic.image_cadence(ca, sa)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        epic.image_cadence_noalloc(cb, sb)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        if k == 1:
            assert free1 == free0, f"device memory changed across the call: {free0} -> {free1}"
        for s, (x, y) in enumerate(zip(sa, sb)):
            assert torch.equal(x.image, y.image), f"station {s}: images differ from image_cadence"
        free_after_first = free1
    assert free_after_first is not None


def test_noalloc_refuses_what_it_cannot_hold():
    torch = torch_cuda()
    from paper_2411_17804_amd import epic
    epic.load()
    # a 128 x 128 station at FP32 needs the footprint-box buffer
    cfg = W.make_config(3, chan_subset=[0], n_time=4, precision=W.FP32_FFT)
    (c, s), _ = _pair(cfg, W.FP32_FFT)
    with pytest.raises(epic.EpicError) as e:
        epic.image_cadence_noalloc(c, s)
    assert e.value.status == epic.EPIC_ERR_UNSUPPORTED, e.value
    # tables beyond the fixed array: the station-scale layout over 4 x 1024
    # channels (about 31 KB of tables per channel, 127 MB in all)
    cfg = W.make_config(2, n_chan=1024, n_time=2, precision=W.FP32_FFT)
    cfg.wavelengths_m = np.tile(cfg.wavelengths_m, 4)
    cfg.chan_ids = np.tile(cfg.chan_ids, 4)
    st = cfg.stations[0]
    img = torch.zeros((cfg.n_chan, 4, st.ny, st.nx, 2), dtype=torch.float32, device="cuda")
    volts = torch.zeros((cfg.n_chan, cfg.n_time, st.n_elem, 2, 2), dtype=torch.int8, device="cuda")
    c = epic.Common(cfg.n_pol, cfg.wavelengths_m, W.GRID_SPACING_WL, cfg.n_time, cfg.volt_type, W.FP32_FFT)
    s = epic.Station(st.pos_m, st.nx, st.ny, st.kernel_type, st.support, st.sigma_cells, volts=volts, image=img)
    with pytest.raises(epic.EpicError) as e:
        epic.image_cadence_noalloc(c, [s])
    assert e.value.status == epic.EPIC_ERR_UNSUPPORTED and "bytes" in e.value.detail, e.value
