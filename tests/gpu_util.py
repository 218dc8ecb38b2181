"""Helpers for the GPU tests: move seeded inputs to the device, run the ABI
calls, bring results back as complex128 numpy arrays."""
from __future__ import annotations

import sys

import numpy as np

import workloads as W


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def to_device_volts(v: np.ndarray):
    """numpy voltages (complex64, or int8 with a trailing (re, im) axis) -> torch."""
    torch = torch_cuda()
    if v.dtype == np.int8:
        return torch.from_numpy(np.ascontiguousarray(v)).cuda()
    return torch.from_numpy(np.ascontiguousarray(v).view(np.float32)).cuda()


def to_complex(t) -> np.ndarray:
    """torch float32 tensor with a trailing (re, im) axis -> complex128 numpy."""
    a = t.detach().cpu().numpy()
    return a[..., 0].astype(np.float64) + 1j * a[..., 1].astype(np.float64)


def from_complex(a: np.ndarray):
    torch = torch_cuda()
    b = np.stack([a.real, a.imag], axis=-1).astype(np.float32)
    return torch.from_numpy(b).cuda()


def station_objects(cfg: W.Config, volts_list, precision=None):
    """epic.Common + epic.Station list with device voltages and zeroed images."""
    from paper_2411_17804_amd import epic
    torch = torch_cuda()
    common = epic.Common(cfg.n_pol, cfg.wavelengths_m, W.GRID_SPACING_WL, cfg.n_time,
                         cfg.volt_type, cfg.precision if precision is None else precision)
    stations = []
    for st, v in zip(cfg.stations, volts_list):
        img = torch.zeros((cfg.n_chan, cfg.n_pol * cfg.n_pol, st.ny, st.nx, 2),
                          dtype=torch.float32, device="cuda")
        stations.append(epic.Station(st.pos_m, st.nx, st.ny, st.kernel_type, st.support,
                                     st.sigma_cells, volts=v, image=img))
    return common, stations


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
