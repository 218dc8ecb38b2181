"""GPU parity of coherent inter-station EPIC (Sec. 6.2, Eq. 10 then Eq. 9):
station fields from grid_voltages + fft2_batched, then array_cadence, against
the FP64 oracle's two-level composition (oracle.station_beams, then
oracle.array_image) on the same seeded inputs.  Tolerance: the c-14 metric,
FP32 gate 1e-5, per (channel, pixel) array image."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import from_complex, say, to_complex, torch_cuda

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    t = torch_cuda()
    from paper_2411_17804_amd import epic
    epic.load()
    return t


def _scene(seed, n_st, n_el, n_pol, n_time, lams):
    # stations of n_el elements within +-3 m of their centres; centres within
    # +-24 m; noise plus a plane wave from l = (1/8, -1/8)
    rng = np.random.default_rng([17804, 10, seed])
    elems = [rng.uniform(-3.0, 3.0, (n_el, 2)) for _ in range(n_st)]
    cen = rng.uniform(-24.0, 24.0, (n_st, 2))
    l = np.array([1.0 / 8, -1.0 / 8])
    volts = []
    for m in range(n_st):
        v = (rng.standard_normal((len(lams), n_time, n_el, n_pol))
             + 1j * rng.standard_normal((len(lams), n_time, n_el, n_pol))) * 0.5
        for c, lam in enumerate(lams):
            ph = np.exp(-2j * np.pi * ((cen[m] + elems[m]) @ l) / lam)
            a = rng.standard_normal(n_time) + 1j * rng.standard_normal(n_time)
            v[c] += 2.0 * a[:, None, None] * ph[None, :, None]
        volts.append(v.astype(np.complex64).astype(np.complex128))
    return elems, cen, volts


def _gpu_beams(epic, torch, elems, volts, lams, n_pol, n_time, nb, K):
    from tests.gpu_util import to_device_volts
    beams = []
    for pos, v in zip(elems, volts):
        common = epic.Common(n_pol, lams, 0.5, n_time, W.CF32, epic.FP32_FFT)
        st = epic.Station(pos, nb, nb, W.KERNEL_GAUSSIAN if K > 1 else W.KERNEL_NEAREST, K,
                          K / 6.0, volts=to_device_volts(v.astype(np.complex64)))
        g = torch.empty((len(lams), n_time, n_pol, nb, nb, 2), dtype=torch.float32, device="cuda")
        epic.grid_voltages(common, st, 0, n_time, g)
        epic.fft2_batched(nb, nb, len(lams) * n_time * n_pol, epic.FP32_FFT, g, g)
        beams.append(g)
    return beams


ARRAY_CASES = {
    # name: (stations, elements, pols, samples, beam grid, station K, array grid, array K, pixels)
    "fp16-array-2pol": (5, 10, 2, 20, 16, 3, 32, 3, "some"),
    "nearest-2pol-all": (4, 12, 2, 24, 16, 3, 16, 1, "all"),
    "gauss-1pol": (6, 9, 1, 20, 16, 1, 32, 3, "some"),
    "32grid-2pol": (3, 20, 2, 16, 32, 3, 16, 3, "some"),
}


@pytest.mark.parametrize("case", sorted(ARRAY_CASES))
def test_array_cadence(torch, case, monkeypatch):
    from paper_2411_17804_amd import epic
    n_st, n_el, n_pol, nt, nb, Ks, na, Ka, sel = ARRAY_CASES[case]
    say(f"array_cadence {case}")
    lams = np.array([2.0, 1.5])
    elems, cen, volts = _scene(len(case), n_st, n_el, n_pol, nt, lams)
    rng = np.random.default_rng([17804, 11])
    pix = (np.arange(nb * nb) if sel == "all"
           else np.sort(rng.choice(nb * nb, 37, replace=False))).astype(np.int32)
    beams = _gpu_beams(epic, torch, elems, volts, lams, n_pol, nt, nb, Ks)
    ktype = W.KERNEL_GAUSSIAN if Ka > 1 else W.KERNEL_NEAREST
    prec = epic.FP16_SPLIT if case.startswith("fp16") else epic.FP32_FFT
    common = epic.Common(n_pol, lams, 4.0, nt, W.CF32, prec)
    img = torch.zeros((len(lams), pix.size, n_pol ** 2, na, na, 2), dtype=torch.float32, device="cuda")
    arr = epic.Station(cen, na, na, ktype, Ka, Ka / 6.0, image=img)
    epic.array_cadence(common, arr, beams, nb, nb, pix)
    torch.cuda.synchronize()
    got = to_complex(img)
    skt = W.KERNEL_GAUSSIAN if Ks > 1 else W.KERNEL_NEAREST
    obeams = [oracle.station_beams(e, lams, 0.5, nb, nb, skt, Ks, Ks / 6.0, v)
              for e, v in zip(elems, volts)]
    ref = oracle.array_image(obeams, pix, cen, lams, 4.0, na, na, ktype, Ka, Ka / 6.0)
    worst = 0.0
    for c in range(len(lams)):
        for s in range(pix.size):
            worst = max(worst, float(oracle.image_error(got[c, s], ref[c, s], n_pol).max()))
    say(f"  {case}: worst image error {worst:.2e} over {len(lams) * pix.size} array images")
    assert worst <= (1e-4 if prec == epic.FP16_SPLIT else FP32_TOL)
    # the chunking of the (channel, pixel) problems never changes the result
    monkeypatch.setenv("EPIC_ARRAY_BUDGET_KB", "16")          # chunks of a few problems
    img2 = torch.zeros_like(img)
    arr.image = img2
    epic.array_cadence(common, arr, beams, nb, nb, pix)
    torch.cuda.synchronize()
    assert torch.equal(img, img2)


@pytest.mark.parametrize("K", [1, 3])
def test_array_xfft_matches_array_cadence(torch, K):
    # the XFFT route at array scale (Eq. 11, 13) against the EPIC route and
    # the oracle: one image, up to FP32 rounding
    from paper_2411_17804_amd import epic
    say(f"array_xfft vs array_cadence, array kernel K={K}")
    n_st, n_el, n_pol, nt, nb, na = 6, 10, 2, 24, 16, 32
    lams = np.array([2.0, 1.5])
    elems, cen, volts = _scene(40 + K, n_st, n_el, n_pol, nt, lams)
    pix = np.sort(np.random.default_rng([17804, 12]).choice(nb * nb, 29, replace=False)).astype(np.int32)
    beams = _gpu_beams(epic, torch, elems, volts, lams, n_pol, nt, nb, 3)
    ktype = W.KERNEL_GAUSSIAN if K > 1 else W.KERNEL_NEAREST
    common = epic.Common(n_pol, lams, 4.0, nt, W.CF32, epic.FP32_FFT)
    shape = (len(lams), pix.size, n_pol ** 2, na, na, 2)
    a = torch.zeros(shape, dtype=torch.float32, device="cuda")
    b = torch.zeros(shape, dtype=torch.float32, device="cuda")
    epic.array_cadence(common, epic.Station(cen, na, na, ktype, K, K / 6.0, image=a), beams, nb, nb, pix)
    epic.array_xfft(common, epic.Station(cen, na, na, ktype, K, K / 6.0, image=b), beams, nb, nb, pix)
    torch.cuda.synchronize()
    ga, gb = to_complex(a), to_complex(b)
    obeams = [oracle.station_beams(e, lams, 0.5, nb, nb, W.KERNEL_GAUSSIAN, 3, 0.5, v)
              for e, v in zip(elems, volts)]
    ref = oracle.array_image(obeams, pix, cen, lams, 4.0, na, na, ktype, K, K / 6.0)
    worst_x = worst_ab = 0.0
    for c in range(len(lams)):
        for si in range(pix.size):
            worst_x = max(worst_x, float(oracle.image_error(gb[c, si], ref[c, si], n_pol).max()))
            worst_ab = max(worst_ab, float(oracle.image_error(gb[c, si], ga[c, si], n_pol).max()))
    say(f"  XFFT vs oracle {worst_x:.2e}, XFFT vs EPIC route {worst_ab:.2e}")
    assert worst_x <= FP32_TOL and worst_ab <= 2 * FP32_TOL
