"""The FP64 oracle against facts fixed outside it (CPU only).

See tests/oracle_pins.py for what each pin is tied to.  The mutation test
compiles deliberately broken copies of the oracle (one plausible mistake each:
a flipped sign, a dropped conjugate, transposed axes, a missing normalisation,
...) and checks that every one of them fails at least one pin other than the
numpy cross-check.
"""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle
from tests import oracle_pins as P


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


@pytest.mark.parametrize("name", sorted(P.ALL_PINS))
def test_pin(lib, name):
    err = P.ALL_PINS[name](lib)
    assert err <= P.PIN_TOL[name], f"pin {name}: error {err:.3e} > {P.PIN_TOL[name]:.1e}"


def test_offgrid_is_an_error(lib):
    # an element whose 3x3 footprint crosses the grid edge (never wrapped)
    pos = np.array([[-7.6, 0.0]])                 # u = 0.4 -> cell 0, footprint -1..1
    with pytest.raises(oracle.OracleError) as e:
        oracle.plan(pos, 2.0, 0.5, 16, 16, oracle.KERNEL_GAUSSIAN, 3, 0.5, lib=lib)
    assert e.value.code == oracle.ERR_OFFGRID
    with pytest.raises(oracle.OracleError):
        oracle.plan(pos, 2.0, 0.5, 16, 16, oracle.KERNEL_NEAREST, 3, 0.5, lib=lib)  # K must be 1


def test_channel_geometry_scales_with_wavelength(lib):
    # the grid is fixed in wavelengths: doubling lambda halves the cell offset of an element
    pos = np.array([[4.0, -2.0]])
    ix1, iy1, _, _ = oracle.plan(pos, 1.0, 0.5, 32, 32, oracle.KERNEL_NEAREST, 1, 0.0, lib=lib)
    ix2, iy2, _, _ = oracle.plan(pos, 2.0, 0.5, 32, 32, oracle.KERNEL_NEAREST, 1, 0.0, lib=lib)
    assert (ix1[0] - 16, iy1[0] - 16) == (8, -4)
    assert (ix2[0] - 16, iy2[0] - 16) == (4, -2)


def test_ci8_conversion_is_exact(lib):
    rng = np.random.default_rng(3)
    raw = rng.integers(-127, 128, (1, 3, 5, 2, 2)).astype(np.int8)
    as_c = (raw[..., 0].astype(np.float64) + 1j * raw[..., 1]).astype(np.complex128)
    pos = rng.uniform(-2, 2, (5, 2))
    a = oracle.image(pos, np.array([2.0]), 0.5, 16, 16, oracle.KERNEL_GAUSSIAN, 3, 0.5, raw, lib=lib)
    b = oracle.image(pos, np.array([2.0]), 0.5, 16, 16, oracle.KERNEL_GAUSSIAN, 3, 0.5, as_c, lib=lib)
    assert np.array_equal(a, b)


def _vis_mutants():
    # plausible slips in the Python correlator (Eq. 4), planted on the CPU
    def prep(volts):
        if volts.dtype == np.int8:
            return volts[..., 0].astype(np.float64) + 1j * volts[..., 1]
        return volts.astype(np.complex128)

    def no_conj(volts):
        v = prep(volts)
        X = v.reshape(v.shape[0], v.shape[1], -1)
        return np.stack([x.T @ x / v.shape[1] for x in X]).reshape(
            v.shape[0], v.shape[2], v.shape[3], v.shape[2], v.shape[3])

    def conj_first(volts):
        v = prep(volts)
        X = v.reshape(v.shape[0], v.shape[1], -1)
        return np.stack([np.conj(x.T) @ x / v.shape[1] for x in X]).reshape(
            v.shape[0], v.shape[2], v.shape[3], v.shape[2], v.shape[3])

    def sum_not_mean(volts):
        return oracle.visibilities(volts) * prep(volts).shape[1]

    def pol_major(volts):
        v = prep(volts)
        n_c, n_t, n_e, n_p = v.shape
        X = np.transpose(v, (0, 1, 3, 2)).reshape(n_c, n_t, -1)     # rows (p, a), read as (a, p)
        return np.stack([x.T @ np.conj(x) / n_t for x in X]).reshape(n_c, n_e, n_p, n_e, n_p)

    return {"no_conj": no_conj, "conj_first": conj_first, "sum_not_mean": sum_not_mean,
            "pol_major": pol_major}


@pytest.mark.parametrize("mutant", sorted(_vis_mutants()))
def test_correlator_pin_catches_mistakes(lib, mutant):
    err = P.pin_visibility_correlator(lib, vis_fn=_vis_mutants()[mutant])
    assert not err <= P.PIN_TOL["visibility_correlator"], mutant


def _array_mutants():
    # plausible slips in the Python inter-station composition (Eq. 10), on the CPU
    def build(transpose_pix=False, conj=False, lam0=False, rev_st=False):
        def fn(beams, pixels, array_pos_m, wavelengths_m, *rest, lib=None):
            b = [np.conj(x) if conj else x for x in beams]
            if rev_st:
                b = b[::-1]
            pix = np.asarray(pixels)
            if transpose_pix:
                ny, nx = np.asarray(beams[0]).shape[-2:]
                pix = (pix % nx) * ny + pix // nx
            lam = np.full_like(np.asarray(wavelengths_m, float), wavelengths_m[0]) if lam0 else wavelengths_m
            return oracle.array_image(b, pix, array_pos_m, lam, *rest, lib=lib)
        return fn

    return {"transposed_pixel": build(transpose_pix=True), "conj_beams": build(conj=True),
            "first_wavelength": build(lam0=True), "stations_reversed": build(rev_st=True)}


@pytest.mark.parametrize("mutant", sorted(_array_mutants()))
def test_array_pins_catch_mistakes(lib, mutant):
    fn = _array_mutants()[mutant]
    errs = [P.pin_array_point_source(lib, array_fn=fn), P.pin_array_single_station(lib, array_fn=fn)]
    assert not (errs[0] <= P.PIN_TOL["array_point_source"]
                and errs[1] <= P.PIN_TOL["array_single_station"]), (mutant, errs)


def _pol_mutants():
    # plausible slips in the polarimetric gridding, planted on the CPU by
    # handing the true routine a mis-indexed kernel table
    def wrap(f):
        return lambda pos, lams, dwl, nx, ny, K, kern, E, lib=None: oracle.image_pol(
            pos, lams, dwl, nx, ny, K, f(np.asarray(kern)), E, lib=lib)

    return {"dropped_conj": wrap(np.conj),
            "pol_axes_swapped": wrap(lambda k: np.swapaxes(k, 2, 3)),
            "dx_dy_swapped": wrap(lambda k: np.swapaxes(k, 4, 5))}


@pytest.mark.parametrize("mutant", sorted(_pol_mutants()))
def test_pol_pin_catches_mistakes(lib, mutant):
    err = P.pin_pol_kernels(lib, image_fn=_pol_mutants()[mutant])
    assert not err <= P.PIN_TOL["pol_kernels"], mutant


# (source fragment, replacement) -- each a plausible slip in the oracle
MUTANTS = {
    "transform_sign": ("const double ang = EO_TWO_PI *", "const double ang = -EO_TWO_PI *"),
    "dropped_conj": ("s[k] += fa[k] * conj(fb[k]);", "s[k] += fa[k] * fb[k];"),
    "transposed_cells": ("(size_t)(iy[a] + dy) * nx + (ix[a] + dx)",
                         "(size_t)(ix[a] + dx) * nx + (iy[a] + dy)"),
    "unnormalised_kernel": ("wx[d] /= sx;", "wx[d] /= 1.0;"),
    "mean_divisor": ("out[k] = S[k] / (double)n_time;", "out[k] = S[k] / (double)(n_time + 1);"),
    "offset_sign": ("const double ex = ((double)d - du)", "const double ex = ((double)d + du)"),
    "product_order": ("S + (size_t)(a * n_pol + b) * npix", "S + (size_t)(b * n_pol + a) * npix"),
    "twiddle_index": ("const double complex w = eo_root(k, len);",
                      "const double complex w = eo_root(k, n);"),
    "rounding": ("const double ci = floor(u + 0.5);", "const double ci = floor(u);"),
    "origin": ("const double u = x_m / delta_m + (double)(nx / 2);",
               "const double u = x_m / delta_m + (double)(nx / 2) + 0.5;"),
}


_RUN_PINS = """
import sys, numpy as np
sys.path.insert(0, {root!r})
import oracle
from tests import oracle_pins as P
lib = oracle.load({so!r})
for name, fn in P.ALL_PINS.items():
    if name == "numpy_crosscheck":
        continue
    try:
        err = fn(lib)
    except oracle.OracleError:
        err = np.inf
    if not err <= P.PIN_TOL[name]:
        print("FAILED", name, flush=True)
"""


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_every_plausible_mistake_fails_a_pin(mutant):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "epic_oracle.c")).read()
    frag, repl = MUTANTS[mutant]
    assert src.count(frag) == 1, f"mutation fragment for {mutant} not found exactly once"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mut.c")
        with open(path, "w") as f:
            f.write(src.replace(frag, repl))
        so = oracle.build(src=path, out=os.path.join(d, "libmut.so"))
        # a mutant may also write out of bounds and crash: that counts as caught
        r = subprocess.run([sys.executable, "-c", _RUN_PINS.format(root=root, so=so)],
                           capture_output=True, text=True, timeout=300)
        caught = "FAILED" in r.stdout or r.returncode != 0
        assert caught, f"mutant {mutant} passes every paper/maths pin"


def _image_error_mutants():
    # plausible slips in the per-image error metric, planted on the CPU
    def autos(ref, n_pol):
        return [np.abs(ref[..., a * n_pol + a, :, :]).max(axis=(-1, -2)) for a in range(n_pol)]

    def with_scale(scale_fn, reduce_axes=(-1, -2), reducer=np.max):
        def fn(img, ref, n_pol):
            diff = reducer(np.abs(np.asarray(img) - np.asarray(ref)), axis=reduce_axes)
            return diff / scale_fn(np.asarray(ref), n_pol, diff.shape)
        return fn

    def sqrt_scale(ref, n_pol, shape):
        au = autos(ref, n_pol)
        return np.stack([np.sqrt(au[a] * au[b]) for a in range(n_pol) for b in range(n_pol)], -1)

    def largest_of_all(ref, n_pol, shape):
        m = np.abs(ref).max(axis=(-1, -2)).max(axis=-1, keepdims=True)
        return np.broadcast_to(m, shape)

    def no_sqrt(ref, n_pol, shape):
        au = autos(ref, n_pol)
        return np.stack([au[a] * au[b] for a in range(n_pol) for b in range(n_pol)], -1)

    def own_max(ref, n_pol, shape):
        return np.abs(ref).max(axis=(-1, -2))

    def other_auto(ref, n_pol, shape):
        au = autos(ref, n_pol)
        return np.stack([np.sqrt(au[n_pol - 1 - a] * au[n_pol - 1 - b])
                         for a in range(n_pol) for b in range(n_pol)], -1)

    def per_pixel(img, ref, n_pol):
        with np.errstate(divide="ignore", invalid="ignore"):
            return (np.abs(img - ref) / np.abs(ref)).max(axis=(-1, -2))

    return {"largest_of_all_four": with_scale(largest_of_all),
            "dropped_sqrt": with_scale(no_sqrt),
            "cross_scaled_by_itself": with_scale(own_max),
            "autos_swapped": with_scale(other_auto),
            "wrong_axes": with_scale(sqrt_scale, reduce_axes=(-3, -1)),
            "mean_not_max": with_scale(sqrt_scale, reducer=np.mean),
            "per_pixel_relative": per_pixel}


@pytest.mark.parametrize("mutant", sorted(_image_error_mutants()))
def test_image_error_pin_catches_mistakes(lib, mutant):
    try:
        err = P.pin_image_error(lib, err_fn=_image_error_mutants()[mutant])
    except (ValueError, IndexError):
        err = float("inf")
    assert not err <= P.PIN_TOL["image_error"], mutant
