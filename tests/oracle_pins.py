"""Pins of the FP64 oracle to facts fixed outside the oracle itself.

Each ``pin_*`` function takes a loaded oracle library (so the mutation test can
run it against deliberately broken builds of the oracle) and returns a
non-negative error that is ~1e-12 or smaller when the oracle is right.  The
thresholds live in ``PIN_TOL``.

What each pin is tied to:

* pin_fft_vs_bruteforce   -- the transform of Eq. 3 evaluated as a direct sum
                             (brute force) and by numpy's FFT library routine.
* pin_bf_equivalence      -- Eq. 1 (voltage beamforming over elements, not
                             cells) for elements on cell centres: EPIC with a
                             nearest-cell kernel must give the same image.
* pin_parseval            -- Parseval's theorem on the unnormalised transform.
* pin_point_source_centre -- a common signal on every element: the (0,0) pixel
                             is N_e^2 <|A|^2> and is the image maximum.
* pin_point_source_offset -- a plane wave from pixel k lands on pixel +k (sign).
* pin_xfft_equivalence    -- Eq. 4 then Eq. 6: visibilities (autocorrelations
                             included) gridded with the cross-correlated element
                             kernels and transformed equal the EPIC image
                             (Wiener-Khinchin on the circular grid).
* pin_visibility_closed_forms -- the directly gridded visibilities (the
                            FFT-correlator output, Eq. 4 then Eq. 6 without a
                            transform): explicit values for elements on cell
                            centres, the total equals the mean beam power at
                            zero, Hermitian symmetry between XY and YX.
* pin_visibility_correlator -- Eq. 4 on its own: element tones give
                            V_ab^{pq} = A_a^p conj(A_b^q) exactly; orthogonal
                            (Hadamard) codes give the identity matrix; random
                            voltages give a Hermitian positive semi-definite
                            matrix whose diagonal is the mean power.
* pin_array_point_source  -- Eq. 10 then Eq. 9 over station beams: a plane
                            wave on every element of M stations, with its
                            direction on both the station and the array pixel
                            grids, gives (M n_e)^2 <|A|^2> at the array pixel
                            of that direction, for the station pixel of that
                            direction, and that is the image maximum.
* pin_array_single_station -- one station at the array origin: its
                            array-scale image is flat and equals its own
                            station image at the selected pixel.
* pin_pol_kernels         -- Eq. 3 with full polarimetric complex kernels:
                            a real diagonal kernel built from the plan's
                            weights reproduces image(); a complex unitary pol
                            mix U turns the image into conj(U) I U^T; a linear
                            phase screen exp(-2 pi i k0.j / N) on the kernels
                            shifts the image by k0 pixels.
* pin_incoherent_combination -- Eq. 7 as a weighted mean: invariant under a
                            per-pixel rescaling of the weights, returns a lone
                            weighted station or identical images unchanged,
                            0 where all weights vanish, the plain mean for
                            equal weights.
* pin_translation         -- shifting every element by whole cells leaves the
                             power image unchanged.
* pin_pol_symmetry        -- YX = conj(XY) and Im XX = 0 exactly, XX >= 0.
* pin_golden_two_element  -- the hand-derived 4-cell example in tests/golden.
* pin_weights_closed_form -- the Gaussian weights' closed forms in tests/golden.
* pin_numpy_crosscheck    -- the separately written numpy oracle.
* pin_image_error         -- the per-image error metric that every GPU parity
                             gate uses, against hand-computed values in
                             tests/golden/image_error_cases.json (auto
                             products scaled by their own maximum, cross
                             products by the Cauchy-Schwarz bound
                             sqrt(max XX * max YY), maximum over pixels).
"""
from __future__ import annotations

import json
import os

import numpy as np

import oracle
from oracle import numpy_oracle as npo

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

PIN_TOL = {
    "fft_vs_bruteforce": 1e-12,
    "bf_equivalence": 1e-12,
    "parseval": 1e-12,
    "point_source_centre": 1e-12,
    "point_source_offset": 1e-12,
    "visibility_closed_forms": 1e-12,
    "incoherent_combination": 1e-13,
    "pol_kernels": 1e-12,
    "array_point_source": 1e-12,
    "array_single_station": 1e-12,
    "visibility_correlator": 1e-12,
    "xfft_equivalence": 1e-12,
    "translation": 1e-12,
    "pol_symmetry": 0.0,
    "golden_two_element": 1e-13,
    "weights_closed_form": 1e-14,
    "numpy_crosscheck": 1e-12,
    "image_error": 1e-15,
}


def _rng(tag):
    return np.random.default_rng([17804, tag])


def _cnormal(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def pin_fft_vs_bruteforce(lib):
    rng = _rng(1)
    worst = 0.0
    for ny, nx in [(4, 8), (8, 8), (16, 16), (16, 4), (2, 16)]:
        g = _cnormal(rng, (2, ny, nx))
        f = oracle.fft2(g, lib=lib)
        d = oracle.dft2(g, lib=lib)
        ref = np.fft.ifft2(g, axes=(-2, -1)) * (nx * ny)
        # the direct sum itself, written out for one output pixel as a third witness
        ky, kx = ny // 2 - 1, 1
        yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        one = np.sum(g[0] * np.exp(2j * np.pi * (kx * xx / nx + ky * yy / ny)))
        worst = max(worst, _rel(f, d), _rel(f, ref), abs(f[0, ky, kx] - one) / np.abs(ref).max())
    return worst


def _on_grid_layout(rng, n_elem, nx, ny, lam, dwl, margin):
    delta = dwl * lam
    cells = set()
    while len(cells) < n_elem:
        cells.add((int(rng.integers(margin, nx - margin)), int(rng.integers(margin, ny - margin))))
    cells = np.array(sorted(cells))
    pos = np.stack([(cells[:, 0] - nx // 2) * delta, (cells[:, 1] - ny // 2) * delta], axis=1)
    return pos


def pin_bf_equivalence(lib):
    rng = _rng(2)
    nx, ny, lam, dwl = 16, 8, 2.0, 0.5
    pos = _on_grid_layout(rng, 11, nx, ny, lam, dwl, 0)
    n_time, n_pol = 5, 2
    E = _cnormal(rng, (1, n_time, pos.shape[0], n_pol))
    img = oracle.image(pos, np.array([lam]), dwl, nx, ny, oracle.KERNEL_NEAREST, 1, 0.0, E,
                       lib=lib)[0]
    # Eq. 1 with unit directional weights: beamform towards every pixel direction
    kx = np.fft.fftfreq(nx, 1.0 / nx)            # natural order, signed k'
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    l = kx / (nx * dwl)
    m = ky / (ny * dwl)
    phase = np.exp(2j * np.pi * (m[:, None, None] * pos[None, None, :, 1]
                                 + l[None, :, None] * pos[None, None, :, 0]) / lam)  # [ny,nx,a]
    beam = np.einsum("yxa,tap->tpyx", phase, E[0])
    ref = np.stack([np.mean(beam[:, a] * np.conj(beam[:, b]), axis=0)
                    for a in range(n_pol) for b in range(n_pol)])
    return _rel(img, ref)


def pin_parseval(lib):
    rng = _rng(3)
    nx, ny, lam, dwl, K, sig = 16, 16, 2.0, 0.5, 3, 0.5
    pos = rng.uniform(-3.0, 3.0, (9, 2))
    E = _cnormal(rng, (1, 7, 9, 2))
    img = oracle.image(pos, np.array([lam]), dwl, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, E,
                       lib=lib)[0]
    G = oracle.grid(pos, lam, dwl, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, E[0], lib=lib)
    worst = 0.0
    for a in range(2):
        for b in range(2):
            lhs = img[a * 2 + b].sum()
            rhs = nx * ny * np.mean(np.sum(G[:, a] * np.conj(G[:, b]), axis=(-1, -2)))
            worst = max(worst, abs(lhs - rhs) / abs(img[0].sum()))
    return worst


def pin_point_source_centre(lib):
    rng = _rng(4)
    nx, ny, lam, dwl, K, sig = 32, 32, 2.0, 0.5, 3, 0.5
    pos = rng.uniform(-6.0, 6.0, (13, 2))
    A = _cnormal(rng, 6)
    E = np.broadcast_to(A[None, :, None, None], (1, 6, 13, 1)).copy()
    img = oracle.image(pos, np.array([lam]), dwl, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, E,
                       lib=lib)[0, 0].real
    expect = 13 ** 2 * np.mean(np.abs(A) ** 2)
    err = abs(img[0, 0] - expect) / expect
    if img.max() > img[0, 0] * (1 + 1e-12):
        err = max(err, 1.0)
    return err


def pin_point_source_offset(lib):
    rng = _rng(5)
    nx, ny, lam, dwl = 16, 16, 2.0, 0.5
    pos = _on_grid_layout(rng, 12, nx, ny, lam, dwl, 0)
    kxp, kyp = 3, -5                             # signed pixel of the source
    l, m = kxp / (nx * dwl), kyp / (ny * dwl)
    A = _cnormal(rng, 4)
    phase = np.exp(-2j * np.pi * (l * pos[:, 0] + m * pos[:, 1]) / lam)
    E = (A[:, None] * phase[None, :])[None, :, :, None]
    img = oracle.image(pos, np.array([lam]), dwl, nx, ny, oracle.KERNEL_NEAREST, 1, 0.0, E,
                       lib=lib)[0, 0].real
    expect = 12 ** 2 * np.mean(np.abs(A) ** 2)
    err = abs(img[kyp % ny, kxp % nx] - expect) / expect
    if np.unravel_index(np.argmax(img), img.shape) != (kyp % ny, kxp % nx):
        err = max(err, 1.0)
    return err


def pin_xfft_equivalence(lib):
    # the EPIC image (grid, + transform, square, mean) against the visibilities
    # of Eq. 4 gridded as in Eq. 6 (oracle.grid_visibilities, no transform)
    # and transformed with numpy: the two routes meet on the circular grid
    rng = _rng(6)
    nx, ny, lam, dwl, K, sig = 16, 16, 2.0, 0.5, 3, 0.5
    n_el, n_time, n_pol = 10, 9, 2
    pos = rng.uniform(-3.5, 3.5, (n_el, 2))
    E = _cnormal(rng, (1, n_time, n_el, n_pol))
    img = oracle.image(pos, np.array([lam]), dwl, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, E,
                       lib=lib)[0]
    Gv = oracle.grid_visibilities(pos, np.array([lam]), dwl, nx, ny, oracle.KERNEL_GAUSSIAN, K,
                                  sig, E, lib=lib)[0]
    ref = np.fft.ifft2(Gv, axes=(-2, -1)) * (nx * ny)
    return _rel(img, ref)


def pin_visibility_closed_forms(lib):
    # (a) nearest kernel, elements on cell centres, one sample: the grid holds
    # E_a conj(E_b) at each baseline cell c_a - c_b and sum_a |E_a|^2 at 0;
    # (b) Gaussian kernels: sum_j G^{pp}[j] = mean_t |sum_a E_a^p(t)|^2 (unit-sum
    # kernels), and G^{pq}[j] = conj(G^{qp}[-j]) (Hermitian)
    rng = _rng(12)
    nx = ny = 16
    lam, dwl = 2.0, 0.5
    cells = np.array([[0, 0], [3, 1], [-2, 4]])
    pos = cells * dwl * lam
    E = _cnormal(rng, (1, 1, 3, 1))
    G = oracle.grid_visibilities(pos, np.array([lam]), dwl, nx, ny, oracle.KERNEL_NEAREST, 1, 1.0,
                                 E, lib=lib)[0, 0]
    want = np.zeros((ny, nx), np.complex128)
    e = E[0, 0, :, 0]
    for a in range(3):
        for b in range(3):
            d = cells[a] - cells[b]
            want[d[1] % ny, d[0] % nx] += e[a] * np.conj(e[b])
    err = _rel(G, want)
    n_el, n_time, n_pol = 7, 5, 2
    pos = rng.uniform(-3.0, 3.0, (n_el, 2))
    E = _cnormal(rng, (1, n_time, n_el, n_pol))
    G = oracle.grid_visibilities(pos, np.array([lam]), dwl, nx, ny, oracle.KERNEL_GAUSSIAN, 3, 0.5,
                                 E, lib=lib)[0]
    for p in range(n_pol):
        tot = np.mean(np.abs(E[0, :, :, p].sum(axis=1)) ** 2)
        err = max(err, abs(G[p * n_pol + p].sum() - tot) / tot)
    flip = lambda g: np.roll(g[::-1, ::-1], 1, axis=(0, 1))   # j -> -j on the circular grid
    err = max(err, _rel(G[1], np.conj(flip(G[2]))))
    return err


def pin_visibility_correlator(lib, vis_fn=None):
    # (a) a tone per element and pol, E_a^p(t) = A_a^p exp(i w t): the mean
    # product is A_a^p conj(A_b^q) whatever w and n_time; (b) orthogonal +-1
    # codes (rows of a Sylvester-Hadamard matrix) with per-element phases give
    # the identity; (c) random voltages: Hermitian, PSD, diagonal = mean power
    vis_fn = vis_fn or oracle.visibilities
    rng = _rng(14)
    n_el, n_pol, n_time = 5, 2, 7
    A = _cnormal(rng, (n_el, n_pol))
    t = np.arange(n_time)
    E = A[None, :, :] * np.exp(1j * 0.7731 * t)[:, None, None]
    V = vis_fn(E[None])[0]
    want = A[:, :, None, None] * np.conj(A)[None, None, :, :]
    err = _rel(V, want)
    H = np.array([[1.0]])
    while H.shape[0] < 8:
        H = np.block([[H, H], [H, -H]])
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, 8))
    E = (H.T * ph[None, :])[:, :, None]                       # [t, a, 1]
    V = vis_fn(E[None])[0, :, 0, :, 0]
    err = max(err, float(np.abs(V - np.eye(8)).max()))
    E = _cnormal(rng, (2, 11, 4, 2))
    V = vis_fn(E).reshape(2, 8, 8)
    for c in range(2):
        err = max(err, _rel(V[c], np.conj(V[c].T)))
        ev = np.linalg.eigvalsh(0.5 * (V[c] + np.conj(V[c].T)))
        err = max(err, max(0.0, -ev.min()) / ev.max())
        power = np.mean(np.abs(E[c].reshape(11, 8)) ** 2, axis=0)
        err = max(err, _rel(np.diag(V[c]), power))
    return err


def _two_level_scene(rng, lams):
    # elements on station-grid cell centres (nearest kernel, exact), stations
    # on array-grid cells; a source at l = (1/8, -1/8): station pixel (1, -1)
    # of a 16-cell grid at lambda/2, array pixel (8, -8) of a 16-cell grid at
    # 4 lambda, for every lambda used
    n_el, n_st, n_time = 6, 3, 5
    cells = rng.choice(7 * 7, n_el, replace=False)
    elem = np.stack([cells % 7 - 3, cells // 7 - 3], axis=1).astype(np.float64)   # metres
    sc = rng.choice(7 * 7, n_st, replace=False)
    cen = np.stack([sc % 7 - 3, sc // 7 - 3], axis=1).astype(np.float64) * 8.0     # metres
    l = np.array([1.0 / 8, -1.0 / 8])
    A = _cnormal(rng, (len(lams), n_time))
    E = np.zeros((n_st, len(lams), n_time, n_el, 1), np.complex128)
    for m in range(n_st):
        for c, lam in enumerate(lams):
            ph = np.exp(-2j * np.pi * ((cen[m] + elem) @ l) / lam)               # [a]
            E[m, c, :, :, 0] = A[c][:, None] * ph[None, :]
    return elem, cen, E, A


def pin_array_point_source(lib, array_fn=None):
    array_fn = array_fn or oracle.array_image
    rng = _rng(15)
    lams = np.array([2.0, 1.0])
    elem, cen, E, A = _two_level_scene(rng, lams)
    n_st, n_el = cen.shape[0], elem.shape[0]
    beams = [oracle.station_beams(elem, lams, 0.5, 16, 16, oracle.KERNEL_NEAREST, 1, 0.0, E[m],
                                  lib=lib) for m in range(n_st)]
    ks = (1 % 16) + 16 * (-1 % 16)                    # station pixel (kx, ky) = (1, -1)
    other = 3 + 16 * 5
    img = array_fn(beams, [ks, other], cen, lams, 4.0, 16, 16, oracle.KERNEL_NEAREST, 1, 0.0,
                   lib=lib)
    err = 0.0
    for c in range(len(lams)):
        want = (n_st * n_el) ** 2 * np.mean(np.abs(A[c]) ** 2)
        got = img[c, 0, 0]
        err = max(err, abs(got[-8 % 16, 8] - want) / want)
        err = max(err, max(0.0, np.abs(got).max() - abs(got[-8 % 16, 8])) / want)
    return err


def pin_array_single_station(lib, array_fn=None):
    array_fn = array_fn or oracle.array_image
    rng = _rng(16)
    lams = np.array([2.0, 1.5])
    pos = rng.uniform(-2.0, 2.0, (7, 2))
    E = _cnormal(rng, (2, 6, 7, 2))
    beams = [oracle.station_beams(pos, lams, 0.5, 16, 16, oracle.KERNEL_GAUSSIAN, 3, 0.5, E,
                                  lib=lib)]
    st_img = oracle.image(pos, lams, 0.5, 16, 16, oracle.KERNEL_GAUSSIAN, 3, 0.5, E, lib=lib)
    pix = [0, 5 + 16 * 2, 15 + 16 * 9]
    img = array_fn(beams, pix, np.zeros((1, 2)), lams, 2.0, 16, 16, oracle.KERNEL_NEAREST, 1, 0.0,
                   lib=lib)
    err = 0.0
    for c in range(2):
        for si, k in enumerate(pix):
            want = st_img[c][:, k // 16, k % 16]                   # the 4 products at pixel k
            got = img[c, si]
            scale = np.abs(want).max()
            err = max(err, float(np.abs(got - want[:, None, None]).max()) / scale)
    return err


def pin_pol_kernels(lib, image_fn=None):
    image_fn = image_fn or oracle.image_pol
    rng = _rng(17)
    nx = ny = 16
    lams = np.array([2.0, 1.6])
    K, sig = 3, 0.5
    n_el, n_time, n_pol = 6, 5, 2
    pos = rng.uniform(-3.0, 3.0, (n_el, 2))
    E = _cnormal(rng, (2, n_time, n_el, n_pol))
    base = oracle.image(pos, lams, 0.5, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, E, lib=lib)
    diag = np.zeros((2, n_el, n_pol, n_pol, K, K), np.complex128)
    cells = []
    for c, lam in enumerate(lams):
        ix, iy, wx, wy = oracle.plan(pos, lam, 0.5, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, lib=lib)
        cells.append((ix, iy))
        for p in range(n_pol):
            diag[c, :, p, p] = wy[:, :, None] * wx[:, None, :]
    err = _rel(image_fn(pos, lams, 0.5, nx, ny, K, diag, E, lib=lib), base)
    # complex unitary pol mix: conj(U) I U^T
    q, _ = np.linalg.qr(_cnormal(rng, (2, 2)))
    kern = np.zeros_like(diag)
    for c in range(2):
        for a in range(n_pol):
            for p in range(n_pol):
                kern[c, :, a, p] = q[a, p] * diag[c, :, p, p]
    got = image_fn(pos, lams, 0.5, nx, ny, K, kern, E, lib=lib).reshape(2, 2, 2, ny, nx)
    b = base.reshape(2, 2, 2, ny, nx)
    want = np.einsum("ap,cpqyx,bq->cabyx", np.conj(q), b, q)
    err = max(err, _rel(got, want))
    # linear phase screen on the absolute cells: the image shifts by k0
    k0 = (3, -2)
    scr = diag.copy()
    h = (K - 1) // 2
    for c in range(2):
        ix, iy = cells[c]
        jx = ix[:, None] - h + np.arange(K)[None, :]          # [elem, dx]
        jy = iy[:, None] - h + np.arange(K)[None, :]          # [elem, dy]
        ph = np.exp(-2j * np.pi * (k0[0] * jx[:, None, :] / nx + k0[1] * jy[:, :, None] / ny))
        scr[c] = diag[c] * ph[:, None, None, :, :]
    got = image_fn(pos, lams, 0.5, nx, ny, K, scr, E, lib=lib)
    want = np.roll(base, (-k0[1], -k0[0]), axis=(-2, -1))
    err = max(err, _rel(got, want))
    return err


def pin_incoherent_combination(lib):
    # Eq. 7 as weighted mean: invariant under a per-pixel rescaling of all
    # weights; a single weighted station is returned as it is; identical
    # images come back unchanged for any weights; all-zero weights give 0
    rng = _rng(13)
    n_st, n_chan, nq, ny, nx = 4, 2, 4, 8, 8
    imgs = [_cnormal(rng, (n_chan, nq, ny, nx)) for _ in range(n_st)]
    w = rng.uniform(0.1, 2.0, (n_st, nq, ny, nx))
    base = oracle.combine_incoherent(imgs, w)
    err = _rel(oracle.combine_incoherent(imgs, w * rng.uniform(0.5, 3.0, (1, nq, ny, nx))), base)
    one = np.zeros_like(w)
    one[2] = rng.uniform(0.5, 1.5, (nq, ny, nx))
    err = max(err, _rel(oracle.combine_incoherent(imgs, one), imgs[2]))
    same = [imgs[0]] * n_st
    err = max(err, _rel(oracle.combine_incoherent(same, w), imgs[0]))
    zero = w.copy()
    zero[:, 1, 3, 5] = 0.0
    z = oracle.combine_incoherent(imgs, zero)
    err = max(err, float(np.abs(z[:, 1, 3, 5]).max()))
    err = max(err, _rel(oracle.combine_incoherent(imgs), np.mean(np.stack(imgs), axis=0)))
    return err


def pin_translation(lib):
    rng = _rng(7)
    nx, ny, lam, dwl, K, sig = 32, 32, 2.0, 0.5, 3, 0.5
    pos = rng.uniform(-4.0, 4.0, (15, 2))
    E = _cnormal(rng, (1, 4, 15, 2))
    a = oracle.image(pos, np.array([lam]), dwl, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, E, lib=lib)
    shift = np.array([3.0, -2.0]) * dwl * lam
    b = oracle.image(pos + shift, np.array([lam]), dwl, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, E,
                     lib=lib)
    return _rel(b, a)


def pin_pol_symmetry(lib):
    rng = _rng(8)
    nx, ny, lam, dwl, K, sig = 16, 16, 2.0, 0.5, 3, 0.5
    pos = rng.uniform(-3.0, 3.0, (8, 2))
    E = _cnormal(rng, (2, 5, 8, 2))
    img = oracle.image(pos, np.array([lam, 2.1]), dwl, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, E,
                       lib=lib)
    bad = 0.0
    bad += float(np.max(np.abs(img[:, 2] - np.conj(img[:, 1]))))
    bad += float(np.max(np.abs(img[:, 0].imag))) + float(np.max(np.abs(img[:, 3].imag)))
    bad += float(max(0.0, -img[:, 0].real.min())) + float(max(0.0, -img[:, 3].real.min()))
    return bad


def pin_golden_two_element(lib):
    g = json.load(open(os.path.join(GOLDEN, "two_element_fringe.json")))
    vx = np.array([complex(*v) for v in g["volts_x"]])
    vy = np.array([complex(*v) for v in g["volts_y"]])
    E = np.stack([vx, vy], axis=-1)[None, None]          # [1 chan, 1 time, 2 el, 2 pol]
    img = oracle.image(np.array(g["pos_m"]), np.array([g["wavelength_m"]]), g["grid_spacing_wl"],
                       g["nx"], g["ny"], oracle.KERNEL_NEAREST, 1, 0.0, E, lib=lib)[0]
    worst = 0.0
    for i, name in enumerate(["XX", "XY", "YX", "YY"]):
        want = np.array([complex(*v) for v in g[name]]).reshape(g["ny"], g["nx"])
        worst = max(worst, float(np.max(np.abs(img[i] - want))))
    return worst


def pin_weights_closed_form(lib):
    g = json.load(open(os.path.join(GOLDEN, "gaussian_weights.json")))
    worst = 0.0
    nx = ny = 16
    lam, dwl = 2.0, 0.5
    delta = lam * dwl
    for case in g["cases"]:
        K, sig, off = case["K"], case["sigma"], case["offset_cells"]
        # element off cell 5 by `off` cells in x and by -off in y
        pos = np.array([[(5 + off - nx // 2) * delta, (9 - off - ny // 2) * delta]])
        ix, iy, wx, wy = oracle.plan(pos, lam, dwl, nx, ny, oracle.KERNEL_GAUSSIAN, K, sig, lib=lib)
        want = np.array(case["w"])
        # x: offset +off; round-half-up moves +0.5 to the next cell
        want_ix = 6 if off == 0.5 else 5
        worst = max(worst, float(np.max(np.abs(wx[0] - want))))
        # y: offset -off is the mirror image (for -0.5 the cell stays, offset -0.5)
        want_y = want[::-1] if off != 0.5 else np.array(case["w"])
        worst = max(worst, float(np.max(np.abs(wy[0] - want_y))))
        if ix[0] != want_ix or iy[0] != 9:
            worst = max(worst, 1.0)
    return worst


def pin_numpy_crosscheck(lib):
    import workloads as W
    cfg = W.make_config(1, n_time=32)
    st = cfg.stations[0]
    v = W.station_volts(cfg, 0)
    a = oracle.image(st.pos_m, cfg.wavelengths_m, W.GRID_SPACING_WL, st.nx, st.ny,
                     st.kernel_type, st.support, st.sigma_cells, v, lib=lib)
    b = npo.image(st.pos_m, cfg.wavelengths_m, W.GRID_SPACING_WL, st.nx, st.ny, st.support,
                  st.sigma_cells, True, v)
    cfg2 = W.make_config(2, n_chan=2, n_time=4)
    st2 = cfg2.stations[0]
    v2 = W.station_volts(cfg2, 0)
    c = oracle.image(st2.pos_m, cfg2.wavelengths_m, W.GRID_SPACING_WL, st2.nx, st2.ny,
                     st2.kernel_type, st2.support, st2.sigma_cells, v2, lib=lib)
    d = npo.image(st2.pos_m, cfg2.wavelengths_m, W.GRID_SPACING_WL, st2.nx, st2.ny, st2.support,
                  st2.sigma_cells, False, v2)
    return max(_rel(a, b), _rel(c, d))


def _golden_complex(a):
    a = np.asarray(a, np.float64)
    return a[..., 0] + 1j * a[..., 1]


def pin_image_error(lib, err_fn=None):
    """The error metric against hand-computed values (no imaging involved:
    lib is unused and kept for the common pin signature)."""
    err_fn = err_fn or oracle.image_error
    g = json.load(open(os.path.join(GOLDEN, "image_error_cases.json")))
    worst = 0.0
    for case in g["cases"]:
        ref = _golden_complex(case["ref"])
        img = ref + _golden_complex(case["delta"])
        want = np.asarray(case["expected"], np.float64)
        got = np.asarray(err_fn(img, ref, case["n_pol"]), np.float64)
        if got.shape != want.shape or not np.all(np.isfinite(got)):
            return float("inf")
        worst = max(worst, float(np.max(np.abs(got - want))))
    return worst


ALL_PINS = {
    "fft_vs_bruteforce": pin_fft_vs_bruteforce,
    "bf_equivalence": pin_bf_equivalence,
    "parseval": pin_parseval,
    "point_source_centre": pin_point_source_centre,
    "point_source_offset": pin_point_source_offset,
    "xfft_equivalence": pin_xfft_equivalence,
    "visibility_closed_forms": pin_visibility_closed_forms,
    "incoherent_combination": pin_incoherent_combination,
    "pol_kernels": pin_pol_kernels,
    "array_point_source": pin_array_point_source,
    "array_single_station": pin_array_single_station,
    "visibility_correlator": pin_visibility_correlator,
    "translation": pin_translation,
    "pol_symmetry": pin_pol_symmetry,
    "golden_two_element": pin_golden_two_element,
    "weights_closed_form": pin_weights_closed_form,
    "numpy_crosscheck": pin_numpy_crosscheck,
    "image_error": pin_image_error,
}
