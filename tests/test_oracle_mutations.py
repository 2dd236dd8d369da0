"""Plausible mistakes planted in copies of the oracle must fail a pin.

Each mutant is a small edit of an oracle function (a flipped sign, a swapped
axis, a dropped normalisation, an off-by-one range).  The pins in
``tests/pins.py`` must reject every one of them; this shows they constrain
the oracle rather than merely re-typing it.  CPU only.
"""

import math

import numpy as np
import pytest

from oracle import optics, pca, post, temporal
from tests import pins


# ---------------------------------------------------------------- AS mutants

def as_z_sign(x, lam, dx, dy, z):
    return optics.angular_spectrum(x, lam, dx, dy, -z)


def as_axes_swapped(x, lam, dx, dy, z):
    return optics.angular_spectrum(x, lam, dy, dx, z)


def as_no_inverse_norm(x, lam, dx, dy, z):
    ny, nx = np.shape(x)[-2:]
    return optics.angular_spectrum(x, lam, dx, dy, z) * (nx * ny)


def as_paraxial_h(x, lam, dx, dy, z):
    ny, nx = np.shape(x)[-2:]
    fx = np.fft.fftfreq(nx, dx)
    fy = np.fft.fftfreq(ny, dy)
    h = np.exp(2j * np.pi * z / lam) * np.exp(-1j * np.pi * lam * z * (fx[None] ** 2 + fy[:, None] ** 2))
    return np.fft.ifft2(np.fft.fft2(x) * h)


@pytest.mark.parametrize("mutant", [as_z_sign, as_axes_swapped, as_no_inverse_norm, as_paraxial_h])
def test_as_mutants_rejected(mutant):
    assert pins.plane_wave_error(mutant) > 1e-6


# ---------------------------------------------------------------- Fresnel mutants

def fr_conj_out(x, lam, dx, dy, z):
    _, q_out = optics.fresnel_chirps(*np.shape(x)[-2:], lam, dx, dy, z)
    return optics.fresnel(x, lam, dx, dy, z) * np.conj(q_out) ** 2


def fr_no_sign_flip(x, lam, dx, dy, z):
    if z > 0:
        return optics.fresnel(x, lam, dx, dy, z)
    # compute with the forward kernel but the negative-z chirps
    ny, nx = np.shape(x)[-2:]
    q_in, q_out = optics.fresnel_chirps(ny, nx, lam, dx, dy, z)
    fx = optics._centered_dft_matrix(nx, 1)
    fy = optics._centered_dft_matrix(ny, 1)
    return q_out * (fy @ (x * q_in) @ fx.T) / math.sqrt(nx * ny)


def fr_wrong_out_pitch(x, lam, dx, dy, z):
    ny, nx = np.shape(x)[-2:]
    m = np.arange(nx) - nx // 2
    n = np.arange(ny) - ny // 2
    q_in, _ = optics.fresnel_chirps(ny, nx, lam, dx, dy, z)
    q_out = np.exp(1j * np.pi * ((m * dx)[None] ** 2 + (n * dy)[:, None] ** 2) / (lam * z))
    s = 1 if z > 0 else -1
    fx = optics._centered_dft_matrix(nx, s)
    fy = optics._centered_dft_matrix(ny, s)
    return q_out * (fy @ (x * q_in) @ fx.T) / math.sqrt(nx * ny)


def fr_uncentred(x, lam, dx, dy, z):
    ny, nx = np.shape(x)[-2:]
    q_in, q_out = optics.fresnel_chirps(ny, nx, lam, dx, dy, z)
    return q_out * np.fft.fft2(x * q_in) / math.sqrt(nx * ny)


@pytest.mark.parametrize("mutant", [fr_conj_out, fr_no_sign_flip, fr_wrong_out_pitch, fr_uncentred])
def test_fresnel_mutants_rejected(mutant):
    errs = [pins.point_source_fresnel_error(mutant, z) for z in (0.5, -0.5)]
    assert max(errs) > 1e-6


# ---------------------------------------------------------------- temporal mutants

def stft_plus_sign(u, w, s):
    return np.conj(temporal.stft(np.conj(u), w, s))


def stft_reversed_time(u, w, s):
    return temporal.stft(u[::-1], w, s)


def moments_amplitude(s, bins, freqs, orders=(0, 1, 2)):
    a = np.abs(np.asarray(s)[:, bins])
    return [np.tensordot(np.asarray(freqs) ** n, a, axes=(0, 1)) for n in orders]


def moments_order_shift(s, bins, freqs, orders=(0, 1, 2)):
    return temporal.moments(s, bins, freqs, tuple(n + 1 for n in orders))


@pytest.mark.parametrize("stft_fn,mom_fn", [
    (stft_plus_sign, temporal.moments),
    (stft_reversed_time, temporal.moments),
    (temporal.stft, moments_amplitude),
    (temporal.stft, moments_order_shift),
])
def test_temporal_mutants_rejected(stft_fn, mom_fn):
    assert pins.pure_tone_errors(stft_fn, mom_fn) > 1e-6


def test_band_rounding_mutant_rejected():
    # rounding instead of ceil/floor moves the 256^2 band's first bin
    w, fs, lo, hi = 32, 71400.0, 3000.0, 35000.0
    assert round(lo * w / fs) != temporal.band_bins(w, fs, lo, hi)[0][0]


# ---------------------------------------------------------------- PCA mutants

def pca_conj_cov(u, c1, c2):
    r = pca.pca_window(np.conj(u), c1, c2)
    return r


def pca_ascending(u, c1, c2):
    r = pca.pca_window(u, c1, c2)
    w = u.shape[0]
    lo, hi = w - 1 - c2, w - 1 - c1
    x = pca.window_matrix(u)
    lam, v = np.linalg.eigh(pca.covariance(x))
    m0 = np.sum(np.abs((x @ v)[:, lo:hi + 1]) ** 2, axis=1).reshape(u.shape[1:])
    return {"cov": r["cov"], "eigvals": lam, "eigvecs": v, "m0": m0}


def pca_range_exclusive(u, c1, c2):
    r = pca.pca_window(u, c1, c2)
    x = pca.window_matrix(u)
    y = x @ r["eigvecs"]
    r["m0"] = np.sum(np.abs(y[:, c1:c2]) ** 2, axis=1).reshape(u.shape[1:])
    return r


@pytest.mark.parametrize("mutant", [pca_conj_cov, pca_ascending, pca_range_exclusive])
def test_pca_mutants_rejected(mutant):
    assert pins.pca_construction_error(mutant) > 1e-6


# ---------------------------------------------------------------- high-pass and volume mutants

def hp_lowpass(x, lam, dx, dy, z, radius):
    """keeps the inside of the circle instead of the outside"""
    full = optics.angular_spectrum(x, lam, dx, dy, z)
    return full - optics.angular_spectrum(x, lam, dx, dy, z, radius)


def hp_radius_in_index_units(x, lam, dx, dy, z, radius):
    """radius compared with the index k instead of k / n"""
    ny, nx = np.shape(x)[-2:]
    return optics.angular_spectrum(x, lam, dx, dy, z, radius * nx)


@pytest.mark.parametrize("mutant", [hp_lowpass, hp_radius_in_index_units])
def test_highpass_mutants_rejected(mutant):
    assert pins.highpass_plane_wave_error(mutant) > 1e-6


def vol_magnitude(u, w, s):
    from oracle import pipeline
    return np.sqrt(pipeline.stft_volume(u, None, w, s))


def vol_reversed_bins(u, w, s):
    from oracle import pipeline
    return pipeline.stft_volume(u, None, w, s)[:, ::-1]


@pytest.mark.parametrize("mutant", [vol_magnitude, vol_reversed_bins])
def test_volume_mutants_rejected(mutant):
    e_tone, e_pars = pins.volume_errors(mutant)
    assert max(e_tone, e_pars) > 1e-6


# ---------------------------------------------------------------- magnitude / argument image mutants

def img_modulus_of_sum(s):
    return np.abs(np.asarray(s).sum(axis=1))


def img_power_sum(s):
    return (np.abs(np.asarray(s)) ** 2).sum(axis=1)


def img_sum_of_angles(s):
    return np.angle(np.asarray(s)).sum(axis=1)


def img_conjugated_argument(s):
    return -post.argument_image(s)


@pytest.mark.parametrize("mag_fn, arg_fn", [
    (img_modulus_of_sum, post.argument_image),
    (img_power_sum, post.argument_image),
    (post.magnitude_image, img_sum_of_angles),
    (post.magnitude_image, img_conjugated_argument),
])
def test_image_mutants_rejected(mag_fn, arg_fn):
    em, ea = pins.tone_image_errors(mag_fn, arg_fn)
    assert max(em, ea) > 1e-6


# ---------------------------------------------------------------- post-processing helper mutants

def disk_max_side(ny, nx, mask_radius):
    """radius scaled by the longer side instead of the shorter"""
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = mask_radius * max(nx, ny) / 2.0
    return (((yy - ny / 2.0) ** 2 + (xx - nx / 2.0) ** 2) <= r * r).astype(np.float64)


def disk_half_pixel_centre(ny, nx, mask_radius):
    """centre at ((ny - 1) / 2, (nx - 1) / 2) instead of the centre pixel"""
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = mask_radius * min(nx, ny) / 2.0
    return (((yy - (ny - 1) / 2.0) ** 2 + (xx - (nx - 1) / 2.0) ** 2) <= r * r).astype(np.float64)


def disk_open_boundary(ny, nx, mask_radius):
    """boundary excluded"""
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = mask_radius * min(nx, ny) / 2.0
    return (((yy - ny / 2.0) ** 2 + (xx - nx / 2.0) ** 2) < r * r).astype(np.float64)


@pytest.mark.parametrize("mutant", [disk_max_side, disk_half_pixel_centre, disk_open_boundary])
def test_disk_mask_mutants_rejected(mutant):
    assert pins.disk_mask_errors(mutant) > 0


def gauss_sigma_squared(sigma):
    """exp(-r^2 / sigma^2): the width of a Gaussian of std sigma / sqrt(2)"""
    r = int(np.ceil(3 * sigma))
    i = np.arange(-r, r + 1)
    g = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (sigma * sigma))
    return g / g.sum()


def gauss_unnormalised(sigma):
    r = int(np.ceil(3 * sigma))
    i = np.arange(-r, r + 1)
    return np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2.0 * sigma * sigma))


def gauss_two_sigma_support(sigma):
    """truncated at 2 sigma"""
    r = int(np.ceil(2 * sigma))
    i = np.arange(-r, r + 1)
    g = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


@pytest.mark.parametrize("mutant", [gauss_sigma_squared, gauss_unnormalised, gauss_two_sigma_support])
def test_gaussian_kernel_mutants_rejected(mutant):
    assert pins.gaussian_kernel_errors(mutant) > 1e-6


def conv_as_correlation(images, kernel):
    from scipy.signal import correlate2d
    return np.stack([correlate2d(im, kernel, mode="same", boundary="fill") for im in np.asarray(images)])


def conv_periodic(images, kernel):
    from scipy.signal import convolve2d
    return np.stack([convolve2d(im, kernel, mode="same", boundary="wrap") for im in np.asarray(images)])


@pytest.mark.parametrize("mutant", [conv_as_correlation, conv_periodic])
def test_convolution_mutants_rejected(mutant):
    assert pins.convolution_shift_error(mutant) > 1e-6


# ---------------------------------------------------------------- SSA + FFT mutants

def _ssa_variant(u, c1, c2, how):
    from oracle import pca as opca
    w = u.shape[0]
    x = opca.window_matrix(u)
    lam, v = opca.eig_descending(opca.covariance(x))
    if how == "ascending":
        v = v[:, ::-1]
    vs = v[:, c1:c2] if how == "exclusive" else v[:, c1:c2 + 1]
    if how == "no_conj":
        xf = x @ vs @ vs.T
    elif how == "spectrum_filtered":
        s = temporal.stft(u, w, w)[0]
        sm = opca.window_matrix(s)
        return (sm @ vs @ vs.conj().T).T.reshape(u.shape)
    elif how == "conj_cov":
        lam2, v2 = opca.eig_descending(opca.covariance(x).conj())
        vs = v2[:, c1:c2 + 1]
        xf = x @ vs @ vs.conj().T
    else:
        xf = x @ vs @ vs.conj().T
    return temporal.stft(xf.T.reshape(u.shape), w, w)[0]


@pytest.mark.parametrize("how", ["ascending", "exclusive", "no_conj", "spectrum_filtered", "conj_cov"])
def test_ssa_mutants_rejected(how):
    assert pins.ssa_tone_errors(lambda u, c1, c2: _ssa_variant(u, c1, c2, how)) > 1e-6
