"""The oracle against closed forms, brute force and invariants (CPU only)."""

import math

import numpy as np
import pytest

from oracle import optics, pca, pipeline, temporal
from tests import pins
from tests.conftest import rel_l2

LAM = pins.LAMBDA


# ------------------------------------------------------------------ angular spectrum

@pytest.mark.parametrize("z", [0.13, -0.2, 0.0])
def test_as_plane_waves_exact(z):
    assert pins.plane_wave_error(optics.angular_spectrum, z=z) < 1e-12


@pytest.mark.parametrize("z,tol", [(0.01, 3e-7), (0.05, 1.5e-6), (0.2, 1e-5)])
def test_as_gaussian_beam_paraxial(z, tol):
    # The residual is the non-paraxial term, growing with z.
    assert pins.gaussian_as_error(optics.angular_spectrum, z) < tol


def test_as_plus_minus_z_is_identity():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 24, 40)) + 1j * rng.standard_normal((3, 24, 40))
    u = optics.angular_spectrum(x, LAM, 20e-6, 12e-6, 0.31)
    back = optics.angular_spectrum(u, LAM, 20e-6, 12e-6, -0.31)
    assert rel_l2(back, x) < 1e-12


def test_as_composition():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((16, 48))
    a = optics.angular_spectrum(optics.angular_spectrum(x, LAM, 20e-6, 25e-6, 0.07), LAM, 20e-6, 25e-6, 0.11)
    b = optics.angular_spectrum(x, LAM, 20e-6, 25e-6, 0.18)
    # the phases k z reach 1.3e6 rad, so float64 rounding of the phase alone
    # is about 1.3e6 * 2.2e-16 = 3e-10 rad per term
    assert rel_l2(a, b) < 2e-9


def test_as_parseval():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((32, 32))
    u = optics.angular_spectrum(x, LAM, 20e-6, 20e-6, 0.4)
    assert abs(np.linalg.norm(u) - np.linalg.norm(x)) / np.linalg.norm(x) < 1e-12


def test_as_evanescent_components_dropped():
    # pitch below lambda/2 puts the grid's highest frequencies beyond 1/lambda
    h = optics.as_transfer_function(8, 8, LAM, 0.3e-6, 0.3e-6, 0.01)
    fx = np.fft.fftfreq(8, 0.3e-6)
    ev = (fx[None, :] ** 2 + fx[:, None] ** 2) >= LAM ** -2
    assert ev.any() and np.all(h[ev] == 0) and np.allclose(np.abs(h[~ev]), 1.0)


def test_as_brute_force_tiny():
    rng = np.random.default_rng(4)
    x = rng.integers(0, 256, (4, 8)).astype(np.float64)
    ref = pins.brute_force_as(x, LAM, 20e-6, 30e-6, 0.05)
    assert rel_l2(optics.angular_spectrum(x, LAM, 20e-6, 30e-6, 0.05), ref) < 1e-12


# ------------------------------------------------------------------ Fresnel

@pytest.mark.parametrize("z", [0.5, -0.5, 0.12])
def test_fresnel_point_source_is_spherical_wave(z):
    assert pins.point_source_fresnel_error(optics.fresnel, z) < 1e-12
    assert pins.point_source_fresnel_error(optics.fresnel, z, at=(8, 16)) < 1e-12


@pytest.mark.parametrize("z", [0.2, 0.5, -0.3])
def test_fresnel_gaussian_beam(z):
    assert pins.gaussian_fresnel_error(optics.fresnel, z) < 1e-9


def test_fresnel_brute_force_tiny():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 4096, (4, 8)).astype(np.float64)
    for z in (0.5, -0.5):
        ref = pins.brute_force_fresnel(x, LAM, 20e-6, 30e-6, z)
        assert rel_l2(optics.fresnel(x, LAM, 20e-6, 30e-6, z), ref) < 1e-12


def test_fresnel_unitary_and_round_trip():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((16, 32)) + 1j * rng.standard_normal((16, 32))
    dx, dy, z = 20e-6, 15e-6, 0.5
    u = optics.fresnel(x, LAM, dx, dy, z)
    assert abs(np.linalg.norm(u) - np.linalg.norm(x)) / np.linalg.norm(x) < 1e-12
    # back-transform on the output grid (pitch lambda|z|/(N d)) returns x
    px = optics.fresnel_output_pitch(32, dx, LAM, z)
    py = optics.fresnel_output_pitch(16, dy, LAM, z)
    back = optics.fresnel(u, LAM, px, py, -z)
    assert rel_l2(back, x) < 1e-12


def test_checkerboard_centred_dft_identity():
    # fftshift(fft2(ifftshift(a))) == (-1)^(m+n) fft2((-1)^(m+n) a) for N/2 even
    rng = np.random.default_rng(8)
    a = rng.standard_normal((256, 128)) + 1j * rng.standard_normal((256, 128))
    sgn = (-1.0) ** np.add.outer(np.arange(256), np.arange(128))
    lhs = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(a)))
    rhs = sgn * np.fft.fft2(sgn * a)
    assert np.max(np.abs(lhs - rhs)) == 0.0


# ------------------------------------------------------------------ temporal

def test_pure_tone_single_bin():
    assert pins.pure_tone_errors(temporal.stft, temporal.moments) < 1e-12


def test_stft_brute_force_tiny():
    rng = np.random.default_rng(9)
    u = rng.standard_normal((8, 3, 2)) + 1j * rng.standard_normal((8, 3, 2))
    for w, s in ((4, 4), (4, 2), (3, 1)):
        assert rel_l2(temporal.stft(u, w, s), pins.brute_force_stft(u, w, s)) < 1e-12


def test_window_count_rule():
    assert temporal.n_windows(64, 32, 32) == 2
    assert temporal.n_windows(65535, 32, 32) == 2047
    assert temporal.n_windows(31, 32, 32) == 0
    assert temporal.n_windows(40, 32, 4) == 3


def _golden_band_rows():
    rows = []
    path = __file__.replace("test_oracle_pins.py", "golden/band_bins.txt")
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            w, fs, lo, hi, sym, k1, k2, spacing = line.split()
            rows.append((int(w), float(fs), float(lo), float(hi), int(sym), int(k1), int(k2), float(spacing)))
    return rows


@pytest.mark.parametrize("row", _golden_band_rows())
def test_band_bins_golden(row):
    w, fs, lo, hi, sym, k1, k2, spacing = row
    bins, freqs = temporal.band_bins(w, fs, lo, hi, bool(sym))
    pos = [b for b in bins if b <= w // 2]
    assert pos == list(range(k1, k2 + 1))
    assert np.allclose(np.diff(freqs[:len(pos)]), spacing, rtol=0, atol=1e-9)
    if sym:
        assert sorted(bins[len(pos):]) == sorted(w - k for k in pos if 0 < k and 2 * k != w)


def test_commutation_spatial_temporal():
    rng = np.random.default_rng(10)
    frames = rng.integers(0, 256, (16, 16, 32)).astype(np.uint8)
    opt = pipeline.Optics(LAM, 20e-6, 20e-6, -0.2)
    a = temporal.stft(pipeline.reconstruct(frames, opt), 8, 8)
    b = optics.angular_spectrum(temporal.stft(frames.astype(np.float64), 8, 8), LAM, 20e-6, 20e-6, -0.2)
    assert rel_l2(a, b) < 1e-12


def test_moment_inequalities_on_generated_data():
    from synth import holograms
    x, spec = holograms.config_c1()
    res = pipeline.stft_moments(x, pipeline.Optics(LAM, spec.pitch, spec.pitch, -spec.z), 32, 32,
                                spec.fs, 2e3, 8e3)
    m0, m1, m2 = res["m0"], res["m1"], res["m2"]
    f = res["freqs"]
    assert np.all(m0 > 0)
    mean_f = m1 / m0
    assert np.all(mean_f >= f.min() * (1 - 1e-12)) and np.all(mean_f <= f.max() * (1 + 1e-12))
    assert np.all(m2 * m0 >= m1 ** 2 * (1 - 1e-12))


# ------------------------------------------------------------------ PCA

def test_pca_constructed_spectrum():
    assert pins.pca_construction_error(pca.pca_window) < 1e-12


def test_pca_rank_one():
    assert pins.pca_rank1_error(pca.pca_window) < 1e-12


def test_pca_trace_and_residual():
    rng = np.random.default_rng(12)
    u = rng.standard_normal((16, 8, 12)) + 1j * rng.standard_normal((16, 8, 12))
    r = pca.pca_window(u)
    x = pca.window_matrix(u)
    fro2 = np.linalg.norm(x) ** 2
    assert abs(r["eigvals"].sum() - fro2) / fro2 < 1e-12
    assert abs(np.trace(r["cov"]).real - fro2) / fro2 < 1e-12
    v, lam = r["eigvecs"], r["eigvals"]
    assert np.linalg.norm(r["cov"] @ v - v * lam[None, :]) / fro2 < 1e-12
    assert np.all(np.diff(lam) <= 0)


def test_pca_covariance_invariant_under_propagation():
    rng = np.random.default_rng(13)
    frames = rng.integers(0, 256, (8, 32, 32)).astype(np.uint8)
    raw = pca.covariance(pca.window_matrix(frames.astype(np.float64)))
    prop = pca.covariance(pca.window_matrix(pipeline.reconstruct(frames, pipeline.Optics(LAM, 20e-6, 20e-6, 0.3))))
    assert rel_l2(prop, raw) < 1e-12


def test_pca_full_range_is_pixel_energy():
    rng = np.random.default_rng(14)
    u = rng.standard_normal((6, 4, 5)) + 1j * rng.standard_normal((6, 4, 5))
    r = pca.pca_window(u, 0, 5)
    assert rel_l2(r["m0"], np.sum(np.abs(u) ** 2, axis=0)) < 1e-12


def test_unpack_exact_and_typed():
    raw = np.array([[0, 255], [4095, 65535]], np.uint16)
    assert np.array_equal(optics.unpack(raw), np.array([[0.0, 255.0], [4095.0, 65535.0]]))
    with pytest.raises(TypeError):
        optics.unpack(np.zeros((2, 2), np.int32))


def test_empty_and_short_stacks():
    x = np.zeros((10, 8, 8), np.uint8)
    res = pipeline.stft_moments(x, None, 16, 16, 1e3, 0, 500)
    assert res["m0"].shape == (0, 8, 8)
    res = pipeline.pca_render(x, None, 16, 16)
    assert res["m0"].shape == (0, 8, 8)
    assert math.isclose(temporal.band_bins(16, 1e3, 0, 500)[1][-1], 500.0)


def test_highpass_plane_waves():
    assert pins.highpass_plane_wave_error(optics.angular_spectrum) < 1e-12


def test_highpass_zero_radius_is_plain_as():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 16, 24))
    a = optics.angular_spectrum(x, pins.LAMBDA, 20e-6, 20e-6, 0.1)
    b = optics.angular_spectrum(x, pins.LAMBDA, 20e-6, 20e-6, 0.1, 0.0)
    assert np.array_equal(a, b)


def test_volume_tone_and_parseval():
    from oracle import pipeline
    e_tone, e_pars = pins.volume_errors(lambda u, w, s: pipeline.stft_volume(u, None, w, s))
    assert e_tone < 1e-12 and e_pars < 1e-12
