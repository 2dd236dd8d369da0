"""The SSA + FFT oracle against closed forms (CPU only)."""

import numpy as np
import pytest

from oracle import pca, pipeline, ssa, temporal
from tests import pins


def _spectrum(u, c1, c2):
    return ssa.ssa_stft_window(u, c1, c2)[0]


def test_ssa_tone_pin():
    assert pins.ssa_tone_errors(_spectrum) < 1e-12


def test_ssa_energy_equals_pca_projection_energy():
    """Parseval in time: sum_k |S_k|^2 = W sum_t |X_f[:, t]|^2, and the
    filtered window's energy per pixel is the projection energy of the same
    components, sum_{c in S} |(X V)[:, c]|^2."""
    rng = np.random.default_rng(3)
    w = 16
    u = rng.standard_normal((w, 6, 7)) + 1j * rng.standard_normal((w, 6, 7)) + 4.0
    s, _ = ssa.ssa_stft_window(u, 2, 12)
    m0_pca = pca.pca_window(u, 2, 12)["m0"]
    assert np.allclose((np.abs(s) ** 2).sum(axis=0), w * m0_pca, rtol=1e-12, atol=0)


def test_ssa_filter_is_a_projector():
    rng = np.random.default_rng(4)
    w = 8
    u = rng.standard_normal((w, 5, 3)) + 1j * rng.standard_normal((w, 5, 3))
    f1, lam = ssa.ssa_filter(u, 1, 5)
    f2, _ = ssa.ssa_filter(f1, 0, 4)  # the filtered window has exactly components 1..5 (now 0..4)
    assert np.allclose(f1, f2, atol=1e-12)
    assert np.all(np.diff(lam) <= 0)


def test_ssa_moments_shapes_and_band():
    rng = np.random.default_rng(5)
    u = rng.standard_normal((40, 4, 4)) + 0j
    r = ssa.ssa_moments(u, 16, 8, 16e3, 2e3, 7e3)
    assert r["m0"].shape == (4, 4, 4) and r["eigvals"].shape == (4, 16)
    bins, _ = temporal.band_bins(16, 16e3, 2e3, 7e3)
    assert list(r["bins"]) == list(bins)
    frames = rng.integers(0, 256, (33, 8, 8)).astype(np.uint8)
    rr = pipeline.ssa_render(frames, None, 16, 16, 16e3, 2e3, 7e3)
    assert rr["m0"].shape == (2, 8, 8)
    with pytest.raises(ValueError):
        ssa.ssa_filter(u[:16], 3, 2)
