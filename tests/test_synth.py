"""The seeded input generator (CPU only)."""

import dataclasses

import numpy as np

from synth import holograms


def test_deterministic_by_seed():
    spec = holograms.HoloSpec(frames=4, ny=32, nx=64, seed=5)
    a = holograms.hologram_stack(spec)
    b = holograms.hologram_stack(spec)
    c = holograms.hologram_stack(dataclasses.replace(spec, seed=6))
    assert a.dtype == np.uint8 and a.shape == (4, 32, 64)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_c1_statistics():
    x, spec = holograms.config_c1()
    assert x.shape == (64, 128, 128) and x.dtype == np.uint8
    assert abs(x.mean() - 64) < 1.0
    assert (x == 255).mean() < 1e-4


def test_twelve_bit_range():
    spec = holograms.HoloSpec(frames=2, ny=64, nx=64, bits=12, seed=2, z=0.5)
    x = holograms.hologram_stack(spec)
    assert x.dtype == np.uint16 and x.max() <= 4095
    assert abs(x.mean() - 1024) < 16


def test_carrier_quarter_cycle():
    # the tilted reference puts the cross terms at +-1/4 cycle per pixel
    spec = holograms.HoloSpec(frames=1, ny=64, nx=64, seed=3)
    x = holograms.hologram_stack(spec)[0].astype(np.float64)
    p = np.abs(np.fft.fft2(x - x.mean())) ** 2
    quarter = p[16, 16] + p[48, 48] + p[15:18, 15:18].sum() + p[47:50, 47:50].sum()
    assert quarter > 0
    # spectral energy is not concentrated at DC after removing the mean
    assert p[0, 0] < 1e-6 * p.sum()


def test_drawn_z_in_range_and_fixed():
    zs = [holograms.drawn_z(s) for s in range(20)]
    assert all(0.1 <= z <= 0.4 for z in zs)
    assert holograms.drawn_z(1) == holograms.drawn_z(1)


def test_temporal_spectrum_inside_doppler_band():
    # per-pixel temporal spectrum of the frames: energy away from DC sits
    # within +-f_max (the Doppler band) plus the Poisson floor
    spec = holograms.HoloSpec(frames=64, ny=32, nx=32, seed=4, fs=33e3, f_max=8e3, z=0.05)
    x = holograms.hologram_stack(spec).astype(np.float64)
    s = np.abs(np.fft.fft(x - x.mean(axis=0), axis=0)) ** 2
    f = np.abs(np.fft.fftfreq(64, 1 / 33e3))
    inband = s[(f > 0) & (f <= 8.5e3)].sum()
    outband = s[f > 9.5e3].sum()
    assert inband > 3 * outband
