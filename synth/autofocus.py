"""Seeded single holograms for autofocus tests (CPU).

Object: complex speckle band-limited to a circular pupil of radius 0.09
cycles/pixel (a low-pass filter applied to white noise) times a mask of 3-8
soft-edged disks (centres at least 32 pixels from the border, radii 8-48
pixels, edge width 1.5 pixels).  The sensor
wave is built with the same paraxial point-source superposition as
``synth.holograms`` (no reconstruction arithmetic), then a reference tilted
by a quarter cycle per pixel (amplitude 3 x rms), intensity scaled to a mean
of 64 DN, Poisson counts, uint8.
"""

from __future__ import annotations

import numpy as np
from .holograms import point_response_1d


PUPIL_CPP = 0.09


def af_object(n: int, rng) -> np.ndarray:
    noise = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    f = np.fft.fftfreq(n)
    pupil = (f[None, :] ** 2 + f[:, None] ** 2) <= PUPIL_CPP ** 2
    sp = np.fft.ifft2(np.fft.fft2(noise) * pupil)
    yy, xx = np.mgrid[0:n, 0:n]
    mask = np.zeros((n, n))
    for _ in range(int(rng.integers(3, 9))):
        cy, cx = rng.uniform(32, n - 32, 2)
        r = rng.uniform(8, 48)
        d = np.hypot(yy - cy, xx - cx)
        mask = np.maximum(mask, 1.0 / (1.0 + np.exp((d - r) / 1.5)))
    return sp * mask


def af_hologram(z: float, seed: int, n: int = 256, pitch: float = 20e-6, wavelength: float = 852e-9,
                ref_ratio: float = 3.0, mean_dn: float = 64.0) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4242]))
    o = af_object(n, rng)
    k = point_response_1d(n, pitch, wavelength, z).astype(np.complex128)
    w = k @ o @ k.T
    w /= np.sqrt(np.mean(np.abs(w) ** 2))
    yy, xx = np.mgrid[0:n, 0:n]
    ref = ref_ratio * (np.cos(np.pi * (xx + yy) / 2) + 1j * np.sin(np.pi * (xx + yy) / 2))
    f = ref + w
    inten = f.real ** 2 + f.imag ** 2
    lam = inten * (mean_dn / inten.mean())
    return np.clip(rng.poisson(lam), 0, 255).astype(np.uint8)
