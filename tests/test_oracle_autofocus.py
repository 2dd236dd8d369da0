"""The autofocus oracle against finite differences, library special cases and
closed forms (CPU only)."""

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import autofocus as af


def _tiny_params(seed=0, scale=1.0):
    th = af.init_params(seed) * scale
    rng = np.random.default_rng(seed + 1)
    # non-zero biases so every term of the backward pass is exercised
    p = af.unflatten(th)
    for i in (1, 3, 5, 7, 9, 11):
        p[i] += 0.05 * rng.standard_normal(p[i].shape)
    return af.flatten(p)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 1, 8, 8))
    z = np.array([0.3, -0.7])
    th = _tiny_params()
    loss, g = af.loss_and_grad(th, x, z)
    assert np.isfinite(loss)
    # coordinates from every parameter group
    offs = np.cumsum([0] + [int(np.prod(s)) for s in af.param_shapes()])
    coords = []
    for a, b in zip(offs[:-1], offs[1:]):
        coords += list(rng.choice(np.arange(a, b), size=min(8, b - a), replace=False))
    h = 1e-6
    for i in coords:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (af.loss_and_grad(tp, x, z)[0] - af.loss_and_grad(tm, x, z)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 3, 9, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = af.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[n, c], w[o, c], mode="same", boundary="fill") for c in range(3)) + b[o]
            assert np.allclose(y[n, o], ref, atol=1e-12)


def test_nll_closed_form():
    out = np.array([[0.5, np.log(0.25)], [-1.0, 0.0]])
    z = np.array([1.0, -1.0])
    loss, d = af.nll(out, z)
    # sample 0: r = 0.5, e = 4 -> 0.5 (log 0.25 + 1) ; sample 1: r = 0 -> 0
    assert np.isclose(loss, 0.5 * (0.5 * (np.log(0.25) + 0.25 * 4)))
    assert np.allclose(d[0], np.array([-0.5 * 4, 0.5 * (1 - 1.0)]) / 2)
    assert np.allclose(d[1], np.array([0.0, 0.5]) / 2)


def test_adam_first_step_closed_form():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    new, m, v = af.adam(th, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # bias-corrected first step moves each coordinate by lr * g / (|g| + eps)
    assert np.allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_sharpness_closed_forms():
    a = np.zeros((10, 12))
    a[:, 7:] = 1.0  # vertical step edge: G = 1 on one interior column of 11
    p = 1 / 11
    assert np.isclose(af.sharpness(a), p * (1 - p))
    ramp = np.tile(np.arange(12) * 0.5, (10, 1))  # constant gradient: no variance
    assert af.sharpness(ramp) == 0.0


def test_crop_is_standardised_and_dc_free():
    rng = np.random.default_rng(5)
    h = rng.integers(0, 256, (256, 256)).astype(np.uint8)
    c = af.spectrum_crop(h)
    assert c.shape == (64, 64)
    assert abs(c.mean()) < 1e-12 and abs(c.std() - 1) < 1e-12
    assert c[32, 32] == c.min()  # log(1 + 0) at DC, every other bin is positive


def test_scan_finds_the_recording_distance():
    """Holograms from the point-superposition generator (not the reconstruction
    method) at known z: the scan lands near z.  The +1 order is confined to
    0.1 cycles/pixel, so the depth of field lambda / NA^2 (NA = lambda *
    0.1 / pitch) is about 47 mm; the median error must stay within two grid
    steps (7 mm) and every error well inside the depth of field."""
    from synth.autofocus import af_hologram
    zc = af.candidates()
    errs = []
    for s, z in enumerate([0.09, 0.17, 0.26, 0.33, 0.41, 0.47]):
        h = af_hologram(z, 50 + s)
        zh, sc = af.scan(h, 852e-9, 20e-6, zc)
        errs.append(abs(zh - z))
    errs = np.array(errs)
    assert np.median(errs) <= 2 * 0.45 / 127 + 1e-9, errs
    assert errs.max() <= 0.035, errs


def test_param_count():
    assert af.n_params() == 30306
