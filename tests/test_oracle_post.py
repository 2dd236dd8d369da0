"""The post-processing oracle against closed forms (CPU only)."""

import numpy as np

from oracle import post, temporal
from tests import pins


def test_delta_kernel_is_identity_and_box_on_constant():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 9, 11))
    d = np.zeros((5, 5))
    d[2, 2] = 1.0
    assert np.allclose(post.convolve(x, d), x, atol=1e-15)
    c = np.full((1, 9, 11), 2.0)
    y = post.convolve(c, np.full((3, 3), 1.0 / 9))
    assert np.allclose(y[0, 1:-1, 1:-1], 2.0)          # interior: the mean of a constant
    assert np.isclose(y[0, 0, 0], 2.0 * 4 / 9)         # corner: 4 of 9 taps inside
    assert np.isclose(y[0, 0, 5], 2.0 * 6 / 9)         # edge: 6 of 9 taps inside


def test_gaussian_kernel_normalised_and_symmetric():
    g = post.gaussian_kernel(1.5)
    assert g.shape == (11, 11) and np.isclose(g.sum(), 1.0)
    assert np.allclose(g, g.T) and np.allclose(g, g[::-1, ::-1])


def test_renormalised_mean_is_one():
    x = np.random.default_rng(2).uniform(1, 3, (3, 8, 8))
    assert np.allclose(post.renormalise(x).mean(axis=(1, 2)), 1.0)


def test_registration_undoes_circular_shifts():
    rng = np.random.default_rng(3)
    base = rng.uniform(0, 1, (32, 48))
    moves = [(0, 0), (3, -5), (-7, 11), (15, 2)]
    stack = np.stack([np.roll(base, m, axis=(0, 1)) for m in moves])
    out, shifts = post.register(stack, ref_count=1, mask_radius=2.0)  # mask covers the image
    for j, (my, mx) in enumerate(moves):
        assert tuple(shifts[j]) == (my % 32, mx % 48)
        assert np.allclose(out[j], base)


def test_moving_average_of_a_ramp():
    x = np.arange(6, dtype=np.float64)[:, None, None] * np.ones((1, 2, 3))
    y = post.accumulate(x, 3)
    assert np.allclose(y[:, 0, 0], [0, 0.5, 1, 2, 3, 4])


def _tones(window, amps, bins, shape=(3, 4)):
    """Frames x_t = sum_i a_i exp(2i pi k_i t / W) at every pixel (a_i may vary
    over the pixels): the oracle's DFT gives S_{k_i} = W a_i, zero elsewhere."""
    t = np.arange(window)[:, None, None]
    x = np.zeros((window,) + shape, dtype=np.complex128)
    for a, k in zip(amps, bins):
        x += a[None] * np.exp(2j * np.pi * k * t / window)
    return x


def test_magnitude_and_argument_of_tones():
    rng = np.random.default_rng(4)
    w = 16
    a1 = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    a2 = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    s = temporal.stft(_tones(w, [a1, a2], [3, 5]), w, w)
    # one-index range: the modulus and the phase of that bin's amplitude
    assert np.allclose(post.magnitude_image(s[:, [3]])[0], w * np.abs(a1))
    assert np.allclose(post.argument_image(s[:, [3]])[0], np.angle(a1))
    # a range over both tones and an empty bin: sum of moduli, phase of the sum
    assert np.allclose(post.magnitude_image(s[:, [3, 4, 5]])[0], w * (np.abs(a1) + np.abs(a2)))
    assert np.allclose(post.argument_image(s[:, [3, 4, 5]])[0], np.angle(a1 + a2))


def test_argument_rotates_with_a_global_phase():
    rng = np.random.default_rng(5)
    s = rng.standard_normal((2, 5, 6, 7)) + 1j * rng.standard_normal((2, 5, 6, 7))
    phi = 2.2
    a0, a1 = post.argument_image(s), post.argument_image(s * np.exp(1j * phi))
    d = np.angle(np.exp(1j * (a1 - a0 - phi)))  # difference wrapped to [-pi, pi]
    assert np.max(np.abs(d)) < 1e-12
    assert np.allclose(post.magnitude_image(s * np.exp(1j * phi)), post.magnitude_image(s))
    assert np.all(np.abs(a0) <= np.pi)


def test_tone_image_pin():
    em, ea = pins.tone_image_errors(post.magnitude_image, post.argument_image)
    assert em < 1e-12 and ea < 1e-12


def test_disk_mask_pin():
    assert pins.disk_mask_errors(post.disk_mask) == 0


def test_gaussian_kernel_pin():
    assert pins.gaussian_kernel_errors(post.gaussian_kernel) < 1e-12


def test_convolution_orientation_pin():
    assert pins.convolution_shift_error(post.convolve) < 1e-15


def test_registration_with_a_disk_inside_the_image():
    """A bright off-centre blob inside the mask, moved circularly: the shift
    is recovered with a mask of half the image (the blob stays inside it)."""
    ny, nx = 40, 56
    yy, xx = np.mgrid[0:ny, 0:nx]
    base = np.exp(-((yy - 17.0) ** 2 + (xx - 31.0) ** 2) / 8.0) + 0.01
    moves = [(0, 0), (2, -3), (-4, 5)]
    stack = np.stack([np.roll(base, m, axis=(0, 1)) for m in moves])
    out, shifts = post.register(stack, ref_count=1, mask_radius=0.5)
    for j, (my, mx) in enumerate(moves):
        assert tuple(shifts[j]) == (my % ny, mx % nx)
        assert np.allclose(out[j], base)
