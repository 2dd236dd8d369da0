"""The post-processing oracle against closed forms (CPU only)."""

import numpy as np

from oracle import post


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
