"""Post-processing of the rendered images (Sec. III-B.2, Post processing and
image accumulation), float64.  Test infrastructure only (see the package
docstring).

The paper lists the steps in this order: convolution with a given kernel
(Gaussian or user-designed), re-normalisation after the convolution,
registration by cross-correlation with a reference frame (the mean of
accumulated frames within a circular mask; each image is shifted by the
offset of the correlation peak), and a moving average over an image
accumulation buffer of user-defined size.  Readings:

* convolution: 2-D linear convolution, output the size of the input, zero
  outside the image (``scipy.signal.convolve2d(mode="same")``);
* re-normalisation: each image divided by its own spatial mean;
* registration: the reference is the mean of the first ``ref_count``
  images, multiplied by a centred disk mask of radius
  ``mask_radius * min(nx, ny) / 2`` pixels; the circular cross-correlation
  c(s) = sum_p img(p + s) ref(p) of each image with it is maximised over
  integer shifts s (ties: the lowest flat index), and the image is shifted
  circularly by -s;
* accumulation: out_j = mean(in_{max(0, j - A + 1)} .. in_j).

Besides the statistical moments, the paper renders the magnitude or the
argument of the windowed spectrum over a range of temporal indices
(Sec. III-B.1) into the buffer these steps work on.  Readings (the paper
does not say how the range is combined):

* magnitude: the sum over the range of the moduli, sum_k |S_k| (a sum, as
  the moments sum their weighted powers);
* argument: the argument of the sum over the range, arg(sum_k S_k) in
  [-pi, pi] (a sum of angles would depend on where each one wraps); for a
  one-index range both are |S_k| and arg(S_k).
"""

from __future__ import annotations

import numpy as np
from scipy.signal import convolve2d


def gaussian_kernel(sigma: float) -> np.ndarray:
    """Normalised Gaussian, size 2 ceil(3 sigma) + 1."""
    r = int(np.ceil(3 * sigma))
    i = np.arange(-r, r + 1)
    g = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def convolve(images, kernel) -> np.ndarray:
    images = np.asarray(images, np.float64)
    k = np.asarray(kernel, np.float64)
    return np.stack([convolve2d(im, k, mode="same", boundary="fill") for im in images])


def renormalise(images) -> np.ndarray:
    images = np.asarray(images, np.float64)
    return images / images.mean(axis=(1, 2), keepdims=True)


def disk_mask(ny: int, nx: int, mask_radius: float) -> np.ndarray:
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = mask_radius * min(nx, ny) / 2.0
    return (((yy - ny / 2.0) ** 2 + (xx - nx / 2.0) ** 2) <= r * r).astype(np.float64)


def register(images, ref_count: int, mask_radius: float):
    """(registered images, shifts [n, 2] as (dy, dx))."""
    images = np.asarray(images, np.float64)
    n, ny, nx = images.shape
    ref = images[:ref_count].mean(axis=0) * disk_mask(ny, nx, mask_radius)
    fr = np.conj(np.fft.fft2(ref))
    out = np.empty_like(images)
    shifts = np.zeros((n, 2), np.int64)
    for j in range(n):
        c = np.fft.ifft2(np.fft.fft2(images[j]) * fr).real  # c[s] = sum_p img[p + s] ref[p]
        dy, dx = np.unravel_index(int(np.argmax(c)), c.shape)
        shifts[j] = (dy, dx)
        out[j] = np.roll(images[j], (-dy, -dx), axis=(0, 1))
    return out, shifts


def accumulate(images, length: int) -> np.ndarray:
    images = np.asarray(images, np.float64)
    out = np.empty_like(images)
    for j in range(images.shape[0]):
        out[j] = images[max(0, j - length + 1): j + 1].mean(axis=0)
    return out


def postprocess(images, kernel=None, renorm: bool = False, ref_count: int = 0, mask_radius: float = 1.0,
                accumulate_length: int = 1):
    """The chain in the paper's order; returns (images, shifts or None)."""
    x = np.asarray(images, np.float64)
    if kernel is not None:
        x = convolve(x, kernel)
    if renorm:
        x = renormalise(x)
    shifts = None
    if ref_count > 0:
        x, shifts = register(x, ref_count, mask_radius)
    if accumulate_length > 1:
        x = accumulate(x, accumulate_length)
    return x, shifts


def magnitude_image(spec) -> np.ndarray:
    """out[j, ...] = sum_k |S[j, k, ...]| over the range held in axis 1 of
    spec (the windowed spectrum restricted to the range)."""
    return np.abs(np.asarray(spec, dtype=np.complex128)).sum(axis=1)


def argument_image(spec) -> np.ndarray:
    """out[j, ...] = arg(sum_k S[j, k, ...]) over the range held in axis 1."""
    return np.angle(np.asarray(spec, dtype=np.complex128).sum(axis=1))
