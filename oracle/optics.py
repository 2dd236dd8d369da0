"""Spatial demodulation in float64: unpack, angular spectrum, Fresnel.

Test infrastructure only (see the package docstring).

Conventions (readings of the paper, which names the transforms but prints no
formula; see Abstract, Sec. II-B.3 and Sec. III-B.1):

* Coordinates: arrays are ``[..., ny, nx]``; x runs along the last axis with
  pitch ``dx``, y along the second-to-last with pitch ``dy``.
* DFT: forward ``sum_m a[m] exp(-2i pi k m / N)`` (unnormalised), inverse with
  ``1/N``.  Spatial frequencies are ``numpy.fft.fftfreq(N, d=pitch)``.
* ``z`` is the signed propagation distance: ``angular_spectrum(x, z)``
  propagates the field *by* ``z``; reconstructing a hologram recorded at
  distance ``z`` uses ``-z``.
"""

from __future__ import annotations

import numpy as np


def unpack(raw) -> np.ndarray:
    """Camera integers to float64, exactly (Sec. III-B.1: input data is
    converted to a complex representation before the spatial FFT).

    uint8 and uint16 values are taken as they are; 12-bit data is low-bit
    aligned in uint16 with no shift."""
    raw = np.asarray(raw)
    if raw.dtype not in (np.uint8, np.uint16):
        raise TypeError(f"unpack expects uint8 or uint16 camera data, got {raw.dtype}")
    return raw.astype(np.float64)


def as_transfer_function(ny: int, nx: int, wavelength: float, dx: float, dy: float,
                         z: float) -> np.ndarray:
    """Angular-spectrum transfer function H_z[q, p] (complex128, [ny, nx]).

    H_z = exp(2i pi z sqrt(1/lambda^2 - fx[p]^2 - fy[q]^2)) for propagating
    components; evanescent components (negative radicand) are set to zero.
    fx = fftfreq(nx, dx), fy = fftfreq(ny, dy)."""
    fx = np.fft.fftfreq(nx, d=dx)
    fy = np.fft.fftfreq(ny, d=dy)
    radicand = wavelength ** -2 - fx[None, :] ** 2 - fy[:, None] ** 2
    h = np.zeros((ny, nx), dtype=np.complex128)
    live = radicand > 0
    h[live] = np.exp(2j * np.pi * z * np.sqrt(radicand[live]))
    return h


def highpass_mask(ny: int, nx: int, radius: float) -> np.ndarray:
    """The spatial high-pass filter of the paper's angular-spectrum benchmark
    (Sec. VI-B.1 names it, without a formula).  Reading: an ideal circular
    mask on the DFT grid that keeps every bin whose frequency, in cycles per
    pixel, lies at or beyond ``radius`` from the origin:
    (k_x / nx)^2 + (k_y / ny)^2 >= radius^2 with signed indices k (fftfreq).
    ``radius = 0`` keeps everything.  Returns a float64 [ny, nx] of 0 and 1."""
    ux = np.fft.fftfreq(nx)
    uy = np.fft.fftfreq(ny)
    return ((ux[None, :] ** 2 + uy[:, None] ** 2) >= radius ** 2).astype(np.float64)


def angular_spectrum(x, wavelength: float, dx: float, dy: float, z: float,
                     highpass: float = 0.0) -> np.ndarray:
    """Propagate each frame of ``x`` ([..., ny, nx], real or complex) by ``z``.

    U = IDFT2( DFT2(x) * H_z ), the angular-spectrum method named in the
    Abstract and Sec. II-B.3.  With the 1/(nx ny) on the inverse only, the
    operator is unitary when no component is evanescent.  ``highpass > 0``
    multiplies the spectrum by ``highpass_mask`` as well."""
    x = np.asarray(x)
    ny, nx = x.shape[-2:]
    h = as_transfer_function(ny, nx, wavelength, dx, dy, z)
    if highpass > 0:
        h = h * highpass_mask(ny, nx, highpass)
    spectrum = np.fft.fft2(x.astype(np.complex128), axes=(-2, -1))
    return np.fft.ifft2(spectrum * h, axes=(-2, -1))


def fresnel_output_pitch(n: int, pitch: float, wavelength: float, z: float) -> float:
    """Output-plane sample spacing of the single-FFT Fresnel transform:
    lambda |z| / (n * pitch)."""
    return wavelength * abs(z) / (n * pitch)


def _centered_dft_matrix(n: int, sign: int) -> np.ndarray:
    """F[p, m] = exp(-i sign 2 pi (p - n/2)(m - n/2) / n) with the integer
    product reduced modulo n before the exponential (exact phase)."""
    idx = np.arange(n, dtype=np.int64) - n // 2
    prod = np.mod(np.outer(idx, idx), n)
    return np.exp(-1j * sign * 2.0 * np.pi * prod / n)


def fresnel_chirps(ny: int, nx: int, wavelength: float, dx: float, dy: float, z: float):
    """The input and output quadratic phases of the single-FFT Fresnel
    transform, each [ny, nx] complex128:

    Q_in[n, m]  = exp(i pi (xi_m^2 + eta_n^2) / (lambda z)),
        xi_m = (m - nx/2) dx,  eta_n = (n - ny/2) dy;
    Q_out[q, p] = exp(i pi (x_p^2 + y_q^2) / (lambda z)),
        x_p = (p - nx/2) lambda|z|/(nx dx),  y_q likewise."""
    m = np.arange(nx) - nx // 2
    n = np.arange(ny) - ny // 2
    xi = m * dx
    eta = n * dy
    ox = m * fresnel_output_pitch(nx, dx, wavelength, z)
    oy = n * fresnel_output_pitch(ny, dy, wavelength, z)
    q_in = np.exp(1j * np.pi * (xi[None, :] ** 2 + eta[:, None] ** 2) / (wavelength * z))
    q_out = np.exp(1j * np.pi * (ox[None, :] ** 2 + oy[:, None] ** 2) / (wavelength * z))
    return q_in, q_out


def fresnel(x, wavelength: float, dx: float, dy: float, z: float) -> np.ndarray:
    """Single-FFT Fresnel transform of each frame of ``x`` ([..., ny, nx]).

    U[q, p] = Q_out[q, p] (nx ny)^(-1/2)
              * sum_{n, m} x[n, m] Q_in[n, m]
                exp(-i sgn(z) 2 pi [(p - nx/2)(m - nx/2)/nx + (q - ny/2)(n - ny/2)/ny])

    This is the Fresnel diffraction integral with its quadratic phase split
    into an input chirp, one Fourier transform and an output chirp (the
    "Fresnel transformation" of the Abstract and Sec. VI-B.2).  The constant
    exp(ikz)/(i lambda z) dx dy is replaced by the unitary scale
    (nx ny)^(-1/2).  Written out as two centred DFT-matrix products (one per
    axis), not through an FFT."""
    if z == 0:
        raise ValueError("the Fresnel transform is undefined at z = 0")
    x = np.asarray(x)
    ny, nx = x.shape[-2:]
    q_in, q_out = fresnel_chirps(ny, nx, wavelength, dx, dy, z)
    s = 1 if z > 0 else -1
    fx = _centered_dft_matrix(nx, s)
    fy = _centered_dft_matrix(ny, s)
    a = x.astype(np.complex128) * q_in
    # sum over m (last axis) with fx, then over n (rows) with fy
    b = a @ fx.T
    c = np.swapaxes(np.swapaxes(b, -1, -2) @ fy.T, -1, -2)
    return q_out * c / np.sqrt(nx * ny)
