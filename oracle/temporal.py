"""Short-time Fourier transform over frames and Doppler moments, float64.

Test infrastructure only (see the package docstring).

Readings of Sec. III-B.1 (the temporal transform over consecutive
reconstructed holograms, "done by FFT", then a statistical moment over a
range of indices) and of Sec. VI-B (window and stride):

* Window j covers frames [j s, j s + W); J = floor((T - W)/s) + 1; a trailing
  partial window is dropped.
* S_j[k] = sum_{t<W} U[j s + t] exp(-2i pi k t / W): rectangular window,
  unnormalised.
* The band [f_lo, f_hi] maps to bins ceil(f_lo W/fs) .. floor(f_hi W/fs),
  limited to 0..W/2 (positive frequencies); the optional symmetric band adds
  the mirrored bins W - k (0 < k < W/2) with |f|.
* f_k = k fs / W (Hz) and M_n = sum_{k in band} f_k^n |S_k|^2, n = 0, 1, 2.
"""

from __future__ import annotations

import math

import numpy as np


def n_windows(n_frames: int, window: int, stride: int) -> int:
    """Number of complete windows, floor((T - W)/s) + 1, or 0 when T < W."""
    if window <= 0 or stride <= 0:
        raise ValueError("window and stride must be positive")
    if n_frames < window:
        return 0
    return (n_frames - window) // stride + 1


def dft_matrix(window: int) -> np.ndarray:
    """D[k, t] = exp(-2i pi k t / W) with k t reduced modulo W (exact phase)."""
    k = np.arange(window, dtype=np.int64)
    return np.exp(-2j * np.pi * np.mod(np.outer(k, k), window) / window)


def stft(u, window: int, stride: int) -> np.ndarray:
    """S[j, k, ...] for every complete window of the frame stack u[t, ...]."""
    u = np.asarray(u)
    j_count = n_windows(u.shape[0], window, stride)
    d = dft_matrix(window)
    out = np.empty((j_count, window) + u.shape[1:], dtype=np.complex128)
    for j in range(j_count):
        block = u[j * stride: j * stride + window].astype(np.complex128)
        out[j] = np.tensordot(d, block, axes=(1, 0))
    return out


def band_bins(window: int, fs: float, f_lo: float, f_hi: float,
              symmetric: bool = False):
    """Return (bins, freqs_hz): the temporal-DFT bins inside [f_lo, f_hi]
    and their (non-negative) frequencies.  The bin edges are decided in
    float64: ceil(f_lo*W/fs) and floor(f_hi*W/fs)."""
    k_lo = max(0, math.ceil(f_lo * window / fs))
    k_hi = min(window // 2, math.floor(f_hi * window / fs))
    bins = list(range(k_lo, k_hi + 1))
    freqs = [k * fs / window for k in bins]
    if symmetric:
        for k in list(bins):
            if 0 < k and 2 * k != window:
                bins.append(window - k)
                freqs.append(k * fs / window)
    return np.array(bins, dtype=np.int64), np.array(freqs, dtype=np.float64)


def moments(s, bins, freqs, orders=(0, 1, 2)):
    """M_n[j, ...] = sum_{k in bins} f_k^n |S[j, k, ...]|^2 for each n."""
    s = np.asarray(s)
    power = np.abs(s[:, bins]) ** 2
    out = []
    for n in orders:
        w = np.asarray(freqs, dtype=np.float64) ** n
        out.append(np.tensordot(w, power, axes=(0, 1)))
    return out
