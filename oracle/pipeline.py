"""End-to-end compositions of the oracle steps (float64).

Test infrastructure only (see the package docstring).

Sec. III-B.1 and Fig. 1 order the work as: convert the camera integers,
spatially transform every frame, push the frames into the temporal window,
apply the temporal transform (STFT or PCA), then reduce each pixel to a
moment over a range of temporal indices.  These helpers chain the oracle
steps in that order, one window at a time.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import optics as _optics
from . import pca as _pca
from . import ssa as _ssa
from . import temporal as _temporal

AS = 0
FRESNEL = 1


@dataclass(frozen=True)
class Optics:
    wavelength: float
    dx: float
    dy: float
    z: float
    method: int = AS
    highpass: float = 0.0  # AS only: high-pass radius in cycles per pixel (0 = none)


def reconstruct(frames, opt: Optics | None) -> np.ndarray:
    """Spatial step for a frame stack [T, ny, nx].  Integer input is unpacked
    first; ``opt=None`` means the input already is a complex field."""
    frames = np.asarray(frames)
    if frames.dtype in (np.uint8, np.uint16):
        x = _optics.unpack(frames)
    else:
        x = frames.astype(np.complex128)
    if opt is None:
        return x.astype(np.complex128)
    if opt.method == AS:
        return _optics.angular_spectrum(x, opt.wavelength, opt.dx, opt.dy, opt.z, opt.highpass)
    if opt.method == FRESNEL:
        if opt.highpass:
            raise ValueError("the high-pass filter belongs to the angular-spectrum path")
        return _optics.fresnel(x, opt.wavelength, opt.dx, opt.dy, opt.z)
    raise ValueError(f"unknown method {opt.method}")


def stft_moments(frames, opt: Optics | None, window: int, stride: int, fs: float,
                 f_lo: float, f_hi: float, symmetric: bool = False,
                 keep_spectrum: bool = False):
    """Moments M0/M1/M2 [J, ny, nx] of every complete window; optionally the
    full windowed spectrum S [J, W, ny, nx]."""
    frames = np.asarray(frames)
    j_count = _temporal.n_windows(frames.shape[0], window, stride)
    bins, freqs = _temporal.band_bins(window, fs, f_lo, f_hi, symmetric)
    shape = frames.shape[1:]
    m = [np.zeros((j_count,) + shape) for _ in range(3)]
    spec = np.zeros((j_count, window) + shape, np.complex128) if keep_spectrum else None
    for j in range(j_count):
        u = reconstruct(frames[j * stride: j * stride + window], opt)
        s = _temporal.stft(u, window, window)  # exactly one window
        for i, mi in enumerate(_temporal.moments(s, bins, freqs)):
            m[i][j] = mi[0]
        if keep_spectrum:
            spec[j] = s[0]
    out = {"m0": m[0], "m1": m[1], "m2": m[2], "bins": bins, "freqs": freqs}
    if keep_spectrum:
        out["spectrum"] = spec
    return out


def pca_render(frames, opt: Optics | None, window: int, stride: int, c1: int = 1,
               c2: int | None = None):
    """PCA path: per window covariance, eigenpairs and projection energy."""
    frames = np.asarray(frames)
    j_count = _temporal.n_windows(frames.shape[0], window, stride)
    res = []
    for j in range(j_count):
        u = reconstruct(frames[j * stride: j * stride + window], opt)
        res.append(_pca.pca_window(u, c1, c2))
    if not res:
        return _pca.pca(np.zeros((0,) + frames.shape[1:], np.complex128), window, stride, c1, c2)
    return {k: np.stack([r[k] for r in res]) for k in res[0]}


def stft_volume(frames, opt: Optics | None, window: int, stride: int) -> np.ndarray:
    """The paper's STFT benchmark output (Sec. VI-B.1: the temporal transform
    over a whole window, rendered as a volume): |S_j[k]|^2 for every bin
    k = 0 .. W-1 of every complete window, [J, W, ny, nx] float64.  Reading:
    the power of each bin, bins in DFT order."""
    frames = np.asarray(frames)
    j_count = _temporal.n_windows(frames.shape[0], window, stride)
    out = np.zeros((j_count, window) + frames.shape[1:])
    for j in range(j_count):
        u = reconstruct(frames[j * stride: j * stride + window], opt)
        s = _temporal.stft(u, window, window)[0]
        out[j] = s.real ** 2 + s.imag ** 2
    return out


def ssa_render(frames, opt: Optics | None, window: int, stride: int, fs: float, f_lo: float, f_hi: float,
               c1: int = 1, c2: int | None = None, symmetric: bool = False, keep_spectrum: bool = False):
    """SSA + FFT path: every window reconstructed, filtered by its components
    c1..c2 (covariance, eigenpairs, projection and back), transformed in
    time, reduced to the moments over the band."""
    frames = np.asarray(frames)
    j_count = _temporal.n_windows(frames.shape[0], window, stride)
    res = []
    for j in range(j_count):
        u = reconstruct(frames[j * stride: j * stride + window], opt)
        res.append(_ssa.ssa_moments(u, window, window, fs, f_lo, f_hi, c1, c2, symmetric, keep_spectrum))
    if not res:
        return _ssa.ssa_moments(np.zeros((0,) + frames.shape[1:], np.complex128), window, stride, fs, f_lo, f_hi,
                                c1, c2, symmetric, keep_spectrum)
    out = {k: np.concatenate([r[k] for r in res]) for k in res[0] if k not in ("bins", "freqs")}
    out["bins"], out["freqs"] = res[0]["bins"], res[0]["freqs"]
    return out
