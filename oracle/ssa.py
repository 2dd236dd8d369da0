"""SSA + FFT temporal path, float64.  Test infrastructure only (see the
package docstring).

Sec. III-B.1 lists three short-time temporal transforms: the FFT, PCA, and
"SSA and FFT", whose underlying SVD is obtained by eigen-decomposition of
the data: a covariance matrix of the window's holograms, its
eigen-decomposition, and a projection of the data onto a sub-basis; Sec.
II-B.3 lists SSA among the temporal analyses.  The paper gives no formula
and no embedding dimension.  Readings (the same as the PCA path's for the
first two steps):

* X is the window's field as a [P x W] matrix (pixel p, frame t): each
  pixel's W values form one row, so the embedding dimension is the window
  length W and the trajectory matrix stacks the pixels.
* C = X^H X (no centring, no 1/P); eigenpairs in descending eigenvalue
  order; V_S = the eigenvectors of the components c1..c2 (default 1..W-1,
  which removes the dominant, static component).
* Projection onto the sub-basis and back: the filtered window is
  X_f = X V_S V_S^H (the rank-|S| SVD reconstruction of the window from the
  chosen components).
* The FFT then runs over the filtered window exactly as in the STFT path:
  S[k] = sum_t X_f[:, t] exp(-2i pi k t / W), and the moments are taken over
  the band as there.

The eigensolver is LAPACK's Hermitian ``eigh`` (as in the PCA oracle).
"""

from __future__ import annotations

import numpy as np

from . import pca as _pca
from . import temporal as _temporal


def ssa_filter(u_window, c1: int = 1, c2: int | None = None):
    """The window u_window[W, ...] rebuilt from its components c1..c2.
    Returns (filtered frames [W, ...], eigenvalues descending)."""
    u = np.asarray(u_window)
    w = u.shape[0]
    if c2 is None:
        c2 = w - 1
    if not (0 <= c1 <= c2 < w):
        raise ValueError("component range must satisfy 0 <= c1 <= c2 < W")
    x = _pca.window_matrix(u)                       # [P, W]
    lam, v = _pca.eig_descending(_pca.covariance(x))
    vs = v[:, c1:c2 + 1]                            # [W, |S|]
    xf = (x @ vs) @ vs.conj().T                     # projection and back: [P, W]
    return xf.T.reshape(u.shape), lam


def ssa_stft_window(u_window, c1: int = 1, c2: int | None = None):
    """S[k, ...] of one window after the SSA filter (all W bins) and the
    eigenvalues."""
    uf, lam = ssa_filter(u_window, c1, c2)
    w = uf.shape[0]
    return _temporal.stft(uf, w, w)[0], lam


def ssa_moments(u, window: int, stride: int, fs: float, f_lo: float, f_hi: float, c1: int = 1,
                c2: int | None = None, symmetric: bool = False, keep_spectrum: bool = False):
    """Moments M0/M1/M2 [J, ...] of every complete window of the field stack
    u[T, ...] after the SSA filter, eigenvalues [J, W], optionally the
    filtered spectrum [J, W, ...]."""
    u = np.asarray(u)
    j_count = _temporal.n_windows(u.shape[0], window, stride)
    bins, freqs = _temporal.band_bins(window, fs, f_lo, f_hi, symmetric)
    shape = u.shape[1:]
    m = [np.zeros((j_count,) + shape) for _ in range(3)]
    lam = np.zeros((j_count, window))
    spec = np.zeros((j_count, window) + shape, np.complex128) if keep_spectrum else None
    for j in range(j_count):
        s, lam[j] = ssa_stft_window(u[j * stride: j * stride + window], c1, c2)
        for i, mi in enumerate(_temporal.moments(s[None], bins, freqs)):
            m[i][j] = mi[0]
        if keep_spectrum:
            spec[j] = s
    out = {"m0": m[0], "m1": m[1], "m2": m[2], "eigvals": lam, "bins": bins, "freqs": freqs}
    if keep_spectrum:
        out["spectrum"] = spec
    return out
