"""PCA over a window of reconstructed frames, float64.

Test infrastructure only (see the package docstring).

Sec. III-B.1 names the three steps: a covariance matrix of a batch of
holograms, its eigendecomposition, and a projection onto a sub-basis.
Readings (the paper gives no formula):

* X is the window's field as a [P x W] matrix (pixel p, frame t).
* C = X^H X: no centring and no 1/P.
* Eigenpairs in descending eigenvalue order (ties keep the lower index of
  LAPACK's ascending order); each eigenvector's phase is rotated so that its
  largest-magnitude entry is real and positive (for reporting only).
* Y = X V; the rendered image is M0_pca[p] = sum_{c=c1..c2} |Y[p, c]|^2,
  default c1 = 1, c2 = W - 1.

The eigensolver is LAPACK's Hermitian ``eigh`` (shares nothing with the GPU
Jacobi solver).
"""

from __future__ import annotations

import numpy as np

from .temporal import n_windows


def window_matrix(u_window) -> np.ndarray:
    """[W, ny, nx] frames -> X [P, W] with P = ny nx (row-major pixels)."""
    u = np.asarray(u_window).astype(np.complex128)
    return u.reshape(u.shape[0], -1).T


def covariance(x) -> np.ndarray:
    """C = X^H X for X [P, W]."""
    x = np.asarray(x, dtype=np.complex128)
    return x.conj().T @ x


def eig_descending(c):
    """Eigenvalues (descending) and eigenvectors (columns) of Hermitian C,
    with each column's largest-magnitude entry made real positive."""
    w, v = np.linalg.eigh(np.asarray(c, dtype=np.complex128))
    order = np.argsort(-w, kind="stable")
    w = w[order]
    v = v[:, order]
    for col in range(v.shape[1]):
        i = int(np.argmax(np.abs(v[:, col])))
        v[:, col] *= np.conj(v[i, col]) / abs(v[i, col])
    return w, v


def pca_window(u_window, c1: int = 1, c2: int | None = None):
    """PCA of one window.  Returns dict with C, eigvals, eigvecs, m0 [ny, nx]."""
    u = np.asarray(u_window)
    w_count = u.shape[0]
    if c2 is None:
        c2 = w_count - 1
    if not (0 <= c1 <= c2 < w_count):
        raise ValueError("component range must satisfy 0 <= c1 <= c2 < W")
    x = window_matrix(u)
    c = covariance(x)
    lam, v = eig_descending(c)
    y = x @ v
    m0 = np.sum(np.abs(y[:, c1:c2 + 1]) ** 2, axis=1).reshape(u.shape[1:])
    return {"cov": c, "eigvals": lam, "eigvecs": v, "m0": m0}


def pca(u, window: int, stride: int, c1: int = 1, c2: int | None = None):
    """PCA of every complete window of u[T, ny, nx]; stacked results."""
    u = np.asarray(u)
    j_count = n_windows(u.shape[0], window, stride)
    res = [pca_window(u[j * stride: j * stride + window], c1, c2) for j in range(j_count)]
    if not res:
        shape = u.shape[1:]
        return {"cov": np.zeros((0, window, window), np.complex128),
                "eigvals": np.zeros((0, window)), "eigvecs": np.zeros((0, window, window), np.complex128),
                "m0": np.zeros((0,) + shape)}
    return {k: np.stack([r[k] for r in res]) for k in res[0]}
