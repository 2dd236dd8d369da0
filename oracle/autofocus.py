"""Autofocus reference in float64: the z-scan with a sharpness metric and the
small CNN that predicts z from a hologram's spectrum.

Test infrastructure only (see the package docstring).

The paper names machine-learning inference only as a future plug-in of the
pipeline (Sec. VIII).  The readings used here:

* Spectrum crop (network input): log(1 + |DFT2(h - mean h)|), centred on DC
  (fftshift), the central 64 x 64 bins, standardised to mean 0 and
  standard deviation 1 over the crop.
* Scan: the +1-order term (the object wave times the conjugate reference)
  sits at minus the reference carrier, (-1/4, -1/4) cycles/pixel.  Its
  sub-band of C x C bins centred there is masked to radius 0.1 cycles/pixel
  around the carrier, demodulated (multiplied by the digital reference, so
  bin f carries the object frequency f + carrier), multiplied by the
  transfer function H_{-z_c} at those object frequencies, inverse-transformed
  at C x C (the field sampled at the band's own rate) and reduced to a
  sharpness:
  forward differences of the amplitude A, G = sqrt(gx^2 + gy^2) on the
  (C-1) x (C-1) interior, score = population variance of G.  The estimate
  is the candidate with the largest score, ties to the lowest z.
* Network: conv3x3(1->32), ReLU, 3 x [conv3x3(32->32), ReLU] (stride 1,
  zero padding 1), global average pooling, FC(32->64), ReLU, FC(64->2) =
  (z_hat, s) with s = log sigma^2; loss = mean over the batch of
  0.5 (s + (z - z_hat)^2 exp(-s)) (Gaussian negative log-likelihood up to a
  constant); Adam with bias correction.
"""

from __future__ import annotations

import numpy as np

from .optics import as_transfer_function

CROP = 64


# ---------------------------------------------------------------- input crop

def spectrum_crop(h, crop: int = CROP) -> np.ndarray:
    """[ny, nx] hologram -> standardised [crop, crop] log-magnitude spectrum
    centred on DC."""
    h = np.asarray(h, dtype=np.float64)
    ny, nx = h.shape
    mag = np.abs(np.fft.fftshift(np.fft.fft2(h - h.mean())))
    c = mag[ny // 2 - crop // 2: ny // 2 + crop // 2, nx // 2 - crop // 2: nx // 2 + crop // 2]
    v = np.log1p(c)
    return (v - v.mean()) / v.std()


# ---------------------------------------------------------------- scan

def sharpness(a) -> float:
    """Population variance of the forward-difference gradient magnitude of
    amplitude a over its (n-1) x (m-1) interior."""
    a = np.asarray(a, dtype=np.float64)
    gx = a[:-1, 1:] - a[:-1, :-1]
    gy = a[1:, :-1] - a[:-1, :-1]
    g = np.sqrt(gx * gx + gy * gy)
    return float(np.var(g))


def order_subband(h, sub: int = 64, radius_cpp: float = 0.1):
    """The masked +1-order sub-band: sub x sub DFT bins centred on
    (-ny/4, -nx/4) (signed indices), zero outside radius_cpp cycles/pixel
    of that carrier.  Returns (values [sub, sub], signed bin indices ky, kx)."""
    h = np.asarray(h, dtype=np.float64)
    ny, nx = h.shape
    spec = np.fft.fft2(h)
    ky = np.arange(sub) - sub // 2 - ny // 4
    kx = np.arange(sub) - sub // 2 - nx // 4
    vals = spec[np.ix_(np.mod(ky, ny), np.mod(kx, nx))]
    dy = (ky + ny // 4) / ny
    dx = (kx + nx // 4) / nx
    mask = (dy[:, None] ** 2 + dx[None, :] ** 2) <= radius_cpp ** 2
    return vals * mask, ky, kx


def scan_scores(h, wavelength, pitch, z_candidates, sub: int = 64, radius_cpp: float = 0.1):
    """Sharpness of the +1-order reconstruction at -z_c for each candidate."""
    h = np.asarray(h, dtype=np.float64)
    ny, nx = h.shape
    vals, ky, kx = order_subband(h, sub, radius_cpp)
    fy = (ky + ny // 4) / (ny * pitch)  # object frequency: bin minus the carrier
    fx = (kx + nx // 4) / (nx * pitch)
    rad = wavelength ** -2 - fx[None, :] ** 2 - fy[:, None] ** 2
    scores = np.empty(len(z_candidates))
    for i, zc in enumerate(z_candidates):
        tf = np.where(rad > 0, np.exp(-2j * np.pi * zc * np.sqrt(np.maximum(rad, 0.0))), 0.0)
        u = np.fft.ifft2(vals * tf)
        scores[i] = sharpness(np.abs(u))
    return scores


def scan(h, wavelength, pitch, z_candidates, sub: int = 64, radius_cpp: float = 0.1):
    """(z estimate, scores): argmax of the sharpness, ties to the lowest z."""
    s = scan_scores(h, wavelength, pitch, z_candidates, sub, radius_cpp)
    return float(np.asarray(z_candidates)[int(np.argmax(s))]), s


def candidates(n: int = 128, lo: float = 0.05, hi: float = 0.5) -> np.ndarray:
    return lo + (hi - lo) * np.arange(n) / (n - 1)


# ---------------------------------------------------------------- network

CONV_SHAPES = [(32, 1), (32, 32), (32, 32), (32, 32)]
FC_SHAPES = [(64, 32), (2, 64)]


def param_shapes():
    """Parameter list in storage order: per conv (weight [co][ci][3][3], bias
    [co]), then per FC (weight [out][in], bias [out])."""
    shapes = []
    for co, ci in CONV_SHAPES:
        shapes += [(co, ci, 3, 3), (co,)]
    for o, i in FC_SHAPES:
        shapes += [(o, i), (o,)]
    return shapes


def n_params() -> int:
    return int(sum(np.prod(s) for s in param_shapes()))


def unflatten(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        out.append(theta[k:k + n].reshape(s))
        k += n
    return out


def flatten(params):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params])


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2/fan_in)), zero biases, from PCG64(seed)."""
    rng = np.random.default_rng(seed)
    ps = []
    for s in param_shapes():
        if len(s) == 1:
            ps.append(np.zeros(s))
        else:
            fan_in = int(np.prod(s[1:]))
            ps.append(rng.standard_normal(s) * np.sqrt(2.0 / fan_in))
    return flatten(ps)


def conv3x3(x, w, b):
    """y[n, o, i, j] = b[o] + sum_{c, di, dj} w[o, c, di, dj] x[n, c, i+di-1, j+dj-1]
    (zero padding 1)."""
    n, c, hh, ww = x.shape
    xp = np.zeros((n, c, hh + 2, ww + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((n, w.shape[0], hh, ww))
    for di in range(3):
        for dj in range(3):
            patch = xp[:, :, di:di + hh, dj:dj + ww]
            y += np.einsum("oc,nchw->nohw", w[:, :, di, dj], patch)
    return y + b[None, :, None, None]


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 w.r.t. its input, weight and bias."""
    n, c, hh, ww = x.shape
    xp = np.zeros((n, c, hh + 2, ww + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for di in range(3):
        for dj in range(3):
            patch = xp[:, :, di:di + hh, dj:dj + ww]
            dw[:, :, di, dj] = np.einsum("nohw,nchw->oc", dy, patch)
            dxp[:, :, di:di + hh, dj:dj + ww] += np.einsum("oc,nohw->nchw", w[:, :, di, dj], dy)
    db = dy.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:-1, 1:-1], dw, db


def forward(theta, x):
    """x [n, 1, h, w] -> (out [n, 2], cache)."""
    p = unflatten(theta)
    acts = [np.asarray(x, dtype=np.float64)]
    for layer in range(4):
        z = conv3x3(acts[-1], p[2 * layer], p[2 * layer + 1])
        acts.append(np.maximum(z, 0.0))
    g = acts[-1].mean(axis=(2, 3))
    w1, b1, w2, b2 = p[8], p[9], p[10], p[11]
    h1 = np.maximum(g @ w1.T + b1, 0.0)
    out = h1 @ w2.T + b2
    return out, (acts, g, h1)


def nll(out, z):
    """Mean Gaussian NLL 0.5 (s + (z - zh)^2 e^{-s}) and d/d out."""
    zh, s = out[:, 0], out[:, 1]
    r = np.asarray(z, dtype=np.float64) - zh
    e = np.exp(-s)
    n = out.shape[0]
    loss = float(np.mean(0.5 * (s + r * r * e)))
    dout = np.stack([-r * e, 0.5 * (1.0 - r * r * e)], axis=1) / n
    return loss, dout


def loss_and_grad(theta, x, z):
    """Loss and the gradient with respect to the flat parameter vector."""
    p = unflatten(theta)
    out, (acts, g, h1) = forward(theta, x)
    loss, dout = nll(out, z)
    w1, w2 = p[8], p[10]
    dw2 = dout.T @ h1
    db2 = dout.sum(axis=0)
    dh1 = (dout @ w2) * (h1 > 0)
    dw1 = dh1.T @ g
    db1 = dh1.sum(axis=0)
    dg = dh1 @ w1
    hw = acts[-1].shape[2] * acts[-1].shape[3]
    da = np.broadcast_to(dg[:, :, None, None] / hw, acts[-1].shape).copy()
    grads = [None] * 12
    grads[8], grads[9], grads[10], grads[11] = dw1, db1, dw2, db2
    for layer in range(3, -1, -1):
        dz = da * (acts[layer + 1] > 0)
        dx, dw, db = conv3x3_backward(acts[layer], p[2 * layer], dz)
        grads[2 * layer], grads[2 * layer + 1] = dw, db
        da = dx
    return loss, flatten(grads)


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
