"""Closed-form checks ("pins") that fix the oracle independently of itself.

Each check takes the oracle function it exercises as an argument and returns
an error figure, so the same check can be run on the oracle (must pass) and
on deliberately broken copies of it (must fail, see test_oracle_mutations).
Expected values come from closed forms, from brute-force sums written with
explicit loops, or from invariants -- never from the oracle itself.
"""

from __future__ import annotations

import cmath
import math

import numpy as np

LAMBDA = 852e-9


def rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


# ---------------------------------------------------------------- angular spectrum

def plane_wave_error(as_fn, z=0.13, ny=24, nx=32, dx=20e-6, dy=15e-6):
    """A sum of plane waves whose frequencies lie on the DFT grid propagates
    exactly: each term picks up exp(2i pi z sqrt(1/lambda^2 - |f|^2))."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    xs, ys = xx * dx, yy * dy
    terms = [(1.0 + 0.5j, 3, -2), (-0.25 + 0.75j, -5, 7), (0.6, 11, 0), (0.3j, 0, -9)]
    x = np.zeros((ny, nx), np.complex128)
    expect = np.zeros((ny, nx), np.complex128)
    for a, i, j in terms:
        fx, fy = i / (nx * dx), j / (ny * dy)
        wave = a * np.exp(2j * np.pi * (fx * xs + fy * ys))
        x += wave
        expect += wave * cmath.exp(2j * math.pi * z * math.sqrt(LAMBDA ** -2 - fx * fx - fy * fy))
    return rel(as_fn(x, LAMBDA, dx, dy, z), expect)


def gaussian_beam(n, pitch, w0, z, coords):
    """Paraxial Gaussian beam exp(ikz)/q exp(-r^2/(w0^2 q)), q = 1 + iz/zR."""
    zr = math.pi * w0 * w0 / LAMBDA
    q = 1 + 1j * z / zr
    r2 = coords[0] ** 2 + coords[1] ** 2
    return cmath.exp(2j * math.pi * z / LAMBDA) / q * np.exp(-r2 / (w0 * w0 * q))


def gaussian_as_error(as_fn, z, n=128, pitch=20e-6, w0_px=8):
    c = (np.arange(n) - n // 2) * pitch
    yy, xx = np.meshgrid(c, c, indexing="ij")
    w0 = w0_px * pitch
    x0 = np.exp(-(xx ** 2 + yy ** 2) / w0 ** 2)
    expect = gaussian_beam(n, pitch, w0, z, (xx, yy))
    return rel(as_fn(x0, LAMBDA, pitch, pitch, z), expect)


def gaussian_fresnel_error(fr_fn, z, n=128, pitch=20e-6, w0_px=8):
    """Fresnel of a Gaussian, rescaled by the omitted physical constant
    sqrt(N^2) exp(ikz)/(i lambda z) dx dy, sampled on the output grid."""
    c = (np.arange(n) - n // 2) * pitch
    yy, xx = np.meshgrid(c, c, indexing="ij")
    w0 = w0_px * pitch
    x0 = np.exp(-(xx ** 2 + yy ** 2) / w0 ** 2)
    out_pitch = LAMBDA * abs(z) / (n * pitch)
    co = (np.arange(n) - n // 2) * out_pitch
    oy, ox = np.meshgrid(co, co, indexing="ij")
    expect = gaussian_beam(n, pitch, w0, z, (ox, oy))
    u = fr_fn(x0, LAMBDA, pitch, pitch, z)
    phys = u * n * cmath.exp(2j * math.pi * z / LAMBDA) / (1j * LAMBDA * z) * pitch * pitch
    return rel(phys, expect)


def point_source_fresnel_error(fr_fn, z, ny=16, nx=32, dx=20e-6, dy=30e-6, at=(5, 21)):
    """A Kronecker delta at (eta0, xi0) gives the paraxial spherical wave
    centred there, exp(i pi ((x - xi0)^2 + (y - eta0)^2) / (lambda z)), with
    the unitary scale 1/sqrt(nx ny)."""
    n0, m0 = at
    x = np.zeros((ny, nx))
    x[n0, m0] = 1.0
    xi0, eta0 = (m0 - nx // 2) * dx, (n0 - ny // 2) * dy
    px = (np.arange(nx) - nx // 2) * LAMBDA * abs(z) / (nx * dx)
    py = (np.arange(ny) - ny // 2) * LAMBDA * abs(z) / (ny * dy)
    yy, xx = np.meshgrid(py, px, indexing="ij")
    expect = np.exp(1j * np.pi * ((xx - xi0) ** 2 + (yy - eta0) ** 2) / (LAMBDA * z)) / math.sqrt(nx * ny)
    return rel(fr_fn(x, LAMBDA, dx, dy, z), expect)


def brute_force_as(x, wavelength, dx, dy, z):
    """Direct O(N^4) sums: forward DFT, transfer function, inverse DFT."""
    ny, nx = x.shape
    spec = np.zeros((ny, nx), np.complex128)
    for q in range(ny):
        for p in range(nx):
            acc = 0j
            for n in range(ny):
                for m in range(nx):
                    acc += x[n, m] * cmath.exp(-2j * math.pi * (p * m / nx + q * n / ny))
            fx = (p if p < (nx + 1) // 2 else p - nx) / (nx * dx)
            fy = (q if q < (ny + 1) // 2 else q - ny) / (ny * dy)
            rad = wavelength ** -2 - fx * fx - fy * fy
            spec[q, p] = acc * (cmath.exp(2j * math.pi * z * math.sqrt(rad)) if rad > 0 else 0)
    out = np.zeros((ny, nx), np.complex128)
    for n in range(ny):
        for m in range(nx):
            acc = 0j
            for q in range(ny):
                for p in range(nx):
                    acc += spec[q, p] * cmath.exp(2j * math.pi * (p * m / nx + q * n / ny))
            out[n, m] = acc / (nx * ny)
    return out


def brute_force_fresnel(x, wavelength, dx, dy, z):
    """Direct sum of the Fresnel integral with the quadratic phase of
    |x - xi|^2 kept whole (not split into chirps), on the output grid."""
    ny, nx = x.shape
    opx = wavelength * abs(z) / (nx * dx)
    opy = wavelength * abs(z) / (ny * dy)
    out = np.zeros((ny, nx), np.complex128)
    for q in range(ny):
        for p in range(nx):
            xo, yo = (p - nx // 2) * opx, (q - ny // 2) * opy
            acc = 0j
            for n in range(ny):
                for m in range(nx):
                    xi, eta = (m - nx // 2) * dx, (n - ny // 2) * dy
                    acc += x[n, m] * cmath.exp(1j * math.pi * ((xo - xi) ** 2 + (yo - eta) ** 2) / (wavelength * z))
            out[q, p] = acc / math.sqrt(nx * ny)
    return out


def brute_force_stft(u, window, stride):
    t_count = u.shape[0]
    j_count = (t_count - window) // stride + 1
    out = np.zeros((j_count, window) + u.shape[1:], np.complex128)
    for j in range(j_count):
        for k in range(window):
            for t in range(window):
                out[j, k] += u[j * stride + t] * cmath.exp(-2j * math.pi * k * t / window)
    return out


# ---------------------------------------------------------------- temporal

def pure_tone_errors(stft_fn, moments_fn, window=32, k0=5, fs=33e3):
    """U[t] = a(r) exp(2i pi k0 t / W): all energy lands in bin k0 with
    |S_k0|^2 = W^2 |a|^2; M1 = f_k0 M0 and M2 = f_k0^2 M0 in a band that
    contains k0."""
    rng = np.random.default_rng(7)
    a = rng.standard_normal((6, 5)) + 1j * rng.standard_normal((6, 5))
    t = np.arange(window)
    u = a[None] * np.exp(2j * np.pi * k0 * t / window)[:, None, None]
    s = stft_fn(u, window, window)
    leak = np.sum(np.abs(np.delete(s[0], k0, axis=0)) ** 2) / np.sum(np.abs(s[0]) ** 2)
    peak = rel(np.abs(s[0, k0]) ** 2, window ** 2 * np.abs(a) ** 2)
    fk = k0 * fs / window
    bins = np.array([k0 - 1, k0, k0 + 1])
    freqs = bins * fs / window
    m0, m1, m2 = moments_fn(s, bins, freqs)
    e0 = rel(m0[0], window ** 2 * np.abs(a) ** 2)
    e1 = rel(m1[0], fk * window ** 2 * np.abs(a) ** 2)
    e2 = rel(m2[0], fk * fk * window ** 2 * np.abs(a) ** 2)
    return max(leak, peak, e0, e1, e2)


# ---------------------------------------------------------------- PCA

def pca_construction_error(pca_window_fn, w=8, ny=12, nx=10, c1=1, c2=5):
    """X = Q diag(sigma) P^H with orthonormal Q [P x W] and unitary P:
    eigenvalues sigma^2 (descending), C = P diag(sigma^2) P^H and
    M0[p] = sum_{c1..c2} sigma_c^2 |Q[p, c]|^2."""
    rng = np.random.default_rng(11)
    npx = ny * nx
    qm, _ = np.linalg.qr(rng.standard_normal((npx, w)) + 1j * rng.standard_normal((npx, w)))
    pm, _ = np.linalg.qr(rng.standard_normal((w, w)) + 1j * rng.standard_normal((w, w)))
    sigma = np.array([9.0, 5.0, 4.0, 3.0, 2.5, 1.5, 1.0, 0.5])[:w]
    x = qm @ np.diag(sigma) @ pm.conj().T
    u = x.T.reshape(w, ny, nx)
    r = pca_window_fn(u, c1, c2)
    e_lam = rel(r["eigvals"], sigma ** 2)
    e_cov = rel(r["cov"], pm @ np.diag(sigma ** 2) @ pm.conj().T)
    m0 = np.sum((sigma[c1:c2 + 1] ** 2)[None, :] * np.abs(qm[:, c1:c2 + 1]) ** 2, axis=1).reshape(ny, nx)
    e_m0 = rel(r["m0"], m0)
    v = r["eigvecs"]
    e_orth = float(np.linalg.norm(v.conj().T @ v - np.eye(w)))
    return max(e_lam, e_cov, e_m0, e_orth)


def pca_rank1_error(pca_window_fn, w=6, ny=5, nx=7):
    """X = a b^T: lambda_0 = |a|^2 |b|^2 and the other eigenvalues vanish;
    M0 over components 1..W-1 is zero."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal(ny * nx) + 1j * rng.standard_normal(ny * nx)
    b = rng.standard_normal(w) + 1j * rng.standard_normal(w)
    x = np.outer(a, b)
    r = pca_window_fn(x.T.reshape(w, ny, nx), 1, w - 1)
    lam0 = np.linalg.norm(a) ** 2 * np.linalg.norm(b) ** 2
    return max(abs(r["eigvals"][0] - lam0) / lam0,
               float(np.max(np.abs(r["eigvals"][1:]))) / lam0,
               float(np.max(r["m0"])) / lam0)


# ---------------------------------------------------------------- high-pass filter and power volume

def highpass_plane_wave_error(as_hp_fn, radius=0.12, z=0.07, ny=24, nx=32, dx=20e-6, dy=15e-6):
    """Plane waves on the DFT grid: the ones inside the radius vanish, the
    ones outside propagate exactly (closed form), whatever their mix."""
    y, x = np.mgrid[0:ny, 0:nx]
    waves = [(0, 0, 1.0), (1, 2, 0.5 - 0.2j), (-2, 1, 0.3j),   # radius < 0.12 cycles/px
             (5, -7, 0.8), (-8, 11, -0.4 + 0.1j), (12, 0, 0.25)]  # radius > 0.12
    field = np.zeros((ny, nx), np.complex128)
    want = np.zeros((ny, nx), np.complex128)
    for ky, kx, a in waves:
        e = a * np.exp(2j * math.pi * (kx * x / nx + ky * y / ny))
        field += e
        r2 = (kx / nx) ** 2 + (ky / ny) ** 2
        if r2 >= radius ** 2:
            fx, fy = kx / (nx * dx), ky / (ny * dy)
            kz = math.sqrt(LAMBDA ** -2 - fx * fx - fy * fy)
            want += e * cmath.exp(2j * math.pi * z * kz)
    return rel(as_hp_fn(field, LAMBDA, dx, dy, z, radius), want)


def volume_errors(volume_fn, window=16, ny=3, nx=4):
    """Closed forms for the per-bin power: a pure tone e^{2 i pi k0 t / W}
    with amplitude a gives W^2 |a|^2 in bin k0 and 0 elsewhere; random data
    obeys Parseval per window (sum_k |S_k|^2 = W sum_t |u_t|^2)."""
    t = np.arange(2 * window)
    k0 = 3
    a = (0.7 - 0.4j) * np.ones((ny, nx))
    u = a[None] * np.exp(2j * math.pi * k0 * t / window)[:, None, None]
    v = volume_fn(u, window, window)
    want = np.zeros_like(v)
    want[:, k0] = window ** 2 * abs(a[0, 0]) ** 2
    e_tone = float(np.max(np.abs(v - want)) / (window ** 2))
    rng = np.random.default_rng(12)
    r = rng.standard_normal((3 * window, ny, nx)) + 1j * rng.standard_normal((3 * window, ny, nx))
    v = volume_fn(r, window, window)
    e = np.stack([(np.abs(r[j * window:(j + 1) * window]) ** 2).sum(axis=0) for j in range(3)])
    e_pars = float(np.max(np.abs(v.sum(axis=1) - window * e)) / np.max(window * e))
    return e_tone, e_pars


# ---------------------------------------------------------------- magnitude / argument images

def tone_image_errors(magnitude_fn, argument_fn, window=16, bins=(3, 5), shape=(3, 4), seed=4):
    """Two tones a_i exp(2i pi k_i t / W) at every pixel have, in closed form,
    the spectrum S_{k_i} = W a_i and zero elsewhere.  Over the range
    k_1 .. k_2 the magnitude image is W (|a_1| + |a_2|) and the argument image
    arg(a_1 + a_2); over k_1 alone, W |a_1| and arg(a_1).  Returns the largest
    (magnitude, wrapped argument) errors over both ranges."""
    rng = np.random.default_rng(seed)
    a = [rng.standard_normal(shape) + 1j * rng.standard_normal(shape) for _ in bins]
    spec = np.zeros((1, window) + shape, np.complex128)
    for ai, k in zip(a, bins):
        spec[0, k] = window * ai
    both = list(range(bins[0], bins[1] + 1))
    one = [bins[0]]

    def wrap(d):
        return np.abs(np.angle(np.exp(1j * d)))

    em = max(np.max(np.abs(magnitude_fn(spec[:, both])[0] - window * (np.abs(a[0]) + np.abs(a[1])))),
             np.max(np.abs(magnitude_fn(spec[:, one])[0] - window * np.abs(a[0]))))
    ea = max(np.max(wrap(argument_fn(spec[:, both])[0] - np.angle(a[0] + a[1]))),
             np.max(wrap(argument_fn(spec[:, one])[0] - np.angle(a[0]))))
    return float(em), float(ea)


# ---------------------------------------------------------------- post-processing helpers

def disk_mask_errors(disk_fn):
    """Count of wrong pixels of the registration mask on three grids whose
    in-disk sets are derived by hand.  A disk of radius r centred on a lattice
    point holds N(r) lattice points (Gauss's circle problem: N(2) = 13,
    N(3) = 29).  The mask radius is ``mask_radius * min(nx, ny) / 2`` about
    the centre pixel (ny/2, nx/2), boundary included:

    * 8 x 8, mask_radius 0.5: r = 2 about (4, 4), all 13 points on the grid;
    * 6 x 10, mask_radius 1.0: r = 3 about (3, 5); of the 29 points, (6, 5)
      lies below the last row, so 28 remain;
    * 8 x 12, mask_radius 0.1: r = 0.4, the centre pixel (4, 6) alone."""
    def expect(ny, nx, cy, cx, r2):
        m = np.zeros((ny, nx))
        for y in range(ny):
            for x in range(nx):
                if (y - cy) ** 2 + (x - cx) ** 2 <= r2:
                    m[y, x] = 1.0
        return m

    bad = 0
    for (ny, nx, rad, count, cy, cx, r2) in ((8, 8, 0.5, 13, 4, 4, 4), (6, 10, 1.0, 28, 3, 5, 9),
                                              (8, 12, 0.1, 1, 4, 6, 0)):
        got = np.asarray(disk_fn(ny, nx, rad), np.float64)
        bad += abs(int(round(got.sum())) - count)
        bad += int(np.sum(got != expect(ny, nx, cy, cx, r2)))
    return bad


def gaussian_kernel_errors(gauss_fn, sigmas=(1.5, 0.4, 2.2)):
    """A Gaussian of standard deviation sigma, g(i, j) proportional to
    exp(-(i^2 + j^2) / (2 sigma^2)), truncated at 3 sigma and normalised:
    the side is 2 ceil(3 sigma) + 1, the sum is 1, and the ratios to the
    centre value are exp(-1/(2 sigma^2)) one step along an axis,
    exp(-1/sigma^2) one step along the diagonal and exp(-5/(2 sigma^2)) at
    (2, 1).  Returns the largest relative error (a wrong side counts as 1)."""
    worst = 0.0
    for s in sigmas:
        g = np.asarray(gauss_fn(s), np.float64)
        r = math.ceil(3 * s)
        if g.shape != (2 * r + 1, 2 * r + 1):
            return 1.0
        c = g[r, r]
        checks = [(g.sum(), 1.0), (g[r + 1, r] / c, math.exp(-1 / (2 * s * s))),
                  (g[r, r - 1] / c, math.exp(-1 / (2 * s * s))),
                  (g[r + 1, r + 1] / c, math.exp(-1 / (s * s))),
                  (g[r - 2, r + 1] / c, math.exp(-5 / (2 * s * s)))]
        for got, want in checks:
            worst = max(worst, abs(got - want) / want)
    return worst


def convolution_shift_error(conv_fn, shift=(1, 2), size=5, shape=(2, 9, 11), seed=6):
    """Convolution with a unit impulse displaced by (a, b) from the kernel
    centre moves the image by +(a, b): (x * k)[i, j] = x[i - a, j - b], zero
    where that falls outside the image.  A correlation would move it the
    other way.  Returns the largest absolute error."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    k = np.zeros((size, size))
    c = size // 2
    k[c + shift[0], c + shift[1]] = 1.0
    want = np.zeros_like(x)
    a, b = shift
    for i in range(shape[1]):
        for j in range(shape[2]):
            if 0 <= i - a < shape[1] and 0 <= j - b < shape[2]:
                want[:, i, j] = x[:, i - a, j - b]
    return float(np.max(np.abs(np.asarray(conv_fn(x, k)) - want)))


# ---------------------------------------------------------------- SSA + FFT

def _orthogonal_pixel_vectors(shape, count, norms, seed):
    """`count` complex pixel images, mutually orthogonal (as vectors over the
    pixels), with the given norms (Gram-Schmidt on random draws)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        for o in out:
            v = v - np.vdot(o, v) / np.vdot(o, o) * o
        out.append(v / np.linalg.norm(v) * norms[i])
    return out


def ssa_tone_errors(ssa_stft_fn, window=16, shape=(5, 6), seed=21):
    """Closed forms of the filter's action on windows whose components are
    known.  A window u_t = b + a_1 e^{2i pi k_1 t/W} + a_2 e^{2i pi k_2 t/W}
    with pixel images b, a_1, a_2 mutually orthogonal and
    |b| > |a_1| > |a_2| has exactly three non-zero eigenpairs of C = X^H X:
    W|b|^2 (the constant time vector), W|a_1|^2 (tone k_1) and W|a_2|^2
    (tone k_2), the time vectors being orthogonal over a whole window.  So
    the spectrum S of the filtered window is, in closed form:

    * components 0..W-1 (everything): S_0 = W b, S_k1 = W a_1, S_k2 = W a_2;
    * components 1..W-1 (the static part removed): S_k1 = W a_1, S_k2 = W a_2;
    * component 1 alone: S_k1 = W a_1;   component 0 alone: S_0 = W b;
    * components 2..W-1: S_k2 = W a_2;
    every other bin zero.  Returns the largest error over the five ranges,
    relative to W |b|."""
    k1, k2 = 3, 11
    b, a1, a2 = _orthogonal_pixel_vectors(shape, 3, (3.0, 2.0, 1.0), seed)
    t = np.arange(window)[:, None, None]
    u = (b[None] + a1[None] * np.exp(2j * np.pi * k1 * t / window)
         + a2[None] * np.exp(2j * np.pi * k2 * t / window))
    cases = [((0, window - 1), {0: b, k1: a1, k2: a2}), ((1, window - 1), {k1: a1, k2: a2}),
             ((1, 1), {k1: a1}), ((0, 0), {0: b}), ((2, window - 1), {k2: a2})]
    worst = 0.0
    scale = window * np.linalg.norm(b)
    for (c1, c2), want in cases:
        s = np.asarray(ssa_stft_fn(u, c1, c2))
        ref = np.zeros((window,) + shape, np.complex128)
        for k, amp in want.items():
            ref[k] = window * amp
        worst = max(worst, float(np.linalg.norm((s - ref).ravel()) / scale))
    return worst
