"""Off-axis Doppler interferogram stacks from a seed (see package docstring).

Recipe (one stack):

1. Object: iid circular-Gaussian speckle s[y, x] ~ CN(0, 1) on the object
   grid (same pitch as the sensor).  Each object pixel carries its own
   Doppler frequency f_d[y, x] ~ U[0, f_max], so at frame t the object is
   a_t = s * exp(+2i pi f_d t / fs).
2. Sensor-plane object wave: o_t = Ky a_t Kx^T, where K[a, b] is the
   paraxial (quadratic-phase) response of a point source at distance z,
   exp(i pi ((a - b) pitch)^2 / (lambda z)), kept only where that chirp is
   sampled below Nyquist (|a - b| pitch <= lambda |z| / (2 pitch)).
3. Reference: a plane wave of amplitude ref_ratio * rms(o_0), tilted by a
   quarter cycle per pixel on both axes: exp(2i pi (x + y) / 4).
4. Intensity I_t = |r + o_t|^2, scaled so that the mean of frame 0 equals
   mean_dn (64 DN for 8 bits, 1024 DN for 12 bits), then Poisson counts with
   a gain of 1 e-/DN, clipped to the bit depth.

Random streams: numpy PCG64 seeded through SeedSequence(seed); the object,
Doppler map and Poisson draws come from one child stream and a drawn z
(when requested) from another, so every array is a function of the seed.
"""

from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class HoloSpec:
    frames: int
    ny: int
    nx: int
    wavelength: float = 852e-9
    pitch: float = 20e-6
    z: float = 0.2
    fs: float = 33e3
    f_max: float = 8e3
    bits: int = 8
    seed: int = 0
    ref_ratio: float = 3.0
    mean_dn: float | None = None

    @property
    def dtype(self):
        return np.uint8 if self.bits <= 8 else np.uint16

    @property
    def max_dn(self) -> int:
        return (1 << self.bits) - 1

    @property
    def target_mean(self) -> float:
        if self.mean_dn is not None:
            return float(self.mean_dn)
        return 64.0 if self.bits <= 8 else 1024.0


def point_response_1d(n: int, pitch: float, wavelength: float, z: float) -> np.ndarray:
    """K[a, b] = exp(i pi ((a-b) pitch)^2 / (lambda z)) on its unaliased support."""
    d = (np.arange(n)[:, None] - np.arange(n)[None, :]) * pitch
    k = np.exp(1j * np.pi * d * d / (wavelength * z))
    k[np.abs(d) > wavelength * abs(z) / (2.0 * pitch)] = 0.0
    return k.astype(np.complex64)


def _child_streams(seed: int):
    obj_seq, z_seq = np.random.SeedSequence(seed).spawn(2)
    return np.random.default_rng(obj_seq), np.random.default_rng(z_seq)


def drawn_z(seed: int, lo: float = 0.1, hi: float = 0.4) -> float:
    """A reconstruction distance drawn once from the seed: lo + (hi-lo) U."""
    _, zrng = _child_streams(seed)
    return float(lo + (hi - lo) * zrng.uniform())


def hologram_stack(spec: HoloSpec, chunk: int | None = None) -> np.ndarray:
    """Frames [T, ny, nx] (uint8 or uint16) following the module recipe.

    Frames are produced ``chunk`` at a time (by default about 1 Mi pixels
    per chunk, which keeps every temporary small)."""
    if chunk is None:
        chunk = max(1, (1 << 20) // (spec.ny * spec.nx))
    rng, _ = _child_streams(spec.seed)
    ny, nx = spec.ny, spec.nx
    s = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))) / np.sqrt(2.0)
    fd = rng.uniform(0.0, spec.f_max, (ny, nx))
    s64 = s.astype(np.complex64)
    kx = point_response_1d(nx, spec.pitch, spec.wavelength, spec.z)
    ky = point_response_1d(ny, spec.pitch, spec.wavelength, spec.z)
    norm = 1.0 / np.sqrt(max(1, np.count_nonzero(kx[nx // 2])) * max(1, np.count_nonzero(ky[ny // 2])))
    yy, xx = np.mgrid[0:ny, 0:nx]
    carrier = np.cos(np.pi * (xx + yy) / 2.0) + 1j * np.sin(np.pi * (xx + yy) / 2.0)
    out = np.empty((spec.frames, ny, nx), dtype=spec.dtype)
    r = None
    scale = None
    kxt = np.ascontiguousarray(kx.T)
    for t0 in range(0, spec.frames, chunk):
        t = np.arange(t0, min(spec.frames, t0 + chunk), dtype=np.float64)
        phase = (2 * np.pi / spec.fs) * fd[None] * t[:, None, None]
        rot = np.empty(phase.shape, np.complex64)  # exp(i phase), via real cos/sin
        rot.real = np.cos(phase)
        rot.imag = np.sin(phase)
        a = s64[None] * rot
        o = (ky[None] @ a @ kxt[None]) * np.float32(norm)
        o = o.astype(np.complex128)
        if r is None:
            rms = np.sqrt(np.mean(o[0].real ** 2 + o[0].imag ** 2))
            r = spec.ref_ratio * rms * carrier
            f0 = r + o[0]
            scale = spec.target_mean / np.mean(f0.real ** 2 + f0.imag ** 2)
        f = r[None] + o
        lam = (f.real ** 2 + f.imag ** 2) * scale
        counts = rng.poisson(lam)
        np.clip(counts, 0, spec.max_dn, out=counts)
        out[t0:t0 + len(t)] = counts.astype(spec.dtype)
    return out


def config_c1() -> tuple[np.ndarray, HoloSpec]:
    """Tiny plain-method case: 64 frames of 128x128 uint8, z = 0.2 m,
    fs = 33 kHz, Doppler up to 8 kHz, seed 0."""
    spec = HoloSpec(frames=64, ny=128, nx=128, z=0.2, fs=33e3, seed=0)
    return hologram_stack(spec), spec


def config_c2_block(frames: int = 2048) -> tuple[np.ndarray, HoloSpec]:
    """Headline shape: 256x256 uint8 at fs = 71.4 kHz with z drawn once in
    [0.1, 0.4] m from seed 1.  Returns a base block of ``frames`` frames;
    the full 65,536-frame stream replays it cyclically."""
    z = drawn_z(1)
    spec = HoloSpec(frames=frames, ny=256, nx=256, z=z, fs=71.4e3, seed=1)
    return hologram_stack(spec), spec


def config_c3(frames: int = 128) -> tuple[np.ndarray, HoloSpec]:
    """Precision case: 1024x1024 uint16 holding 12-bit values, z = 0.5 m,
    seed 2 (fs is not stated; 5 kHz is used)."""
    spec = HoloSpec(frames=frames, ny=1024, nx=1024, z=0.5, fs=5e3, bits=12, seed=2)
    return hologram_stack(spec), spec


STREAM_CLASSES = (
    # (ny, nx, bits, fs, window, base-block frames)
    (256, 256, 8, 71.4e3, 16, 2048),
    (512, 512, 8, 20e3, 32, 1024),
    (512, 1024, 12, 5e3, 64, 512),
)


def stream_block(cls: int, stream_id: int, frames: int | None = None) -> tuple[np.ndarray, HoloSpec]:
    """Synthetic camera block for a serving-loop stream of class ``cls``
    (0: 256^2 u8 71.4 kHz, 1: 512^2 u8 20 kHz, 2: 1024x512 u16 5 kHz);
    z drawn in [0.1, 0.4] m, seed 10000 + stream_id."""
    ny, nx, bits, fs, _, base = STREAM_CLASSES[cls]
    seed = 10000 + stream_id
    spec = HoloSpec(frames=frames or base, ny=ny, nx=nx, z=drawn_z(seed), fs=fs, bits=bits, seed=seed)
    return hologram_stack(spec), spec


def with_frames(spec: HoloSpec, frames: int) -> HoloSpec:
    return replace(spec, frames=frames)
