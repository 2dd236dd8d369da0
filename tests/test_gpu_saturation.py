"""The mixed form at full-scale input, against the FP64 oracle at 2e-3.

The mixed form stores spectra and fields as fp16 with power-of-two scales
chosen from the largest value a coherent full-scale input can reach.  These
cases drive it there: constant frames at the top of the 8-, 12- and 16-bit
ranges (all energy in one spectral bin), a full-scale plane wave on the DFT
grid, and a full-scale off-axis hologram of a point source reconstructed at
its distance (the +1 order focuses to a spot), also modulated in time so the
moments are not trivially zero.  The FP32 form is run on the same inputs at
1e-5.
"""

import numpy as np
import pytest
import torch

from oracle import pipeline
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu

LAM = 852e-9
PITCH = 20e-6
TOL = {0: 1e-5, 1: 2e-3}


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx(hv):
    c = hv.Context(0)
    yield c
    c.close()


def _zone_plate(ny, nx, z, maxv, phase_t=0.0):
    """Intensity of a point source at distance z (paraxial quadratic phase)
    beating with a plane reference tilted a quarter cycle per pixel on both
    axes, at full modulation: maxv/2 (1 + cos(...)), rounded."""
    y, x = np.mgrid[0:ny, 0:nx]
    chirp = np.pi * (((x - nx / 2) * PITCH) ** 2 + ((y - ny / 2) * PITCH) ** 2) / (LAM * z)
    v = maxv / 2.0 * (1.0 + np.cos(np.pi * (x + y) / 2.0 - chirp + phase_t))
    return np.rint(v)


def _as_field_case(ctx, hv, frames, dtype, z, prec):
    opt = hv.Optics(LAM, PITCH, PITCH, z, hv.HV_AS)
    x = frames.astype(dtype)
    u = ctx.hv_propagate(torch.from_numpy(x).cuda(), opt, prec)
    torch.cuda.synchronize()
    ref = pipeline.reconstruct(x, pipeline.Optics(LAM, PITCH, PITCH, z, pipeline.AS))
    err = rel_l2(u.cpu().numpy(), ref)
    assert np.all(np.isfinite(u.cpu().numpy()))
    return err


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dtype,value,side", [(np.uint8, 255, 256), (np.uint16, 4095, 1024),
                                              (np.uint16, 65535, 1024), (np.uint16, 65535, 256)])
def test_constant_full_scale(ctx, hv, dtype, value, side, prec):
    say(f"constant {value} {dtype.__name__} {side}^2 prec={prec}")
    frames = np.full((2, side, side), value, np.float64)
    err = _as_field_case(ctx, hv, frames, dtype, -0.2, prec)
    say(f"  field rel-L2 {err:.2e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dtype,maxv,side", [(np.uint8, 255, 512), (np.uint16, 65535, 1024)])
def test_plane_wave_full_scale(ctx, hv, dtype, maxv, side, prec):
    say(f"plane wave {maxv} {side}^2 prec={prec}")
    y, x = np.mgrid[0:side, 0:side]
    frames = np.rint(maxv / 2.0 * (1.0 + np.cos(2 * np.pi * (37 * x + 11 * y) / side)))[None]
    err = _as_field_case(ctx, hv, frames, dtype, -0.3, prec)
    say(f"  field rel-L2 {err:.2e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dtype,maxv,side", [(np.uint8, 255, 512), (np.uint16, 4095, 1024),
                                              (np.uint16, 65535, 1024)])
def test_point_hologram_full_scale(ctx, hv, dtype, maxv, side, prec):
    say(f"point hologram {maxv} {side}^2 prec={prec}")
    frames = _zone_plate(side, side, 0.5, maxv)[None]
    err = _as_field_case(ctx, hv, frames, dtype, -0.5, prec)
    say(f"  field rel-L2 {err:.2e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("dtype,maxv", [(np.uint8, 255), (np.uint16, 65535)])
def test_point_hologram_moments_full_scale(ctx, hv, dtype, maxv, order, prec):
    """32 frames of a full-scale point-source hologram whose object phase
    advances 2 pi * 5/32 per frame (a Doppler tone in bin 5), 512^2, both
    orders of the moments path."""
    say(f"point hologram moments {maxv} order={order} prec={prec}")
    w, side, fs = 32, 512, 32e3
    frames = np.stack([_zone_plate(side, side, 0.4, maxv, 2 * np.pi * 5 * t / w) for t in range(w)]).astype(dtype)
    opt = hv.Optics(LAM, PITCH, PITCH, -0.4, hv.HV_AS)
    tp = hv.Temporal(w, w, fs, 2 * fs / w, 15 * fs / w)
    ctx.set_stft_order(order)
    try:
        m = [t.cpu().numpy() for t in ctx.hv_stft_moments(torch.from_numpy(frames).cuda(), opt, tp, prec)]
    finally:
        ctx.set_stft_order(hv.HV_ORDER_FRAMES_FIRST)
    ref = pipeline.stft_moments(frames, pipeline.Optics(LAM, PITCH, PITCH, -0.4, pipeline.AS), w, w, fs,
                                2 * fs / w, 15 * fs / w)
    for i, k in enumerate(("m0", "m1", "m2")):
        err = rel_l2(m[i], ref[k])
        say(f"  {k} rel-L2 {err:.2e}")
        assert np.all(np.isfinite(m[i]))
        assert err < TOL[prec]
