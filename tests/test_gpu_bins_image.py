"""Magnitude and argument images over a range of temporal indices
(Sec. III-B.1) through the C-ABI against the FP64 oracle.

The argument is compared as the phasor |sum_k S_k| exp(i arg) against
sum_k S_k (rel-L2), so pixels where the sum nearly cancels, and its angle is
ill-conditioned, weigh by their modulus.  Inputs are seeded and synthetic.
"""

import numpy as np
import pytest
import torch

from oracle import pipeline, post
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx(hv):
    c = hv.Context(0)
    yield c
    c.close()


def images(ctx, hv, spec):
    mag = ctx.hv_bins_image(spec, hv.HV_IMG_MAGNITUDE)
    arg = ctx.hv_bins_image(spec, hv.HV_IMG_ARGUMENT)
    torch.cuda.synchronize()
    return mag.cpu().numpy().astype(np.float64), arg.cpu().numpy().astype(np.float64)


# (windows, bins, ny, nx): several bins; a one-bin range; a ragged pixel count
SHAPES = [(3, 14, 64, 96), (2, 1, 128, 128), (1, 33, 40, 56)]


@pytest.mark.parametrize("shape", SHAPES)
def test_bins_image_matches_oracle(ctx, hv, shape):
    say(f"bins image of a random spectrum {shape}")
    rng = np.random.default_rng(7)
    s = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    mag, arg = images(ctx, hv, torch.from_numpy(s).cuda())
    s64 = s.astype(np.complex128)
    assert rel_l2(mag, post.magnitude_image(s64)) < 2e-6
    total = s64.sum(axis=1)
    assert np.all(np.abs(arg) <= np.pi + 1e-6)
    assert rel_l2(np.abs(total) * np.exp(1j * arg), total) < 2e-6
    assert rel_l2(np.exp(1j * arg), np.exp(1j * post.argument_image(s64))) < 1e-4


def test_bins_image_after_stft_bins(ctx, hv):
    say("bins image after hv_stft_bins, 70 frames of 128x128 u8")
    x = np.random.default_rng(8).integers(0, 256, (70, 128, 128)).astype(np.uint8)
    opt = hv.Optics(852e-9, 20e-6, 20e-6, -0.21, hv.HV_AS)
    tp = hv.Temporal(32, 16, 50e3, 4e3, 20e3)
    spec = ctx.hv_stft_bins(torch.from_numpy(x).cuda(), opt, tp, hv.HV_PREC_FP32)
    mag, arg = images(ctx, hv, spec)
    o = pipeline.Optics(opt.wavelength, opt.pitch_x, opt.pitch_y, opt.z, opt.method, opt.highpass)
    ref = pipeline.stft_moments(x, o, tp.window, tp.stride, tp.fs, tp.f_lo, tp.f_hi, tp.symmetric, True)
    sb = ref["spectrum"][:, ref["bins"]]
    assert mag.shape == (3, 128, 128)
    assert rel_l2(mag, post.magnitude_image(sb)) < 1e-5
    total = sb.sum(axis=1)
    assert rel_l2(np.abs(total) * np.exp(1j * arg), total) < 1e-5


def test_bins_image_errors(ctx, hv):
    s = torch.zeros((1, 2, 16, 16), dtype=torch.complex64, device="cuda")
    with pytest.raises(hv.HvError):
        ctx.hv_bins_image(s, 5)
