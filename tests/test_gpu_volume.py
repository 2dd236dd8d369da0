"""The full-band STFT volume (angular spectrum + spatial high-pass filter +
temporal FFT over whole windows) through the C-ABI against the FP64 oracle."""

import numpy as np
import pytest
import torch

from oracle import optics as oopt
from oracle import pipeline, temporal as otemp
from synth import holograms
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu

LAM = 852e-9
TOL = {0: 1e-5, 1: 2e-3}


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx(hv):
    c = hv.Context(0)
    yield c
    c.close()


def rand_frames(seed, n, ny, nx, dtype):
    rng = np.random.default_rng(seed)
    hi = 255 if dtype == np.uint8 else 4095
    return rng.integers(0, hi + 1, (n, ny, nx)).astype(dtype)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("window,stride,n,shape,hp", [
    (128, 128, 3 * 128, (64, 128), 0.05),
    (256, 96, 256 + 2 * 96 + 40, (64, 64), 0.1),    # overlapping windows, ragged tail
    (512, 512, 2 * 512 + 17, (64, 64), 0.02),
])
def test_volume_matches_oracle(ctx, hv, prec, window, stride, n, shape, hp):
    say(f"volume W={window} s={stride} n={n} {shape} hp={hp} prec={prec}")
    x = rand_frames(window + n, n, *shape, np.uint8)
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.2, hv.HV_AS, hp)
    got = ctx.hv_stft_volume(torch.from_numpy(x).cuda(), opt, window, stride, prec).cpu().numpy()
    ref = pipeline.stft_volume(x, pipeline.Optics(LAM, 20e-6, 20e-6, -0.2, pipeline.AS, hp), window, stride)
    assert got.shape == ref.shape
    err = rel_l2(got, ref)
    say(f"  rel-L2 {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_volume_field_input(ctx, hv, prec):
    say(f"volume from a field, prec={prec}")
    rng = np.random.default_rng(3)
    u = (rng.standard_normal((300, 64, 64)) + 1j * rng.standard_normal((300, 64, 64))).astype(np.complex64)
    got = ctx.hv_stft_volume(torch.from_numpy(u).cuda(), None, 256, 32, prec).cpu().numpy()
    ref = pipeline.stft_volume(u, None, 256, 32)
    assert rel_l2(got, ref) < 1e-5  # the field is read as it is in both forms


def test_volume_rejects_bad_arguments(ctx, hv):
    x = torch.zeros((200, 64, 64), dtype=torch.uint8, device="cuda")
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.2, hv.HV_AS, 0.05)
    with pytest.raises(hv.HvError):
        ctx.hv_stft_volume(x, opt, 100, 100)          # unsupported window
    with pytest.raises(hv.HvError):
        ctx.hv_stft_volume(x, opt, 256, 256)          # no complete window
    fr = hv.Optics(LAM, 20e-6, 20e-6, 0.2, hv.HV_FRESNEL, 0.05)
    with pytest.raises(hv.HvError):
        ctx.hv_stft_volume(x, fr, 128, 128)           # high-pass is an AS-path filter


@pytest.mark.parametrize("prec", [0, 1])
def test_volume_full_size_sampled(ctx, hv, prec):
    """256x256 u8 at W = 512, stride 512 (the benchmark's configuration):
    every bin of 24 sampled pixels against the oracle, computed for those
    pixels only (the spatial transform is per frame, the temporal one per
    pixel)."""
    say(f"volume 256x256 W=512 sampled, prec={prec}")
    block, spec = holograms.config_c2_block(1024)
    hp = 0.05
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS, hp)
    got = ctx.hv_stft_volume(torch.from_numpy(block).cuda(), opt, 512, 512, prec).cpu().numpy()
    u = oopt.angular_spectrum(block.astype(np.float64), LAM, spec.pitch, spec.pitch, -spec.z, hp)
    rng = np.random.default_rng(8)
    ys, xs = rng.integers(0, 256, 24), rng.integers(0, 256, 24)
    d = otemp.dft_matrix(512)
    for j in range(2):
        s = d @ u[j * 512:(j + 1) * 512, ys, xs]
        ref = np.abs(s) ** 2
        err = rel_l2(got[j][:, ys, xs], ref)
        say(f"  window {j}: rel-L2 {err:.3e}")
        assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("in_t", [np.uint8, np.complex64])
def test_propagate_with_highpass(ctx, hv, prec, in_t):
    say(f"propagate with high-pass, {np.dtype(in_t).name}, prec={prec}")
    rng = np.random.default_rng(11)
    if in_t == np.uint8:
        x = rand_frames(12, 3, 64, 128, np.uint8)
    else:
        x = (rng.standard_normal((3, 64, 128)) + 1j * rng.standard_normal((3, 64, 128))).astype(np.complex64)
    opt = hv.Optics(LAM, 20e-6, 15e-6, -0.15, hv.HV_AS, 0.08)
    got = ctx.hv_propagate(torch.from_numpy(x).cuda(), opt, prec).cpu().numpy()
    ref = oopt.angular_spectrum(x.astype(np.complex128), LAM, 20e-6, 15e-6, -0.15, 0.08)
    assert rel_l2(got, ref) < TOL[prec]
