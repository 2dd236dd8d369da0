"""The paper's non-power-of-two Table IV frame sides (1280 x 800, 512 x 320,
384 x 384) through the mixed-radix (3, 5) FFT passes, against the FP64
oracle through the C-ABI."""

import numpy as np
import pytest
import torch

from oracle import optics as oopt
from oracle import pca as opca
from oracle import pipeline, temporal as otemp
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu

LAM = 852e-9
TOL = {0: 1e-5, 1: 2e-3}
SHAPES = [(800, 1280), (320, 512), (384, 384)]


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx(hv):
    c = hv.Context(0)
    yield c
    c.close()


def frames(seed, n, ny, nx):
    return np.random.default_rng(seed).integers(0, 256, (n, ny, nx)).astype(np.uint8)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_propagate_as_and_fresnel(ctx, hv, prec, shape):
    ny, nx = shape
    say(f"propagate {ny}x{nx} prec={prec}")
    x = frames(ny + nx, 2, ny, nx)
    xd = torch.from_numpy(x).cuda()
    for method, z in ((hv.HV_AS, -0.15), (hv.HV_FRESNEL, 0.4)):
        opt = hv.Optics(LAM, 20e-6, 20e-6, z, method)
        got = ctx.hv_propagate(xd, opt, prec).cpu().numpy()
        ref = pipeline.reconstruct(x, pipeline.Optics(LAM, 20e-6, 20e-6, z, method))
        err = rel_l2(got, ref)
        say(f"  method {method}: rel-L2 {err:.3e}")
        assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_moments_384(ctx, hv, prec):
    say(f"moments 384x384 W=32 prec={prec}")
    x = frames(5, 70, 384, 384)
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.2, hv.HV_AS)
    tp = hv.Temporal(32, 32, 20e3, 1.5e3, 9e3)
    m = [t.cpu().numpy() for t in ctx.hv_stft_moments(torch.from_numpy(x).cuda(), opt, tp, prec)]
    ref = pipeline.stft_moments(x, pipeline.Optics(LAM, 20e-6, 20e-6, -0.2), 32, 32, 20e3, 1.5e3, 9e3)
    for i, k in enumerate(("m0", "m1", "m2")):
        assert rel_l2(m[i], ref[k]) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_pca_fresnel_320x512(ctx, hv, prec):
    say(f"PCA Fresnel 320x512 W=16 prec={prec}")
    x = frames(6, 32, 320, 512)
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.3, hv.HV_FRESNEL)
    r = ctx.hv_pca(torch.from_numpy(x).cuda(), opt, 16, 16, 1, 15, prec, want_cov=True)
    u = pipeline.reconstruct(x, pipeline.Optics(LAM, 20e-6, 20e-6, 0.3, pipeline.FRESNEL))
    for j in range(2):
        pr = opca.pca_window(u[16 * j:16 * (j + 1)], 1, 15)
        for k, got in (("cov", r["cov"][j]), ("eigvals", r["eigvals"][j]), ("m0", r["m0"][j])):
            assert rel_l2(got.cpu().numpy(), pr[k]) < TOL[prec], (j, k)


@pytest.mark.parametrize("prec", [0, 1])
def test_volume_1280x800(ctx, hv, prec):
    say(f"volume 800x1280 W=128 high-pass prec={prec}")
    x = frames(7, 128, 800, 1280)
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.2, hv.HV_AS, 0.05)
    got = ctx.hv_stft_volume(torch.from_numpy(x).cuda(), opt, 128, 128, prec).cpu().numpy()
    u = oopt.angular_spectrum(x.astype(np.float64), LAM, 20e-6, 20e-6, -0.2, 0.05)
    rng = np.random.default_rng(2)
    ys, xs = rng.integers(0, 800, 32), rng.integers(0, 1280, 32)
    ref = np.abs(otemp.dft_matrix(128) @ u[:, ys, xs]) ** 2
    assert rel_l2(got[0][:, ys, xs], ref) < TOL[prec]
