"""Moments from pinned host frames into pinned host images (the camera-side
path across PCIe) equal the device-resident call bit for bit."""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

LAM = 852e-9


@pytest.fixture(scope="module")
def ctx(hv):
    c = hv.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("window,stride", [(32, 32), (16, 12)])
def test_host_ingest_matches_device_call(ctx, hv, prec, window, stride):
    print(f"host ingest W={window} s={stride} prec={prec}", flush=True)
    rng = np.random.default_rng(21)
    x = rng.integers(0, 256, (1100, 128, 128)).astype(np.uint8)
    xh = torch.from_numpy(x).pin_memory()
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.2, hv.HV_AS)
    tp = hv.Temporal(window, stride, 20e3, 1.5e3, 9e3)
    got = ctx.hv_stft_moments_host(xh, opt, tp, prec)
    torch.cuda.current_stream().synchronize()
    want = ctx.hv_stft_moments(xh.cuda(), opt, tp, prec)
    for g, w in zip(got, want):
        assert g.shape == w.shape
        assert torch.equal(g, w.cpu())


def test_host_ingest_rejects_field_input(ctx, hv):
    u = torch.zeros((64, 64, 64), dtype=torch.complex64).pin_memory()
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.2, hv.HV_AS)
    tp = hv.Temporal(32, 32, 20e3, 1.5e3, 9e3)
    with pytest.raises(hv.HvError):
        ctx.hv_stft_moments_host(u, opt, tp)
