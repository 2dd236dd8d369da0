"""The entry point that allocates nothing (hv_stft_moments_noalloc) against
hv_stft_moments on the same inputs, through the C-ABI: two calls in a row,
the second with fewer frames, for the fused angular-spectrum path (several
chunks of the fixed scratch), the Fresnel path (field workspace) and both
precision forms; plus its refusals (no plan in the context, a window larger
than the scratch)."""

import numpy as np
import pytest
import torch

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


def _frames(seed, n, ny, nx, dtype):
    rng = np.random.default_rng(seed)
    hi = 256 if dtype == np.uint8 else 4096
    return torch.from_numpy(rng.integers(0, hi, (n, ny, nx)).astype(dtype)).cuda()


def _rel(a, b):
    a = a.double()
    b = b.double()
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("method,shape,dtype,window,stride,counts", [
    (0, (256, 256), np.uint8, 32, 32, (720, 100)),   # fused row inverse + GEMM; 3 chunks FP32, then 1
    (1, (256, 512), np.uint16, 16, 8, (200, 40)),    # Fresnel: field workspace, overlapping windows
])
def test_noalloc_equals_allocating_call(ctx, hv, method, shape, dtype, window, stride, counts, prec):
    ny, nx = shape
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.3, method)
    tp = hv.Temporal(window, stride, 20e3, 2e3, 9e3)
    for call, n in enumerate(counts):
        say(f"no-alloc method={method} {nx}x{ny} W={window} s={stride} n={n} prec={prec} call {call}")
        x = _frames(100 + call, n, ny, nx, dtype)
        ref = ctx.hv_stft_moments(x, opt, tp, prec)  # also builds the plans the no-alloc call needs
        j = ref[0].shape[0]
        out = [torch.full((j, ny, nx), float("nan"), dtype=torch.float32, device="cuda") for _ in range(3)]
        ctx.hv_stft_moments_noalloc(x, opt, tp, prec, out)
        torch.cuda.synchronize()
        for k in range(3):
            err = _rel(out[k], ref[k])
            assert err < TOL[prec], (k, err)
            assert torch.equal(out[k], ref[k]), k  # the same kernels on the same windows


def test_noalloc_refusals(hv):
    say("no-alloc refusals")
    c = hv.Context(0)
    try:
        opt = hv.Optics(LAM, 20e-6, 20e-6, -0.21)
        tp = hv.Temporal(32, 32, 20e3, 2e3, 9e3)
        x = _frames(7, 64, 128, 128, np.uint8)
        out = [torch.empty((2, 128, 128), dtype=torch.float32, device="cuda") for _ in range(3)]
        with pytest.raises(hv.HvError) as e:  # no plan yet: nothing is built here
            c.hv_stft_moments_noalloc(x, opt, tp, 0, out)
        assert e.value.status == hv.HV_ERR_STATE
        big = _frames(8, 64, 1024, 1024, np.uint16)
        tp64 = hv.Temporal(64, 64, 20e3, 2e3, 9e3)
        c.hv_stft_moments(big, opt, tp64, 0)  # plans exist now
        ob = [torch.empty((1, 1024, 1024), dtype=torch.float32, device="cuda") for _ in range(3)]
        with pytest.raises(hv.HvError) as e:  # one window needs 768 MiB of workspace
            c.hv_stft_moments_noalloc(big, opt, tp64, 0, ob)
        assert e.value.status == hv.HV_ERR_SHAPE
        assert "scratch" in str(e.value)
    finally:
        c.close()
