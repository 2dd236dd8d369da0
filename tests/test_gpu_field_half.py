"""hv_propagate with an fp16 complex field out (HV_C32H) against the FP64
oracle, through the C-ABI.

The fp16 field holds U * field_scale(in_t, ny, nx), a power of two.  The
output is stored in fp16, so the mixed form's tolerance (2e-3 rel-L2)
applies to both precision forms; the field is also checked against the
float32 field of the same call at the rounding of fp16 (rel-L2 below 1e-3:
half an fp16 ulp is 2^-11 of a value), and must be finite at full-scale
coherent input, where the scale is chosen to keep it in range.
"""

import numpy as np
import pytest
import torch

from oracle import pipeline
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu

LAM = 852e-9
TOL_HALF = 2e-3


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx(hv):
    c = hv.Context(0)
    yield c
    c.close()


def _half_to_complex(t):
    a = t.float().cpu().numpy()
    return a[..., 0].astype(np.float64) + 1j * a[..., 1]


def _case(ctx, hv, x, method, z, prec, dx=20e-6, dy=20e-6):
    opt = hv.Optics(LAM, dx, dy, z, method)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    h = ctx.hv_propagate(xd, opt, prec, out_dtype=hv.HV_C32H)
    f = ctx.hv_propagate(xd, opt, prec)
    torch.cuda.synchronize()
    in_t = {np.uint8: hv.HV_U8, np.uint16: hv.HV_U16, np.complex64: hv.HV_C64}[x.dtype.type]
    scale = hv.field_scale(in_t, x.shape[1], x.shape[2])
    assert h.dtype == torch.float16 and tuple(h.shape) == x.shape + (2,)
    assert torch.isfinite(h).all().item()
    u = _half_to_complex(h) / scale
    ref = pipeline.reconstruct(x, pipeline.Optics(LAM, dx, dy, z, method))
    e_ref = rel_l2(u, ref)
    e_f32 = rel_l2(u, f.cpu().numpy())
    say(f"  scale {scale}  vs oracle {e_ref:.2e}  vs float32 field {e_f32:.2e}")
    assert e_ref < TOL_HALF
    assert e_f32 < 1e-3
    return u


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,dtype", [((2, 256, 256), np.uint8), ((1, 1024, 1024), np.uint16),
                                         ((2, 320, 512), np.uint8), ((3, 128, 64), np.uint16)])
def test_half_field_as(ctx, hv, shape, dtype, prec):
    say(f"AS C32H {shape} {dtype.__name__} prec={prec}")
    rng = np.random.default_rng(11)
    x = rng.integers(0, 256 if dtype == np.uint8 else 4096, shape).astype(dtype)
    _case(ctx, hv, x, hv.HV_AS, -0.17, prec, 20e-6, 15e-6)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("z", [0.5, -0.5])
@pytest.mark.parametrize("shape,dtype", [((2, 256, 256), np.uint8), ((1, 1024, 1024), np.uint16)])
def test_half_field_fresnel(ctx, hv, shape, dtype, z, prec):
    say(f"Fresnel C32H {shape} {dtype.__name__} z={z} prec={prec}")
    rng = np.random.default_rng(12)
    x = rng.integers(0, 256 if dtype == np.uint8 else 4096, shape).astype(dtype)
    _case(ctx, hv, x, hv.HV_FRESNEL, z, prec, 20e-6, 25e-6)


def test_half_field_complex_input(ctx, hv):
    say("AS C32H complex input")
    rng = np.random.default_rng(13)
    x = (100 * (rng.standard_normal((2, 128, 256)) + 1j * rng.standard_normal((2, 128, 256)))).astype(np.complex64)
    _case(ctx, hv, x, hv.HV_AS, 0.3, 0)


@pytest.mark.parametrize("prec", [0, 1])
def test_half_field_full_scale(ctx, hv, prec):
    # constant 65535 frames put all the energy in one value per pixel, and a
    # full-scale off-axis point hologram focuses its +1 order to a spot at z
    say(f"C32H full scale prec={prec}")
    x = np.full((1, 1024, 1024), 65535, np.uint16)
    u = _case(ctx, hv, x, hv.HV_AS, -0.2, prec)
    assert abs(np.abs(u).max() / 65535 - 1) < 2e-3
    n, pitch, z = 512, 20e-6, 0.15
    y, xx = np.mgrid[0:n, 0:n]
    chirp = np.pi * (((xx - n / 2) * pitch) ** 2 + ((y - n / 2) * pitch) ** 2) / (LAM * z)
    holo = np.rint(127.5 * (1 + np.cos(np.pi * (xx + y) / 2 - chirp)))[None].astype(np.uint8)
    u = _case(ctx, hv, holo, hv.HV_AS, -z, prec, pitch, pitch)
    say(f"  focused peak |U| {np.abs(u).max():.0f}")


def test_half_field_chunks_and_edges(ctx, hv):
    # several chunks per call (offsets into the fp16 output), the empty call
    # and an output type that is not a field
    say("C32H chunked, empty, bad out_t")
    rng = np.random.default_rng(14)
    x = rng.integers(0, 256, (7, 128, 128)).astype(np.uint8)
    ctx.set_chunk_frames(3)
    try:
        for prec in (0, 1):
            _case(ctx, hv, x, hv.HV_AS, 0.1, prec)
            _case(ctx, hv, x, hv.HV_FRESNEL, 0.4, prec)
    finally:
        ctx.set_chunk_frames(0)
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.1, hv.HV_AS)
    empty = ctx.hv_propagate(torch.zeros((0, 64, 64), dtype=torch.uint8, device="cuda"), opt,
                             out_dtype=hv.HV_C32H)
    assert tuple(empty.shape) == (0, 64, 64, 2)
    xd = torch.from_numpy(x).cuda()
    with pytest.raises(hv.HvError) as e:
        ctx.hv_propagate(xd, opt, out=torch.empty((7, 128, 128, 2), dtype=torch.float16, device="cuda"),
                         out_dtype=hv.HV_U8)
    assert e.value.status == hv.HV_ERR_ARG
