"""Post-processing through the C-ABI against the FP64 oracle."""

import numpy as np
import pytest
import torch

from oracle import post
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hv):
    c = hv.Context(0)
    yield c
    c.close()


def images(seed, count, ny, nx, moves):
    rng = np.random.default_rng(seed)
    base = rng.uniform(1, 2, (ny, nx))
    base[ny // 3: ny // 2, nx // 4: nx // 3] += 3.0  # a feature that gives a clear correlation peak
    return np.stack([np.roll(base, m, axis=(0, 1)) + 0.01 * rng.standard_normal((ny, nx)) for m in moves[:count]])


def test_convolution_and_renormalisation(ctx, hv):
    x = np.random.default_rng(1).uniform(0.5, 2.0, (5, 64, 96)).astype(np.float32)
    k = post.gaussian_kernel(1.5).astype(np.float32)
    got, _ = ctx.hv_postprocess(torch.from_numpy(x).cuda(), kernel=k, renormalise=True)
    ref, _ = post.postprocess(x, kernel=k.astype(np.float64), renorm=True)
    assert rel_l2(got.cpu().numpy(), ref) < 1e-5
    k3 = np.arange(9, dtype=np.float32).reshape(3, 3)  # not symmetric: checks the kernel orientation
    got, _ = ctx.hv_postprocess(torch.from_numpy(x).cuda(), kernel=k3)
    assert rel_l2(got.cpu().numpy(), post.convolve(x, k3)) < 1e-6


@pytest.mark.parametrize("shape", [(128, 128), (64, 256), (320, 512)])
def test_registration_and_accumulation(ctx, hv, shape):
    ny, nx = shape
    moves = [(0, 0), (3, -5), (-7, 11), (15, 2), (-2, -9), (6, 6)]
    x = images(2, 6, ny, nx, moves).astype(np.float32)
    got, sh = ctx.hv_postprocess(torch.from_numpy(x).cuda(), ref_count=2, mask_radius=0.9, accumulate=3)
    ref, rsh = post.postprocess(x, ref_count=2, mask_radius=0.9, accumulate_length=3)
    assert np.array_equal(sh.cpu().numpy(), rsh.astype(np.int32))
    assert rel_l2(got.cpu().numpy(), ref) < 1e-6


def test_full_chain(ctx, hv):
    moves = [(0, 0), (2, 3), (-4, 1), (5, -6)]
    x = images(3, 4, 128, 128, moves).astype(np.float32)
    k = post.gaussian_kernel(1.0).astype(np.float32)
    got, sh = ctx.hv_postprocess(torch.from_numpy(x).cuda(), kernel=k, renormalise=True, ref_count=1,
                                 mask_radius=0.8, accumulate=2)
    ref, rsh = post.postprocess(x, kernel=k.astype(np.float64), renorm=True, ref_count=1, mask_radius=0.8,
                                accumulate_length=2)
    assert np.array_equal(sh.cpu().numpy(), rsh.astype(np.int32))
    assert rel_l2(got.cpu().numpy(), ref) < 1e-5


def test_bad_arguments(ctx, hv):
    x = torch.zeros((2, 64, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(hv.HvError):
        ctx.hv_postprocess(x, kernel=np.ones((4, 4), np.float32))  # even size
    with pytest.raises(hv.HvError):
        ctx.hv_postprocess(x, ref_count=3)                           # more references than images
