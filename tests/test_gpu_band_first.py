"""Band-first order of the AS moments path vs the FP64 oracle, through the C-ABI.

The library may form each band bin from the raw frames of a window and then
propagate the bins (the propagation and the temporal combination are both
linear); the oracle always propagates every frame first.  These tests force
that order, check which kernels ran, and compare element by element:
rel-L2 below 1e-5 (FP32 form) and 2e-3 (mixed form) over each output.
Inputs are seeded and synthetic.
"""

import numpy as np
import pytest
import torch

from oracle import pipeline
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def frames(seed, n, ny, nx, dtype):
    rng = np.random.default_rng(seed)
    hi = 256 if dtype == np.uint8 else 4096
    return rng.integers(0, hi, (n, ny, nx)).astype(dtype)


def oracle(x, opt, tp, keep=False):
    o = pipeline.Optics(opt.wavelength, opt.pitch_x, opt.pitch_y, opt.z, opt.method, opt.highpass)
    return pipeline.stft_moments(x, o, tp.window, tp.stride, tp.fs, tp.f_lo, tp.f_hi, tp.symmetric, keep)


def run(ctx, hv, order, fn, chunk=0):
    """fn() under the given order with kernel timing on; returns (result,
    launches of band_rows, launches of the frames-first temporal kernels)."""
    ctx.set_stft_order(order)
    ctx.set_chunk_frames(chunk)
    ctx.set_timing(True)
    try:
        out = fn()
        torch.cuda.synchronize()
        band = ctx.kernel_time("band_rows")[1]
        frames_first = ctx.kernel_time("rowinv_coef")[1] + ctx.kernel_time("field_coef")[1]
    finally:
        ctx.set_timing(False)
        ctx.set_chunk_frames(0)
        ctx.set_stft_order(hv.HV_ORDER_FRAMES_FIRST)
    return out, band, frames_first


# (n, ny, nx, dtype, window, stride, fs, f_lo, f_hi, symmetric, highpass, chunk)
CASES = [
    # headline shape: 3 windows + 5 ragged frames, two chunks of 2 and 1 windows
    (101, 256, 256, np.uint8, 32, 32, 71.4e3, 3e3, 35e3, False, 0.0, 64),
    # overlapping windows, u16, two-sided band
    (40, 128, 256, np.uint16, 16, 8, 20e3, 1.5e3, 9e3, True, 0.0, 0),
    # 33 bins: three 16-bin tiles, the last one ragged; mixed-radix columns
    (64, 320, 256, np.uint8, 64, 64, 40e3, 0.0, 20e3, False, 0.0, 0),
    # W = 8 (half of each MFMA k-step is padding), 512-wide rows, high-pass
    (30, 64, 512, np.uint8, 8, 4, 10e3, 1e3, 4e3, False, 0.05, 0),
    # u16 with W = 64 and 384-row columns
    (70, 384, 256, np.uint16, 64, 64, 64e3, 5e3, 20e3, False, 0.0, 0),
    # one-wave rows (nx = 64)
    (50, 128, 64, np.uint8, 16, 16, 20e3, 2e3, 8e3, False, 0.0, 0),
    # two-wave rows (nx = 128), u16, two-sided band, high-pass, stride 8
    (40, 64, 128, np.uint16, 32, 8, 30e3, 1e3, 14e3, True, 0.02, 0),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_band_first_moments(ctx, hv, case, prec):
    n, ny, nx, dt, w, s, fs, lo, hi, sym, hp, chunk = CASES[case]
    say(f"band-first moments case {case}: {n}x{ny}x{nx} {dt.__name__} W={w} s={s} prec={prec}")
    x = frames(20 + case, n, ny, nx, dt)
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.21, hv.HV_AS, highpass=hp)
    tp = hv.Temporal(w, s, fs, lo, hi, symmetric=sym)
    m, band, ff = run(ctx, hv, hv.HV_ORDER_BAND_FIRST,
                      lambda: [host(t) for t in ctx.hv_stft_moments(dev(x), opt, tp, prec)], chunk)
    assert band > 0 and ff == 0
    ref = oracle(x, opt, tp)
    assert m[0].shape == ref["m0"].shape
    for i, k in enumerate(("m0", "m1", "m2")):
        err = rel_l2(m[i], ref[k])
        say(f"  {k} rel-L2 {err:.3e}")
        assert err < TOL[prec], (k, err)


@pytest.mark.parametrize("prec", [0, 1])
def test_band_first_bins(ctx, hv, prec):
    say(f"band-first spectrum bins prec={prec}")
    x = frames(31, 70, 256, 256, np.uint8)
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.15, hv.HV_AS)
    tp = hv.Temporal(32, 16, 50e3, 4e3, 20e3)
    s, band, ff = run(ctx, hv, hv.HV_ORDER_BAND_FIRST, lambda: host(ctx.hv_stft_bins(dev(x), opt, tp, prec)))
    assert band > 0 and ff == 0
    ref = oracle(x, opt, tp, keep=True)
    bins = ref["bins"]
    assert s.shape == (3, len(bins), 256, 256)
    assert rel_l2(s, ref["spectrum"][:, bins]) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_orders_agree(ctx, hv, prec):
    say(f"band-first vs frames-first prec={prec}")
    x = frames(32, 96, 256, 256, np.uint8)
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.24, hv.HV_AS)
    tp = hv.Temporal(32, 32, 71.4e3, 3e3, 35e3)
    xd = dev(x)
    a, band, ff = run(ctx, hv, hv.HV_ORDER_BAND_FIRST, lambda: [host(t) for t in ctx.hv_stft_moments(xd, opt, tp, prec)])
    assert band > 0 and ff == 0
    b, band, ff = run(ctx, hv, hv.HV_ORDER_FRAMES_FIRST, lambda: [host(t) for t in ctx.hv_stft_moments(xd, opt, tp, prec)])
    assert band == 0 and ff > 0
    for u, v in zip(a, b):
        assert rel_l2(u, v) < 2 * TOL[prec]


def test_auto_order_choice(ctx, hv):
    """AUTO takes band first for the 14-bin, W = 32, stride 32 window of the
    256 x 256 stream, and frames first for a full band at stride 1."""
    say("automatic order choice")
    x = dev(frames(33, 64, 256, 256, np.uint8))
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.24, hv.HV_AS)
    tp = hv.Temporal(32, 32, 71.4e3, 3e3, 35e3)
    _, band, ff = run(ctx, hv, hv.HV_ORDER_AUTO, lambda: ctx.hv_stft_moments(x, opt, tp, 0))
    assert band > 0 and ff == 0
    tp_full = hv.Temporal(16, 1, 20e3, 0.0, 10e3, symmetric=True)
    _, band, ff = run(ctx, hv, hv.HV_ORDER_AUTO, lambda: ctx.hv_stft_moments(x[:24], opt, tp_full, 0))
    assert band == 0 and ff > 0


def test_band_first_deterministic(ctx, hv):
    say("band-first bitwise determinism and chunking")
    x = dev(frames(34, 160, 256, 256, np.uint8))
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.24, hv.HV_AS)
    tp = hv.Temporal(32, 32, 71.4e3, 3e3, 35e3)
    a, _, _ = run(ctx, hv, hv.HV_ORDER_BAND_FIRST, lambda: [host(t) for t in ctx.hv_stft_moments(x, opt, tp, 0)])
    b, _, _ = run(ctx, hv, hv.HV_ORDER_BAND_FIRST, lambda: [host(t) for t in ctx.hv_stft_moments(x, opt, tp, 0)], 64)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_order_knob_errors(ctx, hv):
    with pytest.raises(hv.HvError):
        ctx.set_stft_order(7)
