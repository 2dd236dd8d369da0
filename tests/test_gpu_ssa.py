"""SSA + FFT (hv_ssa_moments) against the FP64 oracle through the C-ABI:
random frames and holograms, both propagation methods, windows 16/32/64,
overlapping windows with a ragged tail, the closed-form background-plus-tones
case, the full component range against the plain STFT, and the 1024^2
12-bit Fresnel precision shape.  Tolerances: 1e-5 (FP32 form), 2e-3 (mixed)."""

import numpy as np
import pytest
import torch

from oracle import optics as oopt
from oracle import pipeline, ssa as ossa
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _oracle(frames, opt, tp, c1, c2):
    o = None if opt is None else pipeline.Optics(opt.wavelength, opt.pitch_x, opt.pitch_y, opt.z, opt.method)
    return pipeline.ssa_render(frames, o, tp.window, tp.stride, tp.fs, tp.f_lo, tp.f_hi, c1, c2, tp.symmetric)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("method,window,stride,comps", [(0, 16, 16, (1, 15)), (1, 32, 24, (1, 31)),
                                                         (0, 64, 64, (1, 63)), (1, 16, 16, (0, 15))])
def test_ssa_random_frames(ctx, hv, method, window, stride, comps, prec):
    """Random frames: one dominant (static) component above a cluster of
    nearly equal noise eigenvalues, so the ranges that end at a spectral gap
    (everything but the static part, or everything) are the well-conditioned
    ones; a range ending inside the cluster would depend on eigenvectors
    that rounding can rotate among themselves, and the static part alone has
    almost no power outside the zero-frequency bin."""
    say(f"SSA random method={method} W={window} s={stride} comps={comps} prec={prec}")
    rng = np.random.default_rng(31)
    n = 2 * window + 7
    x = rng.integers(0, 256, (n, 128, 64)).astype(np.uint8) if method == 0 else \
        rng.integers(0, 4096, (n, 64, 128)).astype(np.uint16)
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.4, method)
    fs = 20e3
    # the static component alone is rendered with its own (zero-frequency)
    # bin in the band: outside it, its power is the small remainder of an
    # eigenvector that is only nearly constant in time
    f_lo = 0.0 if comps[0] == 0 else 2 * fs / window
    tp = hv.Temporal(window, stride, fs, f_lo, 0.45 * fs)
    r = ctx.hv_ssa_moments(dev(x), opt, tp, comps[0], comps[1], prec)
    ref = _oracle(x, opt, tp, *comps)
    assert host(r["offdiag"]).max() < 1e-14
    assert rel_l2(host(r["eigvals"]), ref["eigvals"]) < TOL[prec]
    for k in ("m0", "m1", "m2"):
        err = rel_l2(host(r[k]), ref[k])
        say(f"  {k} rel-L2 {err:.2e}")
        assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_ssa_holograms_symmetric_band(ctx, hv, prec):
    say(f"SSA holograms symmetric band prec={prec}")
    spec = holograms.HoloSpec(frames=70, ny=128, nx=128, z=0.2, fs=33e3, seed=3)
    x = holograms.hologram_stack(spec)
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(32, 16, spec.fs, 2e3, 8e3, True)
    r = ctx.hv_ssa_moments(dev(x), opt, tp, 1, 31, prec)
    ref = _oracle(x, opt, tp, 1, 31)
    for k in ("m0", "m1", "m2"):
        err = rel_l2(host(r[k]), ref[k])
        say(f"  {k} rel-L2 {err:.2e}")
        assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_ssa_partial_range_low_rank(ctx, hv, prec):
    """A field of five components with well separated powers over a weak
    noise floor: ranges 1..3, 2..4 and 0..2 end at spectral gaps."""
    say(f"SSA partial ranges prec={prec}")
    rng = np.random.default_rng(11)
    w, ny, nx, n = 32, 64, 128, 80
    t = np.arange(n)[:, None, None]
    u = 0.01 * (rng.standard_normal((n, ny, nx)) + 1j * rng.standard_normal((n, ny, nx)))
    for i, (amp, k) in enumerate(((40.0, 0), (20.0, 3), (10.0, 5), (5.0, 9), (2.5, 12))):
        img = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
        u = u + amp * img[None] * np.exp(2j * np.pi * (k + 0.3 * i) * t / w)
    u = u.astype(np.complex64)
    tp = hv.Temporal(w, 24, 20e3, 0.0, 10e3)
    for c1, c2 in ((1, 3), (2, 4), (0, 2)):
        r = ctx.hv_ssa_moments(dev(u), None, tp, c1, c2, prec)
        ref = _oracle(u, None, tp, c1, c2)
        for k in ("m0", "m1", "m2"):
            err = rel_l2(host(r[k]), ref[k])
            say(f"  [{c1}, {c2}] {k} rel-L2 {err:.2e}")
            assert err < TOL[prec]


def test_ssa_closed_form_on_gpu(ctx, hv):
    """A field window b + a1 e^{2i pi k1 t/W} + a2 e^{2i pi k2 t/W} with
    orthogonal pixel images (|b| > |a1| > |a2|): with components 1..W-1 the
    band moments are those of the two tones alone, W^2 |a_i|^2 at f_ki."""
    say("SSA closed form")
    w, ny, nx, fs = 16, 64, 64, 16e3
    rng = np.random.default_rng(7)
    vecs = []
    for i, norm in enumerate((3.0, 2.0, 1.0)):
        v = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
        for o in vecs:
            v = v - np.vdot(o, v) / np.vdot(o, o) * o
        vecs.append(v / np.linalg.norm(v) * norm * 100.0)
    b, a1, a2 = vecs
    k1, k2 = 3, 6
    t = np.arange(w)[:, None, None]
    u = b[None] + a1[None] * np.exp(2j * np.pi * k1 * t / w) + a2[None] * np.exp(2j * np.pi * k2 * t / w)
    tp = hv.Temporal(w, w, fs, 0.0, fs / 2)
    r = ctx.hv_ssa_moments(dev(u.astype(np.complex64)), None, tp, 1, w - 1, 0)
    f1, f2 = k1 * fs / w, k2 * fs / w
    p1, p2 = w * w * np.abs(a1) ** 2, w * w * np.abs(a2) ** 2
    assert rel_l2(host(r["m0"])[0], p1 + p2) < 1e-5
    assert rel_l2(host(r["m1"])[0], f1 * p1 + f2 * p2) < 1e-5
    assert rel_l2(host(r["m2"])[0], f1 * f1 * p1 + f2 * f2 * p2) < 1e-5


@pytest.mark.parametrize("prec", [0, 1])
def test_ssa_full_range_is_the_stft(ctx, hv, prec):
    say(f"SSA full range vs STFT prec={prec}")
    x, spec = holograms.config_c1()
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(32, 32, spec.fs, 2e3, 8e3)
    r = ctx.hv_ssa_moments(dev(x), opt, tp, 0, 31, prec)
    ref = pipeline.stft_moments(x, pipeline.Optics(LAM, spec.pitch, spec.pitch, -spec.z), 32, 32, spec.fs, 2e3, 8e3)
    for k in ("m0", "m1", "m2"):
        assert rel_l2(host(r[k]), ref[k]) < TOL[prec]


def test_ssa_errors(ctx, hv):
    say("SSA errors")
    x = dev(np.zeros((40, 64, 64), np.uint8))
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.1)
    with pytest.raises(hv.HvError) as e:
        ctx.hv_ssa_moments(x, opt, hv.Temporal(8, 8, 1e3, 0, 500))
    assert e.value.status == hv.HV_ERR_SHAPE
    with pytest.raises(hv.HvError) as e:
        ctx.hv_ssa_moments(x, opt, hv.Temporal(16, 16, 1e3, 0, 500), 5, 3)
    assert e.value.status == hv.HV_ERR_ARG
    with pytest.raises(hv.HvError) as e:
        ctx.hv_ssa_moments(x, opt, hv.Temporal(16, 16, 1e3, 600, 700))
    assert e.value.status == hv.HV_ERR_ARG


@pytest.mark.parametrize("prec", [0, 1])
def test_ssa_precision_shape(ctx, hv, prec):
    """1024^2 12-bit u16 frames, Fresnel at z = -0.5 m, W = 64: one window
    against the oracle."""
    x, spec = holograms.config_c3(64)
    say(f"SSA 1024^2 u16 Fresnel W=64 prec={prec}")
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_FRESNEL)
    fs = spec.fs
    tp = hv.Temporal(64, 64, fs, 2 * fs / 64, 31 * fs / 64)
    r = ctx.hv_ssa_moments(dev(x), opt, tp, 1, 63, prec)
    u = oopt.fresnel(x.astype(np.float64), LAM, spec.pitch, spec.pitch, -spec.z)
    ref = ossa.ssa_moments(u, 64, 64, fs, 2 * fs / 64, 31 * fs / 64, 1, 63)
    for k in ("m0", "m1", "m2"):
        err = rel_l2(host(r[k]), ref[k])
        say(f"  {k} rel-L2 {err:.2e}")
        assert err < TOL[prec]
    assert rel_l2(host(r["eigvals"]), ref["eigvals"]) < TOL[prec]
