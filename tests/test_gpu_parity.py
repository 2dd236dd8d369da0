"""HIP path vs the FP64 oracle, element by element, through the C-ABI.

Tolerances (relative L2 over each whole output): 1e-5 for the FP32 form,
2e-3 for the mixed form.  Inputs are seeded and synthetic; nothing the oracle
sees comes from the GPU.
"""

import numpy as np
import pytest
import torch

from oracle import optics as oopt
from oracle import pca as opca
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_frames(seed, n, ny, nx, dtype):
    rng = np.random.default_rng(seed)
    hi = 256 if dtype == np.uint8 else 4096
    return rng.integers(0, hi, (n, ny, nx)).astype(dtype)


# ------------------------------------------------------------------ spatial

@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,dtype", [
    ((4, 64, 128), np.uint8), ((3, 128, 128), np.uint8), ((2, 256, 256), np.uint8),
    ((2, 512, 256), np.uint16), ((1, 1024, 1024), np.uint16), ((2, 128, 1024), np.uint8)])
def test_propagate_as(ctx, hv, shape, dtype, prec):
    say(f"AS {shape} {dtype.__name__} prec={prec}")
    x = rand_frames(1, *shape, dtype)
    opt = hv.Optics(LAM, 20e-6, 15e-6, -0.17, hv.HV_AS)
    u = host(ctx.hv_propagate(dev(x), opt, prec))
    ref = oopt.angular_spectrum(x.astype(np.float64), LAM, 20e-6, 15e-6, -0.17)
    assert rel_l2(u, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("z", [0.5, -0.5])
@pytest.mark.parametrize("shape,dtype", [((3, 128, 64), np.uint16), ((2, 256, 256), np.uint8),
                                         ((1, 512, 1024), np.uint16)])
def test_propagate_fresnel(ctx, hv, shape, dtype, z, prec):
    say(f"Fresnel {shape} {dtype.__name__} z={z} prec={prec}")
    x = rand_frames(2, *shape, dtype)
    opt = hv.Optics(LAM, 20e-6, 25e-6, z, hv.HV_FRESNEL)
    u = host(ctx.hv_propagate(dev(x), opt, prec))
    ref = oopt.fresnel(x.astype(np.float64), LAM, 20e-6, 25e-6, z)
    assert rel_l2(u, ref) < TOL[prec]


@pytest.mark.parametrize("method", [0, 1])
def test_propagate_complex_input(ctx, hv, method):
    say(f"complex input method={method}")
    rng = np.random.default_rng(3)
    x = (rng.standard_normal((3, 128, 256)) + 1j * rng.standard_normal((3, 128, 256))).astype(np.complex64)
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.3, method)
    u = host(ctx.hv_propagate(dev(x), opt))
    fn = oopt.angular_spectrum if method == 0 else oopt.fresnel
    ref = fn(x.astype(np.complex128), LAM, 20e-6, 20e-6, 0.3)
    assert rel_l2(u, ref) < 1e-5


def test_gpu_plus_minus_z_and_parseval(ctx, hv):
    say("GPU +z then -z, Parseval")
    rng = np.random.default_rng(4)
    x = (rng.standard_normal((2, 256, 128)) + 1j * rng.standard_normal((2, 256, 128))).astype(np.complex64)
    xd = dev(x)
    u = ctx.hv_propagate(xd, hv.Optics(LAM, 20e-6, 12e-6, 0.31))
    back = host(ctx.hv_propagate(u, hv.Optics(LAM, 20e-6, 12e-6, -0.31)))
    assert rel_l2(back, x) < 1e-5
    un = host(u)
    for f in range(2):
        assert abs(np.linalg.norm(un[f]) / np.linalg.norm(x[f]) - 1) < 1e-6
    # composition z1 + z2
    a = host(ctx.hv_propagate(ctx.hv_propagate(xd, hv.Optics(LAM, 20e-6, 12e-6, 0.07)),
                              hv.Optics(LAM, 20e-6, 12e-6, 0.11)))
    b = host(ctx.hv_propagate(xd, hv.Optics(LAM, 20e-6, 12e-6, 0.18)))
    assert rel_l2(a, b) < 1e-5


def test_gpu_point_source_fresnel(ctx, hv):
    say("GPU Fresnel point source")
    x = np.zeros((1, 128, 256), np.uint16)
    x[0, 37, 201] = 1000
    opt = hv.Optics(LAM, 20e-6, 30e-6, 0.5, hv.HV_FRESNEL)
    u = host(ctx.hv_propagate(dev(x), opt))[0]
    xi0, eta0 = (201 - 128) * 20e-6, (37 - 64) * 30e-6
    px = (np.arange(256) - 128) * LAM * 0.5 / (256 * 20e-6)
    py = (np.arange(128) - 64) * LAM * 0.5 / (128 * 30e-6)
    yy, xx = np.meshgrid(py, px, indexing="ij")
    expect = 1000 * np.exp(1j * np.pi * ((xx - xi0) ** 2 + (yy - eta0) ** 2) / (LAM * 0.5)) / np.sqrt(128 * 256)
    assert rel_l2(u, expect) < 1e-5


# ------------------------------------------------------------------ STFT moments

def _oracle_moments(frames, opt, tp, keep=False):
    o = None if opt is None else pipeline.Optics(opt.wavelength, opt.pitch_x, opt.pitch_y, opt.z, opt.method)
    return pipeline.stft_moments(frames, o, tp.window, tp.stride, tp.fs, tp.f_lo, tp.f_hi, tp.symmetric, keep)


@pytest.mark.parametrize("prec", [0, 1])
def test_c1_moments(ctx, hv, prec):
    say(f"C1 moments prec={prec}")
    x, spec = holograms.config_c1()
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(32, 32, spec.fs, 2e3, 8e3)
    m = [host(t) for t in ctx.hv_stft_moments(dev(x), opt, tp, prec)]
    ref = _oracle_moments(x, opt, tp)
    for i, k in enumerate(("m0", "m1", "m2")):
        err = rel_l2(m[i], ref[k])
        say(f"  {k} rel-L2 {err:.3e}")
        assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("method", [0, 1])
def test_moments_overlap_ragged(ctx, hv, prec, method):
    say(f"overlapping windows, ragged tail, method={method} prec={prec}")
    x = rand_frames(5, 50, 128, 256, np.uint16)
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.3, method)
    tp = hv.Temporal(16, 6, 20e3, 1.5e3, 9e3)
    ctx.set_chunk_frames(28)  # several chunks with overlap
    try:
        m = [host(t) for t in ctx.hv_stft_moments(dev(x), opt, tp, prec)]
    finally:
        ctx.set_chunk_frames(0)
    ref = _oracle_moments(x, opt, tp)
    assert m[0].shape == (6, 128, 256)
    for i, k in enumerate(("m0", "m1", "m2")):
        assert rel_l2(m[i], ref[k]) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("order", [1, 2])
def test_two_streams_match_one(ctx, hv, prec, order):
    """Several chunks alternate over two streams; one chunk runs on the
    caller's stream alone.  Both schedules give bit-identical moments, in
    either order of the AS moments path (1 frames first, 2 band first)."""
    say(f"two-stream chunk schedule vs one chunk, order={order} prec={prec}")
    x = rand_frames(9, 200, 128, 128, np.uint8)
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.2, hv.HV_AS)
    tp = hv.Temporal(16, 16, 20e3, 1.5e3, 9e3)
    try:
        ctx.set_stft_order(order)
        ctx.set_chunk_frames(32)
        two = [host(t) for t in ctx.hv_stft_moments(dev(x), opt, tp, prec)]
        ctx.set_chunk_frames(256)
        one = [host(t) for t in ctx.hv_stft_moments(dev(x), opt, tp, prec)]
    finally:
        ctx.set_chunk_frames(0)
        ctx.set_stft_order(1)
    assert two[0].shape == (12, 128, 128)
    for a, b in zip(two, one):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [0, 1])
def test_pca_two_streams_match_one(ctx, hv, prec):
    """PCA chunks alternate over two streams as well; the result equals the
    single-chunk run bit for bit."""
    say(f"PCA two-stream chunk schedule vs one chunk, prec={prec}")
    x = rand_frames(10, 200, 64, 128, np.uint8)
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.3, hv.HV_FRESNEL)
    try:
        ctx.set_chunk_frames(40)
        two = ctx.hv_pca(dev(x), opt, 16, 16, 1, 15, prec, want_cov=True)
        ctx.set_chunk_frames(256)
        one = ctx.hv_pca(dev(x), opt, 16, 16, 1, 15, prec, want_cov=True)
    finally:
        ctx.set_chunk_frames(0)
    assert two["m0"].shape == (12, 64, 128)
    for k in ("m0", "eigvals", "cov"):
        assert torch.equal(two[k], one[k]), k


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("window", [8, 16, 32, 64])
def test_field_input_moments(ctx, hv, window, prec):
    say(f"field input W={window} prec={prec}")
    rng = np.random.default_rng(6)
    n = 2 * window + 3
    u = (rng.standard_normal((n, 64, 128)) + 1j * rng.standard_normal((n, 64, 128))).astype(np.complex64)
    tp = hv.Temporal(window, window, 1e4, 0.0, 5e3, symmetric=True)
    m = [host(t) for t in ctx.hv_stft_moments(dev(u), None, tp, prec)]
    ref = _oracle_moments(u, None, tp)
    for i, k in enumerate(("m0", "m1", "m2")):
        assert rel_l2(m[i], ref[k]) < TOL[prec]


def test_pure_tone_on_gpu(ctx, hv):
    say("pure tone")
    w, k0, fs = 32, 5, 33e3
    rng = np.random.default_rng(7)
    a = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    t = np.arange(w)
    u = (a[None] * np.exp(2j * np.pi * k0 * t / w)[:, None, None]).astype(np.complex64)
    tp = hv.Temporal(w, w, fs, 3 * fs / w, 7 * fs / w)
    m0, m1, m2 = [host(x)[0] for x in ctx.hv_stft_moments(dev(u), None, tp)]
    e = w * w * np.abs(a) ** 2
    fk = k0 * fs / w
    assert rel_l2(m0, e) < 1e-5 and rel_l2(m1, fk * e) < 1e-5 and rel_l2(m2, fk * fk * e) < 1e-5
    # a band that excludes k0 sees only rounding
    tp2 = hv.Temporal(w, w, fs, 8 * fs / w, 12 * fs / w)
    m0b = host(ctx.hv_stft_moments(dev(u), None, tp2)[0])[0]
    assert np.max(m0b) < 1e-8 * np.max(e)


@pytest.mark.parametrize("prec", [0, 1])
def test_stft_bins(ctx, hv, prec):
    say(f"spectrum bins prec={prec}")
    x, spec = holograms.config_c1()
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(32, 32, spec.fs, 0.0, spec.fs / 2)
    s = host(ctx.hv_stft_bins(dev(x), opt, tp, prec))
    ref = _oracle_moments(x, opt, tp, keep=True)
    bins = ref["bins"]
    assert s.shape == (2, len(bins), 128, 128)
    assert rel_l2(s, ref["spectrum"][:, bins]) < TOL[prec]


def test_deterministic(ctx, hv):
    say("bitwise determinism")
    x, spec = holograms.config_c1()
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(32, 32, spec.fs, 2e3, 8e3)
    xd = dev(x)
    a = host(ctx.hv_stft_moments(xd, opt, tp)[0])
    b = host(ctx.hv_stft_moments(xd, opt, tp)[0])
    assert np.array_equal(a, b)
    p1 = host(ctx.hv_pca(xd, opt, 32, 32)["m0"])
    p2 = host(ctx.hv_pca(xd, opt, 32, 32)["m0"])
    assert np.array_equal(p1, p2)


# ------------------------------------------------------------------ PCA

@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("method,window", [(0, 16), (1, 32), (0, 64)])
def test_pca(ctx, hv, method, window, prec):
    say(f"PCA method={method} W={window} prec={prec}")
    n = 2 * window + 5
    x = rand_frames(8, n, 128, 64, np.uint8) if method == 0 else rand_frames(8, n, 64, 128, np.uint16)
    ny, nx = x.shape[1:]
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.4, method)
    r = ctx.hv_pca(dev(x), opt, window, window, 1, window - 1, prec, want_cov=True)
    m0, ev, cov, off = host(r["m0"]), host(r["eigvals"]), host(r["cov"]), host(r["offdiag"])
    ref = pipeline.pca_render(x, pipeline.Optics(LAM, 20e-6, 20e-6, 0.4, method), window, window, 1, window - 1)
    assert m0.shape == (2, ny, nx)
    e_cov, e_ev, e_m0 = rel_l2(cov, ref["cov"]), rel_l2(ev, ref["eigvals"]), rel_l2(m0, ref["m0"])
    say(f"  cov {e_cov:.2e} eigvals {e_ev:.2e} m0 {e_m0:.2e} offdiag {off.max():.1e}")
    assert np.all(off < 1e-14)  # every window's Jacobi converged
    assert e_cov < TOL[prec]
    assert e_ev < TOL[prec]
    assert e_m0 < TOL[prec]


def test_pca_trace_and_rank_one(ctx, hv):
    say("PCA invariants on GPU")
    rng = np.random.default_rng(9)
    a = rng.standard_normal(64 * 64) + 1j * rng.standard_normal(64 * 64)
    b = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    u = np.outer(a, b).T.reshape(16, 64, 64).astype(np.complex64)
    r = ctx.hv_pca(dev(u), None, 16, 16, 1, 15, want_cov=True)
    ev = host(r["eigvals"])[0]
    lam0 = np.linalg.norm(a) ** 2 * np.linalg.norm(b) ** 2
    assert abs(ev[0] - lam0) / lam0 < 1e-5
    assert np.max(np.abs(ev[1:])) < 1e-5 * lam0
    assert np.max(host(r["m0"])) < 1e-5 * lam0
    u2 = (rng.standard_normal((16, 64, 64)) + 1j * rng.standard_normal((16, 64, 64))).astype(np.complex64)
    r2 = ctx.hv_pca(dev(u2), None, 16, 16, 0, 15, want_cov=True)
    ev2 = host(r2["eigvals"])[0]
    fro = np.sum(np.abs(u2.astype(np.complex128)) ** 2)
    assert abs(ev2.sum() - fro) / fro < 1e-5
    assert rel_l2(host(r2["m0"])[0], np.sum(np.abs(u2.astype(np.complex128)) ** 2, axis=0)) < 1e-5


# ------------------------------------------------------------------ errors and edges

def test_errors(ctx, hv):
    say("error paths")
    x = dev(np.zeros((4, 64, 64), np.uint8))
    opt = hv.Optics(LAM, 20e-6, 20e-6, 0.1)
    with pytest.raises(hv.HvError) as e:
        ctx.hv_stft_moments(x, opt, hv.Temporal(8, 8, 1e3, 0, 500))
    assert e.value.status == hv.HV_ERR_SHAPE
    with pytest.raises(hv.HvError) as e:
        ctx.hv_propagate(dev(np.zeros((1, 96, 64), np.uint8)), opt)
    assert e.value.status == hv.HV_ERR_SHAPE
    with pytest.raises(hv.HvError) as e:
        ctx.hv_stft_moments(dev(np.zeros((16, 64, 64), np.uint8)), opt, hv.Temporal(8, 8, 1e3, 600, 700))
    assert e.value.status == hv.HV_ERR_ARG
    with pytest.raises(hv.HvError) as e:
        ctx.hv_propagate(x, hv.Optics(LAM, 20e-6, 20e-6, 0.0, hv.HV_FRESNEL))
    assert e.value.status == hv.HV_ERR_ARG
    with pytest.raises(hv.HvError) as e:
        ctx.hv_pca(dev(np.zeros((16, 64, 64), np.uint8)), opt, 16, 16, 3, 2)
    assert e.value.status == hv.HV_ERR_ARG
    # zero frames is a no-op
    out = ctx.hv_propagate(dev(np.zeros((0, 64, 64), np.uint8)), opt)
    assert out.shape == (0, 64, 64)


# ------------------------------------------------------------------ full-size workloads (sampled)

@pytest.fixture(scope="module")
def c2_block():
    return holograms.config_c2_block(2048)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("order", [1, 2])
def test_c2_block_sampled_windows(ctx, hv, c2_block, prec, order):
    x, spec = c2_block
    say(f"256^2 headline block: 2048 frames, order={order} prec={prec}")
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(32, 32, spec.fs, 3e3, 35e3)
    ctx.set_stft_order(order)
    try:
        m = [host(t) for t in ctx.hv_stft_moments(dev(x), opt, tp, prec)]
    finally:
        ctx.set_stft_order(1)
    assert m[0].shape == (64, 256, 256)
    for j in (0, 31, 63):
        ref = _oracle_moments(x[32 * j:32 * j + 32], opt, tp)
        for i, k in enumerate(("m0", "m1", "m2")):
            err = rel_l2(m[i][j], ref[k][0])
            assert err < TOL[prec], (j, k, err)


@pytest.fixture(scope="module")
def c3_frames():
    return holograms.config_c3(64)


@pytest.mark.parametrize("prec", [0, 1])
def test_c3_shape_fresnel_stft_pca(ctx, hv, c3_frames, prec):
    x, spec = c3_frames
    say(f"1024^2 u16 Fresnel, W=64, prec={prec}")
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_FRESNEL)
    xd = dev(x)
    u_ref = oopt.fresnel(x.astype(np.float64), LAM, spec.pitch, spec.pitch, -spec.z)
    fs = spec.fs
    tp = hv.Temporal(64, 64, fs, 2 * fs / 64, 31 * fs / 64)
    m = [host(t) for t in ctx.hv_stft_moments(xd, opt, tp, prec)]
    s_ref = otemp.stft(u_ref, 64, 64)
    bins, freqs = otemp.band_bins(64, fs, 2 * fs / 64, 31 * fs / 64)
    for i, mr in enumerate(otemp.moments(s_ref, bins, freqs)):
        err = rel_l2(m[i], mr)
        say(f"  M{i} rel-L2 {err:.3e}")
        assert err < TOL[prec]
    r = ctx.hv_pca(xd, opt, 64, 64, 1, 63, prec, want_cov=True)
    pr = opca.pca_window(u_ref, 1, 63)
    for k, got in (("cov", host(r["cov"])[0]), ("eigvals", host(r["eigvals"])[0]), ("m0", host(r["m0"])[0])):
        err = rel_l2(got, pr[k])
        say(f"  PCA {k} rel-L2 {err:.3e}")
        assert err < TOL[prec]


# ------------------------------------------------------------------ full sizes of the benchmark launches

@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("order", [1, 2])
def test_c2_full_stream(ctx, hv, c2_block, prec, order):
    """The 65,536-frame stream as the benchmark times it (the 2,048-frame
    block replayed 32 times, same chunks and streams).  Windows 64 apart see
    the same frames, so every window must equal its counterpart in the first
    block bit for bit; three windows are checked against the oracle."""
    x, spec = c2_block
    say(f"256^2 full stream: 65536 frames, order={order} prec={prec}")
    xs = dev(x).repeat(32, 1, 1).contiguous()
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(32, 32, spec.fs, 3e3, 35e3)
    ctx.set_stft_order(order)
    try:
        m = ctx.hv_stft_moments(xs, opt, tp, prec)
        torch.cuda.synchronize()
    finally:
        ctx.set_stft_order(1)
    del xs
    assert m[0].shape == (2048, 256, 256)
    for t in m:
        per = t.view(32, 64, 256, 256)
        assert torch.equal(per, per[:1].expand_as(per)), "windows over the same frames differ"
    for j in (0, 1029, 2047):
        b = j % 64
        ref = _oracle_moments(x[32 * b:32 * b + 32], opt, tp)
        for i, k in enumerate(("m0", "m1", "m2")):
            err = rel_l2(host(m[i][j]), ref[k][0])
            assert err < TOL[prec], (j, k, err)


@pytest.fixture(scope="module")
def c3_block():
    return holograms.config_c3(128)


@pytest.mark.parametrize("prec", [0, 1])
def test_c3_full_size(ctx, hv, c3_block, prec):
    """4,096 u16 frames of 1024^2 (a 128-frame block replayed 32 times):
    Fresnel, W = 64 moments and PCA over every window at full size.  Windows
    two apart see the same frames and must agree bit for bit; windows 0 and
    63 are checked against the oracle."""
    x, spec = c3_block
    say(f"1024^2 u16 full size: 4096 frames, prec={prec}")
    xs = dev(x).repeat(32, 1, 1).contiguous()
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_FRESNEL)
    fs = spec.fs
    tp = hv.Temporal(64, 64, fs, 2 * fs / 64, 31 * fs / 64)
    m = ctx.hv_stft_moments(xs, opt, tp, prec)
    r = ctx.hv_pca(xs, opt, 64, 64, 1, 63, prec, want_cov=True)
    torch.cuda.synchronize()
    del xs
    assert m[0].shape == (64, 1024, 1024) and r["m0"].shape == (64, 1024, 1024)
    for t in list(m) + [r["m0"], r["eigvals"], r["cov"]]:
        per = t.view(32, 2, *t.shape[1:])
        assert torch.equal(per, per[:1].expand_as(per)), "windows over the same frames differ"
    bins, freqs = otemp.band_bins(64, fs, 2 * fs / 64, 31 * fs / 64)
    for j in (0, 63):
        b = j % 2
        u_ref = oopt.fresnel(x[64 * b:64 * b + 64].astype(np.float64), LAM, spec.pitch, spec.pitch, -spec.z)
        s_ref = otemp.stft(u_ref, 64, 64)
        for i, mr in enumerate(otemp.moments(s_ref, bins, freqs)):
            err = rel_l2(host(m[i][j]), mr[0])
            assert err < TOL[prec], (j, i, err)
        pr = opca.pca_window(u_ref, 1, 63)
        for k, got in (("cov", host(r["cov"][j])), ("eigvals", host(r["eigvals"][j])), ("m0", host(r["m0"][j]))):
            err = rel_l2(got, pr[k])
            assert err < TOL[prec], (j, k, err)
