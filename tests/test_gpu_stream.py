"""Serving loop on the GPU: each stream's images equal the offline path on the
same frames, overflow and budget refusals are reported, a short replay keeps
every frame."""

import time

import numpy as np
import pytest
import torch

from synth import holograms

pytestmark = pytest.mark.gpu

LAM = 852e-9


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx(hv):
    c = hv.Context(0)
    yield c
    c.close()


def _wait_and_pop(stream, want, store, ny, nx, timeout=20.0):
    t0 = time.time()
    while True:
        m = [torch.empty((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3)]
        r = stream.pop(*m)
        if r is not None:
            store.append([t.cpu().numpy() for t in m])
            continue
        if stream.counters()["windows_done"] >= want and r is None:
            c = stream.counters()
            if len(store) >= want or c["windows_done"] >= want:
                # one more pop round to collect what completed last
                m = [torch.empty((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3)]
                while stream.pop(*m) is not None:
                    store.append([t.cpu().numpy() for t in m])
                    m = [torch.empty((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3)]
                return
        if time.time() - t0 > timeout:
            raise TimeoutError("windows did not complete")
        time.sleep(0.001)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("method,stride,order", [(0, 8, 1), (1, 16, 1), (0, 16, 2)])
def test_stream_images_equal_offline(ctx, hv, prec, method, stride, order):
    """Images popped from a stream equal the offline call bit for bit (order 2:
    the band-first order in both, the stream's workspaces sized for it)."""
    say(f"stream vs offline method={method} stride={stride} order={order} prec={prec}")
    ctx.set_stft_order(order)
    try:
        _stream_vs_offline(ctx, hv, prec, method, stride)
    finally:
        ctx.set_stft_order(hv.HV_ORDER_FRAMES_FIRST)


def _stream_vs_offline(ctx, hv, prec, method, stride):
    spec = holograms.HoloSpec(frames=100, ny=128, nx=256, z=0.25, fs=20e3, seed=42)
    x = holograms.hologram_stack(spec)
    xd = torch.from_numpy(x).cuda()
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, method)
    tp = hv.Temporal(16, stride, spec.fs, 1e3, 9e3)
    ref = [t.cpu().numpy() for t in ctx.hv_stft_moments(xd, opt, tp, prec)]
    j_total = ref[0].shape[0]
    s = ctx.hv_stream_open(128, 256, torch.uint8, opt, tp, prec, ring_frames=64)
    got = []
    pos = 0
    sizes = [5, 7, 13, 1, 16, 3, 9]
    i = 0
    while pos < 100:
        n = min(sizes[i % len(sizes)], 100 - pos)
        s.push(xd[pos:pos + n])
        pos += n
        i += 1
        want = 0 if pos < 16 else (pos - 16) // stride + 1
        _wait_and_pop(s, want, got, 128, 256)
    c = s.counters()
    s.close()
    assert c["pushed"] == 100 and c["dropped"] == 0 and c["windows_done"] == j_total
    assert len(got) == j_total
    for j in range(j_total):
        for k in range(3):
            assert np.array_equal(got[j][k], ref[k][j]), (j, k)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("source", ["pinned", "pageable", "alternating"])
def test_stream_host_push_equals_offline(ctx, hv, source, prec):
    """Frames pushed from host memory: every packet goes through one staging
    buffer that is overwritten with the next packet as soon as the push
    returns (pinned or pageable; "alternating" mixes pinned and device
    packets); the images equal the offline call on the same frames bit for
    bit."""
    say(f"stream host push {source} prec={prec}")
    spec = holograms.HoloSpec(frames=90, ny=128, nx=256, z=0.25, fs=20e3, seed=43)
    x = holograms.hologram_stack(spec)
    xd = torch.from_numpy(x).cuda()
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(16, 8, spec.fs, 1e3, 9e3)
    ref = [t.cpu().numpy() for t in ctx.hv_stft_moments(xd, opt, tp, prec)]
    j_total = ref[0].shape[0]
    stage = torch.empty((16, 128, 256), dtype=torch.uint8)
    if source != "pageable":
        stage = stage.pin_memory()
    s = ctx.hv_stream_open(128, 256, torch.uint8, opt, tp, prec, ring_frames=64)
    got = []
    pos, i = 0, 0
    sizes = [5, 7, 13, 1, 16, 3, 9]
    while pos < 90:
        n = min(sizes[i % len(sizes)], 90 - pos)
        if source == "alternating" and i % 2:
            s.push(xd[pos:pos + n])
        else:
            stage[:n].copy_(torch.from_numpy(x[pos:pos + n]))
            s.push(stage[:n])
            stage.fill_(0)  # the push has returned: the buffer is the caller's again
        pos += n
        i += 1
        want = 0 if pos < 16 else (pos - 16) // 8 + 1
        _wait_and_pop(s, want, got, 128, 256)
    c = s.counters()
    s.close()
    assert c["pushed"] == 90 and c["dropped"] == 0 and c["windows_done"] == j_total
    assert len(got) == j_total
    for j in range(j_total):
        for k in range(3):
            assert np.array_equal(got[j][k], ref[k][j]), (j, k)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("cls", [1, 2])
def test_stream_class_equals_offline(ctx, hv, cls, prec):
    """The larger serving classes: 512^2 u8 with W = 32 and 1024 x 512
    (nx x ny) 12-bit u16 with W = stride = 64; every popped image equals the
    offline call on the same frames bit for bit."""
    ny, nx, bits, fs, w, _ = holograms.STREAM_CLASSES[cls]
    say(f"stream class {cls}: {nx}x{ny} {bits}-bit W={w} prec={prec}")
    n = 3 * w + 7
    x, spec = holograms.stream_block(cls, 5, frames=n)
    xd = torch.from_numpy(x).cuda()
    opt = hv.Optics(LAM, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(w, w, fs, 2 * fs / w, (w // 2 - 1) * fs / w)
    ref = [t.cpu().numpy() for t in ctx.hv_stft_moments(xd, opt, tp, prec)]
    j_total = ref[0].shape[0]
    s = ctx.hv_stream_open(ny, nx, xd.dtype, opt, tp, prec, ring_frames=4 * w)
    got = []
    pos, i = 0, 0
    sizes = [8, 13, 5, 16, 1]
    while pos < n:
        k = min(sizes[i % len(sizes)], n - pos)
        s.push(xd[pos:pos + k])
        pos += k
        i += 1
        _wait_and_pop(s, 0 if pos < w else (pos - w) // w + 1, got, ny, nx)
    c = s.counters()
    s.close()
    assert c["pushed"] == n and c["dropped"] == 0 and c["windows_done"] == j_total == 3
    assert len(got) == j_total
    for j in range(j_total):
        for k in range(3):
            assert np.array_equal(got[j][k], ref[k][j]), (j, k)


def test_stream_open_checks_optics(ctx, hv):
    say("stream open: optics and band checks")
    tp = hv.Temporal(16, 16, 20e3, 1e3, 9e3)
    bad = [hv.Optics(-LAM, 20e-6, 20e-6, -0.2), hv.Optics(LAM, 0.0, 20e-6, -0.2),
           hv.Optics(LAM, 20e-6, 20e-6, -0.2, hv.HV_FRESNEL, highpass=0.1),
           hv.Optics(LAM, 20e-6, 20e-6, -0.2, hv.HV_AS, highpass=1.5)]
    for opt in bad:
        with pytest.raises(hv.HvError) as e:
            ctx.hv_stream_open(64, 64, torch.uint8, opt, tp)
        assert e.value.status == hv.HV_ERR_ARG
    with pytest.raises(hv.HvError) as e:  # a band with no bin
        ctx.hv_stream_open(64, 64, torch.uint8, hv.Optics(LAM, 20e-6, 20e-6, -0.2),
                           hv.Temporal(16, 16, 20e3, 9.1e3, 9.2e3))
    assert e.value.status == hv.HV_ERR_ARG


def test_stream_close_returns_table_bytes(hv):
    """Opening and closing an angular-spectrum stream twice leaves the
    context's held bytes where the first close left them (both transfer
    tables are returned)."""
    say("stream close: held bytes")
    c = hv.Context(0)
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.23)
    tp = hv.Temporal(16, 16, 20e3, 1e3, 9e3)
    held = []
    for _ in range(2):
        s = c.hv_stream_open(128, 128, torch.uint8, opt, tp)
        s.close()
        held.append(c.workspace_bytes())
    c.close()
    assert held[0] == held[1]


def test_stream_overflow_is_refused(ctx, hv):
    say("stream overflow")
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.2)
    tp = hv.Temporal(16, 16, 20e3, 1e3, 9e3)
    s = ctx.hv_stream_open(64, 64, torch.uint8, opt, tp, 0, ring_frames=32)
    frames = torch.zeros((40, 64, 64), dtype=torch.uint8, device="cuda")
    st = s.try_push(frames)
    assert st == hv.HV_ERR_OVERFLOW
    assert s.counters()["dropped"] == 40 and s.counters()["pushed"] == 0
    s.close()


def test_budget_refusal(hv):
    say("budget refusal")
    small = hv.Context(0, hbm_budget=1 << 20)
    opt = hv.Optics(LAM, 20e-6, 20e-6, -0.2)
    tp = hv.Temporal(16, 16, 20e3, 1e3, 9e3)
    with pytest.raises(hv.HvError) as e:
        small.hv_stream_open(256, 256, torch.uint8, opt, tp)
    assert e.value.status == hv.HV_ERR_BUDGET
    assert small.stats()["streams_refused"] == 1
    small.close()


def test_replay_short_no_drops(ctx, hv):
    say("short replay")
    blocks = []
    for cls in (0, 1):
        x, spec = holograms.stream_block(cls, cls, frames=256)
        blocks.append((torch.from_numpy(x).cuda(), spec))
    classes = []
    for (b, spec), w in zip(blocks, (16, 32)):
        classes.append(dict(ny=spec.ny, nx=spec.nx, raw_t=0, fps=spec.fs, window=w, stride=w,
                            f_lo=2 * spec.fs / w, f_hi=(w // 2 - 1) * spec.fs / w, block=b, max_active=2,
                            ring_frames=0))
    r = ctx.hv_replay_run(classes, wavelength=LAM, pitch=20e-6, z_lo=0.1, z_hi=0.4, prec=1, arrival_hz=6.0,
                          mean_life_s=0.5, duration_s=2.0, warmup_s=0.2, packet_frames=8, seed=3)
    say(f"  {r}")
    assert r["errors"] == 0
    assert r["frames_dropped"] == 0
    assert r["streams_admitted"] >= 1 and r["windows_done"] > 0
    assert 0 < r["lat_p50_ns"] <= r["lat_p99_ns"] <= r["lat_max_ns"]
