"""Host logic of bench.py (CPU only): the one-GPU refusal, the algorithmic
byte counts of the headline kernels, and the tie between the committed HBM
counter summary and the library sources it was taken from."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bytes_per_pixel_frame():
    # per u8 pixel-frame at W = 32 with 14 bins: frames first reads 1 B and
    # moves the half spectrum (e/2 out, e/2 in), the full spectrum (e out,
    # e in) and 3 float images per window; band first moves the 14 bin
    # fields of 32 frames four times (written, read and rewritten in place,
    # read)
    ff = ("row_r2c", "col_as", "rowinv_coef")
    bf = ("band_rows", "band_cols", "band_power")
    f32, f16 = bench.bytes_per_pxf(0, 14), bench.bytes_per_pxf(1, 14)
    assert sum(f32[k] for k in ff) == 1 + 4 + 4 + 8 + 8 + 12 / 32 == 25.375
    assert sum(f16[k] for k in ff) == 1 + 2 + 2 + 4 + 4 + 12 / 32 == 13.375
    assert sum(f32[k] for k in bf) == 1 + 4 * 14 * 8 / 32 + 12 / 32 == 15.375
    assert sum(f16[k] for k in bf) == 1 + 4 * 14 * 4 / 32 + 12 / 32 == 8.375


def test_traffic_is_reported_only_for_the_sources_it_was_taken_from(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "hbm_traffic_as_stft32_256x256.json")) as f:
        summary = json.load(f)
    monkeypatch.setattr(bench, "source_sha", lambda: summary["source_sha"])
    t = bench.measured_traffic("col_as", "fp32")
    algorithmic = 128 * 256 * 256 * (4 + 8)  # one 128-frame launch of the column pass
    assert t is not None and 1.0 <= t / algorithmic < 1.1
    monkeypatch.setattr(bench, "source_sha", lambda: "0" * 16)
    assert bench.measured_traffic("col_as", "fp32") is None
