"""The library's .holo reader and writer against the layout oracle (host
code only; runs without a GPU)."""

import numpy as np
import torch

from oracle import holo


def test_library_writes_the_oracle_bytes(hv_host, tmp_path):
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, (4, 20, 36)).astype(np.uint8)
    a, b = tmp_path / "lib.holo", tmp_path / "ref.holo"
    hv_host.holo_write(a, torch.from_numpy(x), footer='{"z": 0.2}')
    holo.write(b, x, footer={"z": 0.2})
    assert a.read_bytes() == b.read_bytes()


def test_library_reads_oracle_files(hv_host, tmp_path):
    rng = np.random.default_rng(4)
    x = rng.integers(0, 4096, (6, 8, 10)).astype(np.uint16)
    for end in (0, 1):
        p = tmp_path / f"e{end}.holo"
        holo.write(p, x, footer={"k": [1, 2]}, endianness=end, data_type=1)
        head, frames, footer = hv_host.holo_read(p, first=2, count=3)
        assert head["bits_per_pixel"] == 16 and head["image_count"] == 6 and head["data_type"] == 1
        assert head["endianness"] == end and head["data_size"] == x.nbytes
        assert np.array_equal(frames.numpy().view(np.uint16), x[2:5])
        assert footer == '{"k": [1, 2]}'


def test_big_endian_write_matches_oracle(hv_host, tmp_path):
    x = np.arange(2 * 3 * 4, dtype=np.uint16).reshape(2, 3, 4) * 257
    a, b = tmp_path / "lib.holo", tmp_path / "ref.holo"
    hv_host.holo_write(a, torch.from_numpy(x.view(np.int16)), endianness=1)
    holo.write(b, x, endianness=1)
    assert a.read_bytes() == b.read_bytes()


def test_bad_files_are_refused(hv_host, tmp_path):
    p = tmp_path / "bad.holo"
    p.write_bytes(b"HOLA" + bytes(60))
    try:
        hv_host.holo_read(p)
    except hv_host.HvError:
        pass
    else:
        raise AssertionError("a file without the magic was accepted")
