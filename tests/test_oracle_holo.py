"""The .holo layout oracle against a header derived by hand from the paper's
field list and against hand-checked bytes (CPU only)."""

import os

import numpy as np
import pytest

from oracle import holo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "holo_header_512x320x1000_u8.txt")


def golden_header() -> bytes:
    hexes = []
    for line in open(GOLDEN):
        if not line.startswith("#"):
            hexes += line.split()
    return bytes(int(h, 16) for h in hexes)


def test_header_matches_hand_derived_bytes():
    g = golden_header()
    assert len(g) == 64
    assert holo.pack_header(8, 512, 320, 1000) == g
    assert holo.unpack_header(g) == {"version": 7, "bits": 8, "width": 512, "height": 320, "count": 1000,
                                     "data_size": 163840000, "endianness": 0, "data_type": 0}


def test_big_endian_pixels_on_disk(tmp_path):
    x = np.array([[[0x0102, 0xA0B0]]], dtype=np.uint16)  # one 1 x 2 image
    p = tmp_path / "be.holo"
    holo.write(p, x, endianness=1)
    b = p.read_bytes()
    assert b[64:68] == bytes([0x01, 0x02, 0xA0, 0xB0])
    p2 = tmp_path / "le.holo"
    holo.write(p2, x)
    assert p2.read_bytes()[64:68] == bytes([0x02, 0x01, 0xB0, 0xA0])
    for path in (p, p2):
        hd, frames, footer = holo.read(path)
        assert hd["bits"] == 16 and footer is None
        assert np.array_equal(frames, x)


def test_round_trip_with_footer(tmp_path):
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, (5, 6, 7)).astype(np.uint8)
    p = tmp_path / "f.holo"
    holo.write(p, x, footer={"compute_settings": {"z": 0.2}}, data_type=1)
    hd, frames, footer = holo.read(p)
    assert hd["data_type"] == 1 and hd["data_size"] == x.size
    assert np.array_equal(frames, x) and footer == {"compute_settings": {"z": 0.2}}
    assert os.path.getsize(p) == 64 + x.size + len(b'{"compute_settings": {"z": 0.2}}')


def test_rejects_foreign_file():
    with pytest.raises(ValueError):
        holo.unpack_header(b"HOLA" + bytes(60))
