"""The .holo file layout, written out with ``struct`` (test infrastructure
only; see the package docstring).

Sec. IV (Holofile system) fixes the file as three parts:

* a 64-byte header: the magic "HOLO" (4 bytes), the version, 7 (2 bytes),
  bits per pixel (2), image width (4), image height (4), number of images
  (4), total data size in bytes (8), endianness (1 byte; 0 little, 1 big),
  data type (1 byte; 0 raw, 1 processed), zero padding to 64 bytes;
* the images as one binary stream, a whole number of bytes per pixel;
* an optional JSON footer of rendering settings.

Readings: the header's integer fields are little endian; the endianness
byte describes the pixel data (16-bit pixels of a big-endian file are
byte-swapped when read); the footer is the rest of the file after the data.
"""

from __future__ import annotations

import json
import struct

import numpy as np

MAGIC = b"HOLO"
HEADER_BYTES = 64
_FIELDS = "<4sHHIIIQBB"  # 30 bytes, then padding


def pack_header(bits: int, width: int, height: int, count: int, data_type: int = 0, endianness: int = 0,
                version: int = 7) -> bytes:
    size = width * height * count * (bits // 8)
    head = struct.pack(_FIELDS, MAGIC, version, bits, width, height, count, size, endianness, data_type)
    return head + bytes(HEADER_BYTES - len(head))


def unpack_header(b: bytes) -> dict:
    if len(b) < HEADER_BYTES:
        raise ValueError("short header")
    magic, version, bits, width, height, count, size, endianness, data_type = struct.unpack_from(_FIELDS, b)
    if magic != MAGIC:
        raise ValueError("not a .holo file")
    return {"version": version, "bits": bits, "width": width, "height": height, "count": count,
            "data_size": size, "endianness": endianness, "data_type": data_type}


def write(path, frames, footer: dict | None = None, data_type: int = 0, endianness: int = 0) -> None:
    frames = np.ascontiguousarray(frames)
    if frames.dtype not in (np.uint8, np.uint16):
        raise TypeError("frames must be uint8 or uint16")
    n, h, w = frames.shape
    bits = 8 * frames.dtype.itemsize
    data = frames.astype(frames.dtype.newbyteorder(">" if endianness else "<"), copy=False).tobytes()
    with open(path, "wb") as f:
        f.write(pack_header(bits, w, h, n, data_type, endianness))
        f.write(data)
        if footer is not None:
            f.write(json.dumps(footer).encode())


def read(path):
    """(header dict, frames [n][h][w] in native byte order, footer dict or None)."""
    with open(path, "rb") as f:
        blob = f.read()
    hd = unpack_header(blob[:HEADER_BYTES])
    bpp = hd["bits"] // 8
    dt = {1: np.uint8, 2: np.uint16}[bpp]
    end = HEADER_BYTES + hd["data_size"]
    raw = np.frombuffer(blob[HEADER_BYTES:end], dtype=np.dtype(dt).newbyteorder(">" if hd["endianness"] else "<"))
    frames = raw.astype(dt).reshape(hd["count"], hd["height"], hd["width"])
    rest = blob[end:]
    return hd, frames, (json.loads(rest.decode()) if rest else None)
