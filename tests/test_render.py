"""Image products (PNG and iso-intensity contours) on the CPU."""
import struct
import zlib

import numpy as np

from paper_2609_08989_amd import render


def parse_png(b):
    assert b[:8] == b"\x89PNG\r\n\x1a\n"
    pos, chunks = 8, {}
    while pos < len(b):
        (n,) = struct.unpack(">I", b[pos:pos + 4])
        tag, data = b[pos + 4:pos + 8], b[pos + 8:pos + 8 + n]
        (crc,) = struct.unpack(">I", b[pos + 8 + n:pos + 12 + n])
        assert crc == zlib.crc32(tag + data) & 0xFFFFFFFF
        chunks.setdefault(tag, b"")
        chunks[tag] += data
        pos += 12 + n
    w, h, depth, ctype, _, _, _ = struct.unpack(">IIBBBBB", chunks[b"IHDR"])
    raw = zlib.decompress(chunks[b"IDAT"])
    rows = [raw[j * (w + 1):(j + 1) * (w + 1)] for j in range(h)]
    assert all(r[0] == 0 for r in rows)
    return w, h, depth, ctype, np.array([list(r[1:]) for r in rows], dtype=np.uint8)


def test_png_round_trip_and_orientation():
    ny, nx = 5, 7
    img = np.arange(ny * nx, dtype=np.float64).reshape(ny, nx)
    w, h, depth, ctype, px = parse_png(render.png_bytes(render.to_8bit(img)))
    assert (w, h, depth, ctype) == (nx, ny, 8, 0)
    want = np.round(255 * img / img.max()).astype(np.uint8)[::-1]   # largest beta on top
    assert np.array_equal(px, want)
    assert render.to_8bit(np.zeros((2, 2))).max() == 0


def test_intensity_map_layout():
    nx, ny = 4, 3
    out = {"intensity": np.arange(2 * nx * ny, dtype=np.float64)}
    m1 = render.intensity_map(out, nx, ny, camera=1)
    assert m1.shape == (ny, nx) and m1[2, 3] == nx * ny + 2 * nx + 3


def test_contours_of_a_cone_are_circles():
    n, cx, cy = 81, 40.3, 39.7
    y, x = np.mgrid[0:n, 0:n]
    img = np.hypot(x - cx, y - cy)            # linear along every grid edge it crosses, nearly
    for level in (7.0, 18.5, 30.0):
        segs = render.contours(img, level)
        pts = np.array([p for s in segs for p in s])
        d = np.hypot(pts[:, 0] - cx, pts[:, 1] - cy)
        assert np.abs(d - level).max() < 0.06
        length = sum(np.hypot(s[1][0] - s[0][0], s[1][1] - s[0][1]) for s in segs)
        assert abs(length / (2 * np.pi * level) - 1) < 0.01


def test_contours_saddle_and_empty():
    img = np.array([[1.0, 0.0], [0.0, 1.0]])
    segs = render.contours(img, 0.5)
    assert len(segs) == 2
    assert render.contours(np.ones((3, 3)), 2.0) == []
