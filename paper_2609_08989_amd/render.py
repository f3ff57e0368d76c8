"""Image products of a trace (the rendered outputs of Sec. 3 and Fig. KerrUHD):
the intensity map of a camera as a 2-D array, an 8-bit grayscale PNG of it,
and iso-intensity contours (panel c of that figure).

Host-side post-processing of the traced outputs (numpy arrays as returned by
``tartarus.to_numpy``); it needs no GPU and no imaging library.
"""
from __future__ import annotations

import struct
import zlib

import numpy as np


def intensity_map(out: dict, nx: int, ny: int, camera: int = 0) -> np.ndarray:
    """The camera's I_pix as an (ny, nx) array: row j holds beta_j, column i
    alpha_i (pixel index c * nx * ny + j * nx + i)."""
    n = nx * ny
    return np.asarray(out["intensity"], dtype=np.float64)[camera * n:(camera + 1) * n].reshape(ny, nx)


def to_8bit(img: np.ndarray, vmax: float | None = None, gamma: float = 1.0) -> np.ndarray:
    """Scale [0, vmax] (default: the image maximum) to 0..255 with x^(1/gamma)."""
    v = float(np.max(img)) if vmax is None else float(vmax)
    if not v > 0.0:
        return np.zeros(img.shape, dtype=np.uint8)
    x = np.clip(np.asarray(img, dtype=np.float64) / v, 0.0, 1.0) ** (1.0 / gamma)
    return np.round(255.0 * x).astype(np.uint8)


def _chunk(tag: bytes, data: bytes) -> bytes:
    return struct.pack(">I", len(data)) + tag + data + struct.pack(">I", zlib.crc32(tag + data) & 0xFFFFFFFF)


def png_bytes(img8: np.ndarray, beta_up: bool = True) -> bytes:
    """An 8-bit grayscale PNG (filter type 0 on every row).  With beta_up the
    largest beta is the top row, as on the sky."""
    img8 = np.asarray(img8, dtype=np.uint8)
    if img8.ndim != 2:
        raise ValueError("expected a 2-D image")
    h, w = img8.shape
    rows = img8[::-1] if beta_up else img8
    raw = b"".join(b"\x00" + rows[j].tobytes() for j in range(h))
    header = struct.pack(">IIBBBBB", w, h, 8, 0, 0, 0, 0)
    return (b"\x89PNG\r\n\x1a\n" + _chunk(b"IHDR", header) + _chunk(b"IDAT", zlib.compress(raw, 6))
            + _chunk(b"IEND", b""))


def write_png(path: str, img: np.ndarray, vmax: float | None = None, gamma: float = 1.0) -> None:
    with open(path, "wb") as fh:
        fh.write(png_bytes(to_8bit(img, vmax, gamma)))


# marching squares: corner order (x, y) = (0,0), (1,0), (1,1), (0,1); bit k set
# when corner k is at or above the level.  Edges: 0 bottom (c0-c1), 1 right
# (c1-c2), 2 top (c3-c2), 3 left (c0-c3).  Each case lists edge pairs joined.
_CASES = {
    0: (), 15: (),
    1: ((3, 0),), 14: ((3, 0),),
    2: ((0, 1),), 13: ((0, 1),),
    3: ((3, 1),), 12: ((3, 1),),
    4: ((1, 2),), 11: ((1, 2),),
    6: ((0, 2),), 9: ((0, 2),),
    7: ((3, 2),), 8: ((3, 2),),
}


def contours(img: np.ndarray, level: float) -> list:
    """Line segments ((x0, y0), (x1, y1)) in pixel coordinates (x = column,
    y = row) along which the bilinear interpolant of img equals level.
    Saddle cells take the connection the cell-centre average selects."""
    a = np.asarray(img, dtype=np.float64)
    ny, nx = a.shape
    segs = []

    def cross(x0, y0, v0, x1, y1, v1):
        t = (level - v0) / (v1 - v0)
        return (x0 + t * (x1 - x0), y0 + t * (y1 - y0))

    for y in range(ny - 1):
        for x in range(nx - 1):
            c = (a[y, x], a[y, x + 1], a[y + 1, x + 1], a[y + 1, x])
            idx = sum(1 << k for k in range(4) if c[k] >= level)
            if idx in (0, 15):
                continue
            pts = {
                0: lambda: cross(x, y, c[0], x + 1, y, c[1]),
                1: lambda: cross(x + 1, y, c[1], x + 1, y + 1, c[2]),
                2: lambda: cross(x, y + 1, c[3], x + 1, y + 1, c[2]),
                3: lambda: cross(x, y, c[0], x, y + 1, c[3]),
            }
            if idx in (5, 10):
                centre_hi = 0.25 * sum(c) >= level
                # corners 0 and 2 above (5) or 1 and 3 above (10)
                if (idx == 5) == centre_hi:
                    pairs = ((0, 1), (2, 3))
                else:
                    pairs = ((3, 0), (1, 2))
            else:
                pairs = _CASES[idx]
            for e0, e1 in pairs:
                segs.append((pts[e0](), pts[e1]()))
    return segs
