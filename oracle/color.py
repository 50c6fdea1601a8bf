"""NV12 -> RGB BT.601, bilinear resize and 16-bin HIST (oracle; test infrastructure only).

Scanner treats the frame-format conversion that follows video decode as
decoder post-processing that is skipped for frames a graph does not need
(Sec. 4.3), resizing as an ordinary map operation (Sec. 3.1, the Resize stage
of the face-detection example) and HIST as "compute the pixel colour
histogram for all frames" (Sec. 5.1.2).  The paper fixes no colour matrix,
fixed-point format or bin layout; the readings below fix them.

Readings:
* NV12 = Y plane (H rows x pitch bytes) followed by an interleaved U,V plane
  (H/2 rows x pitch bytes, U first), both 8-bit.  Pixel (x, y) takes chroma
  sample (x >> 1, y >> 1) (nearest replication; chroma siting ignored).
* BT.601 limited range: Y' = (Y - 16)/219, Pb, Pr = (C - 128)/224, with
  Kr = 0.299, Kb = 0.114, Kg = 0.587.  The real coefficients are rounded
  half-to-even to Q14 from exact rationals; the result is
  clamp((sum + 2^13) >> 14, 0, 255) with an arithmetic (floor) shift.
* Resize: convert at full resolution, then bilinear with half-pixel centres
  and 8-bit integer weights (exact integer arithmetic, round half up).
* HIST: 16 uniform bins of width 16 over [0, 256) per R, G, B channel of the
  full-resolution converted frame, uint32 counts, layout [3][16].

Pins (tests): exhaustive comparison against the exact rational formula over
all 2^24 (Y, U, V) triples; grey axis and extreme codes; resize identity,
exact 2x = 2x2 mean, constant images; brute-force interval HIST on tiny
frames and bin sums.  Parity pinned.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

KR = Fraction(299, 1000)
KB = Fraction(114, 1000)
KG = 1 - KR - KB


def real_coefficients():
    """Exact rational BT.601 limited-range coefficients (cY, cRV, cGU, cGV, cBU)."""
    s = Fraction(255, 224)
    c_y = Fraction(255, 219)
    c_rv = s * 2 * (1 - KR)
    c_gu = s * 2 * KB * (1 - KB) / KG
    c_gv = s * 2 * KR * (1 - KR) / KG
    c_bu = s * 2 * (1 - KB)
    return c_y, c_rv, c_gu, c_gv, c_bu


def _round_half_even(fr: Fraction) -> int:
    return round(fr)  # Python's round on Fraction is half-to-even


def q14_coefficients():
    return tuple(_round_half_even(c * (1 << 14)) for c in real_coefficients())


def split_nv12(frame: np.ndarray, width: int, height: int):
    """frame: uint8 [height*3/2, pitch] -> Y [H, W], U [H/2, W/2], V [H/2, W/2]."""
    y = frame[:height, :width]
    uv = frame[height:height + height // 2, :width]
    return y, uv[:, 0::2], uv[:, 1::2]


def nv12_to_rgb(y: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Q14 BT.601 conversion; returns uint8 [H, W, 3] (R, G, B)."""
    c_y, c_rv, c_gu, c_gv, c_bu = q14_coefficients()
    H, W = y.shape
    uu = np.repeat(np.repeat(u.astype(np.int64), 2, axis=0), 2, axis=1)[:H, :W] - 128
    vv = np.repeat(np.repeat(v.astype(np.int64), 2, axis=0), 2, axis=1)[:H, :W] - 128
    yy = y.astype(np.int64) - 16
    half = 1 << 13
    r = (c_y * yy + c_rv * vv + half) >> 14
    g = (c_y * yy - c_gu * uu - c_gv * vv + half) >> 14
    b = (c_y * yy + c_bu * uu + half) >> 14
    rgb = np.stack([r, g, b], axis=-1)
    return np.clip(rgb, 0, 255).astype(np.uint8)


def nv12_to_rgb_exact_real(y: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """The real-valued BT.601 formula with exact rational arithmetic and round-half-up,
    clamped to 0..255.  Used as an independent pin of the Q14 path."""
    c_y, c_rv, c_gu, c_gv, c_bu = real_coefficients()
    coeffs = [c_y, c_rv, c_gu, c_gv, c_bu]
    den = 1
    for c in coeffs:
        den = den * c.denominator // np.gcd(den, c.denominator)
    num = [int(c * den) for c in coeffs]
    H, W = y.shape
    uu = np.repeat(np.repeat(u.astype(np.int64), 2, axis=0), 2, axis=1)[:H, :W] - 128
    vv = np.repeat(np.repeat(v.astype(np.int64), 2, axis=0), 2, axis=1)[:H, :W] - 128
    yy = y.astype(np.int64) - 16
    # value = N / den; round half up = floor((2N + den) / (2 den))
    n_r = num[0] * yy + num[1] * vv
    n_g = num[0] * yy - num[2] * uu - num[3] * vv
    n_b = num[0] * yy + num[4] * uu
    out = [np.floor_divide(2 * n + den, 2 * den) for n in (n_r, n_g, n_b)]
    return np.clip(np.stack(out, axis=-1), 0, 255).astype(np.uint8)


def _resize_taps(n_in: int, n_out: int):
    """Per output index: (i0, i1, f) with f the 8-bit weight of i1."""
    taps = []
    for x in range(n_out):
        n = (2 * x + 1) * n_in - n_out
        if n < 0:
            n = 0
        i0 = n // (2 * n_out)
        r = n % (2 * n_out)
        f = (256 * r + n_out) // (2 * n_out)
        i0 = min(i0, n_in - 1)
        i1 = min(i0 + 1, n_in - 1)
        taps.append((i0, i1, f))
    return taps


def resize_bilinear_q8(img: np.ndarray, out_w: int, out_h: int) -> np.ndarray:
    """Bilinear resize with half-pixel centres and exact 8-bit weights.

    img: uint8 [H, W] or [H, W, C]; returns the same dtype at [out_h, out_w(, C)]."""
    H, W = img.shape[:2]
    x0, x1, fx = (np.array(a, dtype=np.int64) for a in zip(*_resize_taps(W, out_w)))
    y0, y1, fy = (np.array(a, dtype=np.int64) for a in zip(*_resize_taps(H, out_h)))
    src = img.astype(np.int64)
    extra = (1,) * (img.ndim - 2)
    fx = fx.reshape((1, -1) + extra)
    fy = fy.reshape((-1, 1) + extra)
    p00 = src[y0][:, x0]
    p01 = src[y0][:, x1]
    p10 = src[y1][:, x0]
    p11 = src[y1][:, x1]
    acc = ((256 - fx) * (256 - fy) * p00 + fx * (256 - fy) * p01
           + (256 - fx) * fy * p10 + fx * fy * p11)
    return ((acc + (1 << 15)) >> 16).astype(np.uint8)


def convert(frame: np.ndarray, width: int, height: int, out_w: int | None = None,
            out_h: int | None = None, fmt: str = "rgb24") -> np.ndarray:
    """One sampled row -> RGB24 [out_h, out_w, 3] or GRAY8 [out_h, out_w]."""
    out_w = width if out_w is None else out_w
    out_h = height if out_h is None else out_h
    y, u, v = split_nv12(frame, width, height)
    if fmt == "gray8":
        img = np.ascontiguousarray(y)
    else:
        img = nv12_to_rgb(y, u, v)
    if (out_w, out_h) == (width, height):
        return img.copy()
    return resize_bilinear_q8(img, out_w, out_h)


def hist16(rgb: np.ndarray) -> np.ndarray:
    """16-bin-per-channel histogram of uint8 [H, W, 3] -> uint32 [3, 16]."""
    out = np.zeros((3, 16), dtype=np.uint32)
    for c in range(3):
        out[c] = np.bincount((rgb[..., c].astype(np.int64) >> 4).ravel(), minlength=16)[:16]
    return out


def hist_frame(frame: np.ndarray, width: int, height: int) -> np.ndarray:
    y, u, v = split_nv12(frame, width, height)
    return hist16(nv12_to_rgb(y, u, v))
