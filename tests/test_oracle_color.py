"""Pins of the colour / resize / HIST oracle against what the mathematics fixes:
the exact rational BT.601 formula over every (Y, U, V) triple, the grey axis and
the extreme codes, resize identities, and a brute-force interval histogram."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import color as C


def exhaustive_frame():
    """4096x4096 NV12 planes holding every (Y, U, V) triple exactly once:
    chroma block b carries (U, V) = divmod(b mod 65536, 256) and its four luma
    samples are 4 * (b div 65536) + 0..3."""
    b = np.arange(2048 * 2048, dtype=np.int64).reshape(2048, 2048)
    uv = b % 65536
    u = (uv >> 8).astype(np.uint8)
    v = (uv & 255).astype(np.uint8)
    g = b // 65536
    y = np.empty((4096, 4096), dtype=np.uint8)
    y[0::2, 0::2] = 4 * g + 0
    y[0::2, 1::2] = 4 * g + 1
    y[1::2, 0::2] = 4 * g + 2
    y[1::2, 1::2] = 4 * g + 3
    return y, u, v


def exact_real_rgb(y, u, v):
    """Real-valued BT.601 limited range with exact rationals, round half up, clamp.
    Coefficients are computed here from Kr, Kb independently of the oracle."""
    kr, kb = Fraction(299, 1000), Fraction(114, 1000)
    kg = 1 - kr - kb
    s = Fraction(255, 224)
    cs = [Fraction(255, 219), s * 2 * (1 - kr), s * 2 * kb * (1 - kb) / kg,
          s * 2 * kr * (1 - kr) / kg, s * 2 * (1 - kb)]
    den = 1
    for c in cs:
        den = den * c.denominator // np.gcd(den, c.denominator)
    n = [int(c * den) for c in cs]
    H, W = y.shape
    uu = np.repeat(np.repeat(u.astype(np.int64), 2, 0), 2, 1)[:H, :W] - 128
    vv = np.repeat(np.repeat(v.astype(np.int64), 2, 0), 2, 1)[:H, :W] - 128
    yy = y.astype(np.int64) - 16
    chans = [n[0] * yy + n[1] * vv, n[0] * yy - n[2] * uu - n[3] * vv, n[0] * yy + n[4] * uu]
    return np.stack([np.clip((2 * c + den) // (2 * den), 0, 255) for c in chans], -1)


def test_exhaustive_triples_within_one_lsb_of_exact():
    y, u, v = exhaustive_frame()
    # every triple exactly once
    key = (y.astype(np.int64) << 16) | (np.repeat(np.repeat(u, 2, 0), 2, 1).astype(np.int64) << 8) \
        | np.repeat(np.repeat(v, 2, 0), 2, 1)
    assert np.unique(key).size == 1 << 24
    q = C.nv12_to_rgb(y, u, v).astype(np.int64)
    ex = exact_real_rgb(y, u, v)
    d = np.abs(q - ex)
    assert d.max() == 1
    counts = [(d[..., c] != 0).sum() for c in range(3)]
    # counts of 1-LSB differences between Q14 and the exact formula
    assert counts == [18688, 32128, 13824]


def test_grey_axis_and_extremes():
    y = np.arange(256, dtype=np.uint8).reshape(16, 16)
    u = np.full((8, 8), 128, np.uint8)
    v = np.full((8, 8), 128, np.uint8)
    rgb = C.nv12_to_rgb(y, u, v)
    assert (rgb[..., 0] == rgb[..., 1]).all() and (rgb[..., 1] == rgb[..., 2]).all()
    g = rgb[..., 0].ravel()
    assert g[16] == 0 and g[235] == 255 and g[0] == 0 and g[255] == 255
    assert (np.diff(g.astype(int)) >= 0).all()


def test_nv12_split_layout():
    W, H, pitch = 6, 4, 8
    fr = np.zeros((H * 3 // 2, pitch), np.uint8)
    fr[:H, :W] = 10
    fr[H:, 0:W:2] = 20   # U
    fr[H:, 1:W:2] = 30   # V
    fr[:, W:] = 99       # padding never read
    y, u, v = C.split_nv12(fr, W, H)
    assert y.shape == (4, 6) and u.shape == (2, 3) and v.shape == (2, 3)
    assert (y == 10).all() and (u == 20).all() and (v == 30).all()


def test_resize_identity_half_and_constant():
    rng = np.random.default_rng(0)
    img = rng.integers(0, 256, (12, 18, 3), dtype=np.uint8)
    assert np.array_equal(C.resize_bilinear_q8(img, 18, 12), img)
    half = C.resize_bilinear_q8(img, 9, 6).astype(np.int64)
    s = img.astype(np.int64)
    mean = (s[0::2, 0::2] + s[0::2, 1::2] + s[1::2, 0::2] + s[1::2, 1::2] + 2) >> 2
    assert np.array_equal(half, mean)
    const = np.full((7, 11), 77, np.uint8)
    for ow, oh in [(3, 5), (11, 7), (22, 14), (5, 2), (1, 1)]:
        assert (C.resize_bilinear_q8(const, ow, oh) == 77).all()


def test_resize_upscale_linear_ramp():
    # a horizontal ramp upscaled 2x: interior samples sit at quarter positions
    img = (np.arange(8, dtype=np.uint8) * 32).reshape(1, 8).repeat(2, 0)
    up = C.resize_bilinear_q8(img, 16, 4).astype(int)
    # output x maps to source (x + 0.5)/2 - 0.5; ramp slope 32 -> expected 32*src, rounded half up
    xs = (np.arange(16) + 0.5) / 2 - 0.5
    exp = np.floor(np.clip(xs, 0, 7) * 32 + 0.5).astype(int)
    assert np.array_equal(up[0], exp)


@pytest.mark.parametrize("W,H", [(2, 2), (4, 2), (6, 4), (16, 16)])
def test_hist_bruteforce_intervals(W, H):
    rng = np.random.default_rng(W * 100 + H)
    for _ in range(8):
        rgb = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
        h = C.hist16(rgb)
        brute = np.zeros((3, 16), np.int64)
        for yy, xx, c in itertools.product(range(H), range(W), range(3)):
            val = int(rgb[yy, xx, c])
            for k in range(16):
                if 16 * k <= val < 16 * k + 16:
                    brute[c, k] += 1
        assert np.array_equal(h, brute)
        assert (h.sum(1) == W * H).all()


def test_hist_all_codes_hit_all_bins():
    rgb = np.stack([np.arange(256, dtype=np.uint8)] * 3, -1).reshape(16, 16, 3)
    h = C.hist16(rgb)
    assert (h == 16).all()
