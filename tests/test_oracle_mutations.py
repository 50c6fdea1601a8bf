"""Mutation check of the Horn-Schunck oracle's pins (CPU only).

Each case plants one plausible mistake in the oracle (a module attribute
replaced for the duration of the test) and runs the pin that is meant to
catch it: the pin must fail.  This shows that the pins constrain the oracle
at the places where a reading of the method could silently go wrong (border
handling, coordinate conventions, signs, weights), not only in the
interior."""
import numpy as np
import pytest

from oracle import hs
from tests import test_oracle_hs as pins

_orig = {name: getattr(hs, name) for name in
         ["blur5", "pyr_down", "dx", "dy", "bilinear", "upsample_flow", "neighbour_avg", "level_setup", "jacobi"]}


def _blur_pad(mode):
    def blur5(img):
        k = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0
        H, W = img.shape
        p = np.pad(img, ((0, 0), (2, 2)), mode=mode)
        h = sum(k[i] * p[:, i:i + W] for i in range(5))
        p = np.pad(h, ((2, 2), (0, 0)), mode=mode)
        return sum(k[i] * p[i:i + H, :] for i in range(5))
    return blur5


def _dx_pad(mode, scale=0.5):
    def dx(img):
        p = np.pad(img, ((0, 0), (1, 1)), mode=mode)
        return (p[:, 2:] - p[:, :-2]) * scale
    return dx


def _dy_pad(mode):
    def dy(img):
        p = np.pad(img, ((1, 1), (0, 0)), mode=mode)
        return (p[2:, :] - p[:-2, :]) / 2.0
    return dy


def _dx_one_sided(img):
    p = np.pad(img, ((0, 0), (0, 1)), mode="edge")
    return p[:, 1:] - p[:, :-1]


def _upsample_half_pixel(f_coarse, H, W):
    xs, ys = hs.grid(H, W)
    return 2.0 * hs.bilinear(f_coarse, (xs + 0.5) / 2.0 - 0.5, (ys + 0.5) / 2.0 - 0.5)


def _upsample_no_scale(f_coarse, H, W):
    xs, ys = hs.grid(H, W)
    return hs.bilinear(f_coarse, xs / 2.0, ys / 2.0)


def _bilinear_variant(swap=False, clamp=True, corner=True):
    def bilinear(img, X, Y):
        H, W = img.shape
        if clamp:
            X = np.clip(X, 0.0, W - 1.0)
            Y = np.clip(Y, 0.0, H - 1.0)
        x0 = np.floor(X).astype(np.int64)
        y0 = np.floor(Y).astype(np.int64)
        x1 = np.minimum(x0 + 1, W - 1) if corner else x0
        y1 = np.minimum(y0 + 1, H - 1)
        fx = X - x0
        fy = Y - y0
        if swap:
            fx = 1.0 - fx
        top = (1.0 - fx) * img[y0 % H, x0 % W] + fx * img[y0 % H, x1 % W]
        bot = (1.0 - fx) * img[y1 % H, x0 % W] + fx * img[y1 % H, x1 % W]
        return (1.0 - fy) * top + fy * bot
    return bilinear


def _neighbour_equal_weights(f):
    H, W = f.shape
    p = np.pad(f, 1, mode="edge")
    edge = p[0:H, 1:W + 1] + p[2:H + 2, 1:W + 1] + p[1:H + 1, 0:W] + p[1:H + 1, 2:W + 2]
    diag = p[0:H, 0:W] + p[0:H, 2:W + 2] + p[2:H + 2, 0:W] + p[2:H + 2, 2:W + 2]
    return (edge + diag) / 8.0


def _setup_variant(kind):
    def level_setup(I1, I2, u0, v0):
        I2w = hs.warp(I2, u0, v0)
        Ix = 0.5 * (hs.dx(I1) + hs.dx(I2w))
        Iy = 0.5 * (hs.dy(I1) + hs.dy(I2w))
        if kind == "no_average":
            Ix, Iy = hs.dx(I1), hs.dy(I1)
        if kind == "swap":
            Ix, Iy = Iy, Ix
        It = I2w - I1
        if kind == "it_sign":
            It = -It
        Itp = It - Ix * u0 - Iy * v0
        if kind == "lin_sign":
            Itp = It + Ix * u0 + Iy * v0
        return Ix, Iy, Itp
    return level_setup


def _jacobi_wrong_denominator(u, v, Ix, Iy, Itp, alpha, iters):
    den = alpha + Ix * Ix + Iy * Iy
    for _ in range(iters):
        ub = hs.neighbour_avg(u)
        vb = hs.neighbour_avg(v)
        t = (Ix * ub + Iy * vb + Itp) / den
        u = ub - Ix * t
        v = vb - Iy * t
    return u, v


def _pyr_odd(img):
    return hs.blur5(img)[1::2, 1::2]


CASES = [
    # (mistake, oracle attribute, replacement, pins that must fail)
    ("blur zero padding", "blur5", _blur_pad("constant"), ["test_blur_clamps_to_edge_at_the_border"]),
    ("blur periodic padding", "blur5", _blur_pad("wrap"), ["test_blur_clamps_to_edge_at_the_border"]),
    ("blur mirrored padding", "blur5", _blur_pad("reflect"), ["test_blur_clamps_to_edge_at_the_border",
                                                              "test_pyr_down_keeps_even_samples_of_the_clamped_blur"]),
    ("odd-sample decimation", "pyr_down", _pyr_odd, ["test_pyr_down_keeps_even_samples_of_the_clamped_blur",
                                                     "test_pyramid_sizes_and_even_samples"]),
    ("dx zero padding", "dx", _dx_pad("constant"), ["test_central_differences_are_half_one_sided_at_the_border"]),
    ("dx periodic padding", "dx", _dx_pad("wrap"), ["test_central_differences_are_half_one_sided_at_the_border"]),
    ("dx missing 1/2", "dx", _dx_pad("edge", 1.0), ["test_central_differences_are_half_one_sided_at_the_border",
                                                    "test_level_setup_linear_ramp"]),
    ("dx one-sided difference", "dx", _dx_one_sided, ["test_central_differences_are_half_one_sided_at_the_border"]),
    ("dy zero padding", "dy", _dy_pad("constant"), ["test_central_differences_are_half_one_sided_at_the_border"]),
    ("upsample half-pixel centres", "upsample_flow", _upsample_half_pixel,
     ["test_upsample_flow_samples_the_coarse_grid_at_half_coordinates"]),
    ("upsample without x2", "upsample_flow", _upsample_no_scale,
     ["test_upsample_flow_samples_the_coarse_grid_at_half_coordinates",
      "test_integer_warp_is_exact_shift_and_upsample_constant"]),
    ("bilinear swapped weights", "bilinear", _bilinear_variant(swap=True),
     ["test_bilinear_is_exact_on_bilinear_functions_and_clamps"]),
    ("bilinear without clamp", "bilinear", _bilinear_variant(clamp=False),
     ["test_bilinear_is_exact_on_bilinear_functions_and_clamps"]),
    ("bilinear wrong corner", "bilinear", _bilinear_variant(corner=False),
     ["test_bilinear_is_exact_on_bilinear_functions_and_clamps"]),
    ("equal neighbour weights", "neighbour_avg", _neighbour_equal_weights,
     ["test_jacobi_fixed_point_equals_sparse_solve"]),
    ("gradients of I1 only", "level_setup", _setup_variant("no_average"), ["test_level_setup_linear_ramp"]),
    ("Ix and Iy swapped", "level_setup", _setup_variant("swap"), ["test_level_setup_linear_ramp"]),
    ("It sign", "level_setup", _setup_variant("it_sign"), ["test_translation_recovery_noise_free_and_sign"]),
    ("linearisation sign", "level_setup", _setup_variant("lin_sign"), ["test_level_setup_linear_ramp"]),
    ("alpha instead of alpha^2", "jacobi", _jacobi_wrong_denominator,
     ["test_jacobi_fixed_point_equals_sparse_solve"]),
]


@pytest.mark.parametrize("mistake,attr,repl,must_fail", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_fails_its_pins(monkeypatch, mistake, attr, repl, must_fail):
    monkeypatch.setattr(hs, attr, repl)
    for name in must_fail:
        with pytest.raises((AssertionError, IndexError)):
            getattr(pins, name)()


def test_pins_pass_on_the_unmodified_oracle():
    for attr, fn in _orig.items():
        assert getattr(hs, attr) is fn
    names = sorted({n for c in CASES for n in c[3]})
    for name in names:
        getattr(pins, name)()
