"""Pins of the Farnebäck oracle (CPU only): values fixed by the mathematics
of polynomial expansion and of the displacement estimate, independent
solvers, symmetries, and a mutation check that plants one mistake at a
time in the oracle and shows that some pin fails."""
import math

import numpy as np
import pytest

import synth
from oracle import farneback as F
from oracle import hs as H

N, SIGMA, M, LAM = F.POLY_N, F.POLY_SIGMA, F.WIN, F.LAMBDA


def _quadratic(h, w, A, b, c, shift=(0.0, 0.0)):
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    x = xs - shift[0]
    y = ys - shift[1]
    return A[0][0] * x * x + 2 * A[0][1] * x * y + A[1][1] * y * y + b[0] * x + b[1] * y + c


def _textured(seed, w=96, h=72):
    s, _ = synth.translation_scene(seed, w, h, 2)
    return [s.nv12(t).numpy()[:h].astype(np.float64) for t in range(2)]


# --- polynomial expansion ---------------------------------------------------

def test_applicability_values():
    """a(t) = exp(-|t|^2 / (2 sigma^2)) with sigma = 1.1, by hand: a(1,0) =
    exp(-1/2.42), a(2,0) = exp(-4/2.42), a(1,1) = exp(-2/2.42), a(2,2) =
    exp(-8/2.42); row-major order over t in {-2..2}^2."""
    a = F.applicability().reshape(5, 5)
    assert a[2, 2] == 1.0
    assert abs(a[2, 3] - 0.6615147) < 1e-6 and abs(a[3, 2] - 0.6615147) < 1e-6
    assert abs(a[2, 4] - 0.1914952) < 1e-6
    assert abs(a[3, 3] - 0.4376016) < 1e-6
    assert abs(a[0, 0] - 0.0366704) < 1e-6


def test_expansion_exact_on_quadratics():
    """Every pixel whose window stays inside the image recovers the quadratic's
    A, its gradient 2 A x + b (the local linear term) and its value."""
    rng = np.random.default_rng(1)
    for _ in range(3):
        A = rng.normal(0, 0.3, (2, 2))
        A = (A + A.T) / 2
        b = rng.normal(0, 2, 2)
        c = rng.normal(0, 10)
        f = _quadratic(30, 41, A, b, c)
        A11, A22, A12, b1, b2 = F.coeffs(F.poly_exp(f))
        r0 = F.poly_exp(f)[0]
        ys, xs = np.mgrid[0:30, 0:41].astype(np.float64)
        i = (slice(N, -N), slice(N, -N))
        assert np.abs(A11[i] - A[0, 0]).max() < 1e-9
        assert np.abs(A22[i] - A[1, 1]).max() < 1e-9
        assert np.abs(A12[i] - A[0, 1]).max() < 1e-9
        assert np.abs(b1[i] - (2 * A[0, 0] * xs + 2 * A[0, 1] * ys + b[0])[i]).max() < 1e-9
        assert np.abs(b2[i] - (2 * A[0, 1] * xs + 2 * A[1, 1] * ys + b[1])[i]).max() < 1e-9
        assert np.abs(r0[i] - f[i]).max() < 1e-8


def test_expansion_equals_per_pixel_weighted_lstsq_with_clamped_windows():
    """On a random 7 x 9 image the expansion of every pixel, borders included,
    equals numpy's least-squares solve of the weighted system built with
    explicit loops over the clamped window."""
    rng = np.random.default_rng(2)
    img = rng.uniform(0, 255, (7, 9))
    r = F.poly_exp(img)
    s2 = 2 * SIGMA * SIGMA
    for y in range(7):
        for x in range(9):
            rows, vals = [], []
            for ty in range(-N, N + 1):
                for tx in range(-N, N + 1):
                    wgt = math.sqrt(math.exp(-(tx * tx + ty * ty) / s2))
                    yy = min(max(y + ty, 0), 6)
                    xx = min(max(x + tx, 0), 8)
                    rows.append([wgt * v for v in (1, tx, ty, tx * tx, ty * ty, tx * ty)])
                    vals.append(wgt * img[yy, xx])
            sol = np.linalg.lstsq(np.array(rows), np.array(vals), rcond=None)[0]
            assert np.abs(sol - r[:, y, x]).max() < 1e-8 * max(1.0, np.abs(sol).max()), (y, x)


def test_box_mean_equals_explicit_clamped_loops():
    rng = np.random.default_rng(3)
    img = rng.normal(0, 1, (6, 11))
    got = F.box_mean(img, 2)
    for y in range(6):
        for x in range(11):
            s = 0.0
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    s += img[min(max(y + dy, 0), 5), min(max(x + dx, 0), 10)]
            assert abs(got[y, x] - s / 25.0) < 1e-12


# --- displacement estimate ----------------------------------------------------

def _quad_pair(d, A=((0.02, 0.006), (0.006, 0.015)), b=(0.7, -0.4), c=90.0, h=64, w=80):
    A = np.array(A)
    return _quadratic(h, w, A, b, c), _quadratic(h, w, A, b, c, shift=d), A


@pytest.mark.parametrize("d", [(0.6, -0.3), (-1.7, 2.2)])
def test_translated_quadratic_closed_form(d):
    """f2(x) = f1(x - d) with f1 quadratic: then A2 = A1 and b2 = b1 - 2 A1 d,
    so the constraint is A1 d = db exactly and the estimate is
    (A1'A1 + lambda I)^-1 A1'A1 d at every pixel whose expansions and box
    window are exact (margin n + m, plus the displacement)."""
    f1, f2, A = _quad_pair(d)
    z = np.zeros_like(f1)
    u, v = F.displacement(F.poly_exp(f1), F.poly_exp(f2), z, z)
    G = A.T @ A
    exp = np.linalg.solve(G + LAM * np.eye(2), G @ np.array(d))
    g = N + M + 3
    i = (slice(g, -g), slice(g, -g))
    assert np.abs(u[i] - exp[0]).max() < 1e-9
    assert np.abs(v[i] - exp[1]).max() < 1e-9


def test_iterations_keep_the_quadratic_solution():
    """On the translated quadratic the constraint does not depend on the prior
    (b2 at x + d~ is 2 A (x + d~ - d) + b, and A d~ cancels it), so every
    further iteration returns the same estimate."""
    d = (1.3, 0.8)
    f1, f2, A = _quad_pair(d)
    r1, r2 = F.poly_exp(f1), F.poly_exp(f2)
    z = np.zeros_like(f1)
    u1, v1 = F.displacement(r1, r2, z, z)
    u2, v2 = F.displacement(r1, r2, u1, v1)
    u3, v3 = F.displacement(r1, r2, u2, v2)
    g = N + M + 4
    i = (slice(g, -g), slice(g, -g))
    assert np.abs(u3[i] - u1[i]).max() < 1e-9 and np.abs(v3[i] - v1[i]).max() < 1e-9


def test_one_step_is_antisymmetric_in_the_frames():
    """From a zero prior, swapping the frames leaves A = (A1 + A2)/2 and
    negates db, so the estimate changes sign exactly (textured frames, whose
    A fields differ)."""
    a, b = _textured(4)
    ra, rb = F.poly_exp(a), F.poly_exp(b)
    z = np.zeros_like(a)
    u1, v1 = F.displacement(ra, rb, z, z)
    u2, v2 = F.displacement(rb, ra, z, z)
    assert np.abs(u1 + u2).max() < 1e-12 and np.abs(v1 + v2).max() < 1e-12
    assert np.abs(u1).max() > 0.01


def test_identical_and_constant_frames_give_zero():
    a, _ = _textured(5)
    u, v = F.fb_flow(a, a, levels=3)
    assert (u == 0).all() and (v == 0).all()
    c = np.full((48, 64), 77.0)
    u, v = F.fb_flow(c, c + 0.0, levels=2)
    assert np.abs(u).max() == 0 and np.abs(v).max() == 0


def test_subpixel_translations_recovered():
    """Seeded band-limited textures translated by known sub-pixel shifts
    (320 x 240, noise sigma = 2, 3 levels): the interior mean recovers the
    shift within 0.02 px and 95% of the interior pixels within 0.2 px."""
    sc, ds = synth.translation_scene(1, 320, 240, 4)
    fr = [sc.nv12(t).numpy()[:240] for t in range(4)]
    m = (slice(16, -16), slice(16, -16))
    for t in range(3):
        u, v = F.fb_flow(fr[t], fr[t + 1], levels=3)
        assert abs(u[m].mean() - ds[t][0]) < 0.02 and abs(v[m].mean() - ds[t][1]) < 0.02
        assert np.quantile(np.hypot(u[m] - ds[t][0], v[m] - ds[t][1]), 0.95) < 0.2


def test_transpose_swaps_u_and_v():
    a, b = _textured(6)
    u, v = F.fb_flow(a, b, levels=2)
    ut, vt = F.fb_flow(a.T.copy(), b.T.copy(), levels=2)
    assert np.abs(ut - v.T).max() < 1e-9 and np.abs(vt - u.T).max() < 1e-9


def test_single_level_mirror_negates_u():
    a, b = _textured(7)
    u, v = F.fb_flow(a, b, levels=1)
    um, vm = F.fb_flow(a[:, ::-1].copy(), b[:, ::-1].copy(), levels=1)
    assert np.abs(um + u[:, ::-1]).max() < 1e-9 and np.abs(vm - v[:, ::-1]).max() < 1e-9


# --- mutation check ------------------------------------------------------------

def _m_coeffs_full_a12(r):
    return r[3], r[4], r[5], r[1], r[2]


def _m_applicability_sigma2(n=N, sigma=SIGMA):
    tx, ty, _ = F.basis(n)
    return np.exp(-(tx * tx + ty * ty) / (sigma * sigma))


def _m_basis_swapped(n=N):
    tx, ty, B = F._orig_basis(n)
    return tx, ty, B[:, [0, 1, 2, 4, 3, 5]]


def _m_box_zero_pad(img, m=M):
    Hh, W = img.shape
    k = 2 * m + 1
    p = np.pad(img, ((0, 0), (m, m)))
    rows = sum(p[:, i:i + W] for i in range(k))
    p = np.pad(rows, ((m, m), (0, 0)))
    return sum(p[i:i + Hh, :] for i in range(k)) / float(k * k)


def _m_poly_zero_pad(img, n=N, sigma=SIGMA):
    Hh, W = img.shape
    tx, ty, B = F.basis(n)
    a = F.applicability(n, sigma)
    p = np.pad(img.astype(np.float64), n)
    Fs = np.stack([p[n + int(dy):n + int(dy) + Hh, n + int(dx):n + int(dx) + W] for dx, dy in zip(tx, ty)])
    G = B.T @ (a[:, None] * B)
    return np.linalg.solve(G, (B * a[:, None]).T @ Fs.reshape(len(a), -1)).reshape(6, Hh, W)


def _displacement_variant(sign_db=-0.5, prior_term=True, average=True, warp_sign=1.0, det_plus=False,
                          lam_both=True):
    def displacement(r1, r2, du, dv, m=M, lam=LAM):
        A11a, A22a, A12a, b1a, b2a = F.coeffs(r1)
        Hh, W = du.shape
        xs, ys = H.grid(Hh, W)
        X, Y = xs + warp_sign * du, ys + warp_sign * dv
        A11b, A22b, A12b, b1b, b2b = (H.bilinear(q, X, Y) for q in F.coeffs(r2))
        if average:
            A11, A22, A12 = 0.5 * (A11a + A11b), 0.5 * (A22a + A22b), 0.5 * (A12a + A12b)
        else:
            A11, A22, A12 = A11a, A22a, A12a
        db1 = sign_db * (b1b - b1a) + ((A11 * du + A12 * dv) if prior_term else 0.0)
        db2 = sign_db * (b2b - b2a) + ((A12 * du + A22 * dv) if prior_term else 0.0)
        G11 = A11 * A11 + A12 * A12
        G12 = A11 * A12 + A12 * A22
        G22 = A12 * A12 + A22 * A22
        h1 = A11 * db1 + A12 * db2
        h2 = A12 * db1 + A22 * db2
        G11, G12, G22, h1, h2 = (F.box_mean(q, m) for q in (G11, G12, G22, h1, h2))
        G11 = G11 + lam
        G22 = G22 + (lam if lam_both else 0.0)
        det = G11 * G22 + G12 * G12 if det_plus else G11 * G22 - G12 * G12
        return (G22 * h1 - G12 * h2) / det, (G11 * h2 - G12 * h1) / det
    return displacement


_PINS = [test_applicability_values, test_expansion_exact_on_quadratics,
         test_expansion_equals_per_pixel_weighted_lstsq_with_clamped_windows,
         test_box_mean_equals_explicit_clamped_loops,
         lambda: test_translated_quadratic_closed_form((0.6, -0.3)), test_iterations_keep_the_quadratic_solution,
         test_one_step_is_antisymmetric_in_the_frames, test_identical_and_constant_frames_give_zero]


@pytest.mark.parametrize("name,attr,fake", [
    ("A12 not halved", "coeffs", _m_coeffs_full_a12),
    ("applicability over sigma^2", "applicability", _m_applicability_sigma2),
    ("basis columns swapped", "basis", _m_basis_swapped),
    ("box sums zero-padded", "box_mean", _m_box_zero_pad),
    ("expansion zero-padded", "poly_exp", _m_poly_zero_pad),
    ("db sign flipped", "displacement", _displacement_variant(sign_db=0.5)),
    ("prior term A d~ dropped", "displacement", _displacement_variant(prior_term=False)),
    ("A of frame 1 only", "displacement", _displacement_variant(average=False)),
    ("warp at x - d~", "displacement", _displacement_variant(warp_sign=-1.0)),
    ("determinant sign", "displacement", _displacement_variant(det_plus=True)),
    ("lambda on one diagonal entry", "displacement", _displacement_variant(lam_both=False)),
])
def test_each_planted_mistake_fails_a_pin(monkeypatch, name, attr, fake):
    if attr == "basis":
        monkeypatch.setattr(F, "_orig_basis", F.basis, raising=False)
    monkeypatch.setattr(F, attr, fake)
    failed = 0
    for pin in _PINS:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed > 0, name
