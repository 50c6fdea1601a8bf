"""Pins of the Horn-Schunck oracle against what the mathematics fixes: exact
zeros, known sub-pixel translations, symmetries, a sparse direct solve of the
Horn-Schunck normal equations, the binomial impulse response, exact integer
warps and constant upsampling."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import hs


def _c1_frames(noise=2.0, n=16):
    s, ds = synth.translation_scene(1, 320, 240, n, noise_sigma=noise)
    return [s.nv12(t).numpy()[:240] for t in range(n)], ds


def test_identical_and_constant_frames_give_exact_zero():
    fr, _ = _c1_frames(n=2)
    u, v = hs.hs_flow(fr[0], fr[0], levels=3, alpha=10.0, iters=50)
    assert (u == 0).all() and (v == 0).all()
    c = np.full((37, 53), 91, np.uint8)
    u, v = hs.hs_flow(c, c, levels=3)
    assert (u == 0).all() and (v == 0).all()


def test_translation_recovery_c1():
    fr, ds = _c1_frames()
    m = 16
    for t in range(15):
        u, v = hs.hs_flow(fr[t], fr[t + 1], levels=3, alpha=10.0, iters=50)
        ui, vi = u[m:-m, m:-m], v[m:-m, m:-m]
        dxt, dyt = ds[t]
        assert abs(ui.mean() - dxt) < 0.03 and abs(vi.mean() - dyt) < 0.03
        e = np.hypot(ui - dxt, vi - dyt)
        assert np.percentile(e, 95) < 0.35


def test_translation_recovery_noise_free_and_sign():
    s, ds = synth.translation_scene(1, 320, 240, 6, noise_sigma=0.0)
    m = 16
    for t in range(5):
        a = s.nv12(t).numpy()[:240]
        b = s.nv12(t + 1).numpy()[:240]
        u, v = hs.hs_flow(a, b, levels=3)
        e = np.hypot(u[m:-m, m:-m] - ds[t][0], v[m:-m, m:-m] - ds[t][1])
        assert np.percentile(e, 95) < 0.15
        # sign: content moving by +d gives +d; reversing the pair gives -d
        u2, v2 = hs.hs_flow(b, a, levels=3)
        assert np.sign(u2[m:-m, m:-m].mean()) == -np.sign(ds[t][0]) or abs(ds[t][0]) < 0.05


def test_transpose_swaps_components():
    fr, _ = _c1_frames(n=3)
    a, b = fr[1][:96, :128], fr[2][:96, :128]
    u, v = hs.hs_flow(a, b, levels=3)
    ut, vt = hs.hs_flow(a.T.copy(), b.T.copy(), levels=3)
    assert np.abs(ut - v.T).max() < 1e-9 and np.abs(vt - u.T).max() < 1e-9


def test_single_level_mirror_negates_u():
    fr, _ = _c1_frames(n=3)
    a, b = fr[0][:64, :90], fr[1][:64, :90]
    u, v = hs.hs_flow(a, b, levels=1)
    um, vm = hs.hs_flow(a[:, ::-1].copy(), b[:, ::-1].copy(), levels=1)
    assert np.abs(um + u[:, ::-1]).max() < 1e-9 and np.abs(vm - v[:, ::-1]).max() < 1e-9


def test_level_setup_linear_ramp():
    # I1 = 3x + 2y; I2 is I1 moved by (+2, +1); starting flow (2, 1) warps I2 back onto I1
    H, W = 20, 30
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    I1 = 3 * xs + 2 * ys
    I2 = 3 * (xs - 2) + 2 * (ys - 1)
    u0 = np.full((H, W), 2.0)
    v0 = np.full((H, W), 1.0)
    Ix, Iy, Itp = hs.level_setup(I1, I2, u0, v0)
    inner = (slice(2, H - 3), slice(2, W - 4))
    assert np.allclose(Ix[inner], 3.0) and np.allclose(Iy[inner], 2.0)
    assert np.allclose(Itp[inner], -3.0 * 2 - 2.0 * 1)
    # frames with different slopes (I2 = 5x - y + 7, no start flow): the
    # gradients are the means of the two frames' slopes, (3 + 5)/2 and
    # (2 - 1)/2, and It = I2 - I1 = 2x - 3y + 7 (catches gradients taken
    # from one frame only)
    J2 = 5 * xs - ys + 7
    z = np.zeros((H, W))
    Jx, Jy, Jt = hs.level_setup(I1, J2, z, z)
    inner = (slice(1, H - 1), slice(1, W - 1))
    assert np.allclose(Jx[inner], 4.0) and np.allclose(Jy[inner], 0.5)
    assert np.allclose(Jt, 2 * xs - 3 * ys + 7)


def _neighbour_matrix(H, W):
    """Sparse operator of the clamp-to-edge 3x3 Horn-Schunck neighbour average."""
    rows, cols, vals = [], [], []
    for y in range(H):
        for x in range(W):
            i = y * W + x
            for dy_, dx_ in [(-1, 0), (1, 0), (0, -1), (0, 1), (-1, -1), (-1, 1), (1, -1), (1, 1)]:
                w = 1 / 6 if dy_ == 0 or dx_ == 0 else 1 / 12
                yy = min(max(y + dy_, 0), H - 1)
                xx = min(max(x + dx_, 0), W - 1)
                rows.append(i)
                cols.append(yy * W + xx)
                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(H * W, H * W))


def test_jacobi_fixed_point_equals_sparse_solve():
    H, W, alpha = 16, 24, 10.0
    rng = np.random.default_rng(5)
    Ix = rng.normal(0, 8, (H, W))
    Iy = rng.normal(0, 8, (H, W))
    It = rng.normal(0, 5, (H, W))
    A = _neighbour_matrix(H, W)
    n = H * W
    I = sp.identity(n)
    a2 = alpha * alpha
    # Euler-Lagrange of the Horn-Schunck energy with the discrete Laplacian (ubar - u):
    # alpha^2 (u - ubar) + Ix (Ix u + Iy v + It) = 0, and the v analogue
    Kuu = a2 * (I - A) + sp.diags(Ix.ravel() ** 2)
    Kuv = sp.diags((Ix * Iy).ravel())
    Kvv = a2 * (I - A) + sp.diags(Iy.ravel() ** 2)
    K = sp.bmat([[Kuu, Kuv], [Kuv, Kvv]]).tocsc()
    rhs = -np.concatenate([(Ix * It).ravel(), (Iy * It).ravel()])
    sol = spla.spsolve(K, rhs)
    u, v = hs.jacobi(np.zeros((H, W)), np.zeros((H, W)), Ix, Iy, It, alpha, 20000)
    assert np.abs(u.ravel() - sol[:n]).max() < 1e-9
    assert np.abs(v.ravel() - sol[n:]).max() < 1e-9


def test_blur_impulse_response():
    img = np.zeros((11, 13))
    img[5, 6] = 1.0
    b = hs.blur5(img)
    k = np.array([1, 4, 6, 4, 1], float)
    assert np.allclose(b[3:8, 4:9], np.outer(k, k) / 256.0, atol=0, rtol=0)
    assert b.sum() == pytest.approx(1.0)


def test_pyramid_sizes_and_even_samples():
    assert hs.level_sizes(1920, 1080, 4) == [(1920, 1080), (960, 540), (480, 270), (240, 135)]
    assert hs.level_sizes(320, 240, 3)[-1] == (80, 60)
    assert hs.level_sizes(2048, 2048, 5)[-1] == (128, 128)
    img = np.random.default_rng(1).normal(size=(9, 7))
    p = hs.pyramid(img, 3)
    assert [q.shape for q in p] == [(9, 7), (5, 4), (3, 2)]
    assert np.array_equal(p[1], hs.blur5(img)[0::2, 0::2])


def test_integer_warp_is_exact_shift_and_upsample_constant():
    img = np.random.default_rng(2).normal(size=(20, 25))
    w = hs.warp(img, np.full(img.shape, 3.0), np.full(img.shape, -2.0))
    assert np.array_equal(w[2:, :-3], img[:-2, 3:])
    up = hs.upsample_flow(np.full((5, 7), 1.25), 10, 13)
    assert (up == 2.5).all()


# ---------------------------------------------------------------------------
# Border and coordinate conventions (steps 2, 4, 5, 6 of the oracle header),
# each pinned by values worked out by hand from the definition.  Every test
# names the plausible mistake it catches; tests/test_oracle_mutations.py
# plants each of those mistakes in the oracle and checks that the pin fails.


def test_blur_clamps_to_edge_at_the_border():
    """Catches zero (or periodic, or mirrored) padding in blur5.

    An impulse in the corner: clamp-to-edge replicates it twice outside the
    image in each axis, so the 1-D response at x = 0, 1, 2 is
    (1 + 4 + 6, 1 + 4, 1) / 16 = (11, 5, 1) / 16, and the corner of the 2-D
    response is their outer product (zero padding would give (6, 4, 1)/16)."""
    img = np.zeros((9, 11))
    img[0, 0] = 1.0
    b = hs.blur5(img)
    k = np.array([11.0, 5.0, 1.0]) / 16.0
    assert np.array_equal(b[:3, :3], np.outer(k, k))
    assert (b[3:, :] == 0).all() and (b[:, 3:] == 0).all()
    # a ramp f(x) = x: the symmetric kernel keeps it in the interior; at the
    # left edge the clamped taps read f(0) twice: (0 + 0 + 0 + 4*1 + 2)/16,
    # and at x = 1: (0 + 4*0 + 6*1 + 4*2 + 3)/16; at the right edge (x = 10)
    # (8 + 4*9 + 6*10 + 4*10 + 10)/16
    ramp = np.tile(np.arange(11.0), (7, 1))
    br = hs.blur5(ramp)
    assert np.array_equal(br[:, 2:9], ramp[:, 2:9])
    assert (br[:, 0] == 6.0 / 16).all() and (br[:, 1] == 17.0 / 16).all()
    assert (br[:, 10] == 154.0 / 16).all()
    # the vertical pass clamps the same way (a ramp in y)
    bt = hs.blur5(ramp.T.copy())
    assert np.array_equal(bt, br.T)


def test_pyr_down_keeps_even_samples_of_the_clamped_blur():
    """Catches odd-sample decimation and unclamped borders in pyr_down.

    A 1-D ramp x on 5 columns: coarse samples sit at fine x = 0, 2, 4; the
    clamped blur there is 6/16, 2 and (2 + 4*3 + 6*4 + 4*4 + 4)/16 = 58/16."""
    ramp = np.tile(np.arange(5.0), (4, 1))
    p = hs.pyr_down(ramp)
    assert p.shape == (2, 3)
    assert np.array_equal(p, np.tile([6.0 / 16, 2.0, 58.0 / 16], (2, 1)))


def test_central_differences_are_half_one_sided_at_the_border():
    """Catches zero or periodic padding (and a missing 1/2) in dx / dy.

    I(x) = x^2 + 5: in the interior (I(x+1) - I(x-1))/2 = 2x; at x = 0 the
    clamped left neighbour is I(0), giving (I(1) - I(0))/2 = 1/2; at the last
    column x = W-1, (I(W-1) - I(W-2))/2 = (2W - 3)/2.  Zero padding would
    give (6 - 0)/2 at x = 0, periodic padding (I(1) - I(W-1))/2."""
    W = 9
    f = np.arange(W, dtype=np.float64) ** 2 + 5.0
    img = np.tile(f, (4, 1))
    d = hs.dx(img)
    exp = np.concatenate([[0.5], 2.0 * np.arange(1, W - 1), [(2 * W - 3) / 2.0]])
    assert np.array_equal(d, np.tile(exp, (4, 1)))
    assert (hs.dy(img) == 0).all()
    dyv = hs.dy(img.T.copy())
    assert np.array_equal(dyv, d.T)


def test_upsample_flow_samples_the_coarse_grid_at_half_coordinates():
    """Catches half-pixel centres ((x + 0.5)/2 - 0.5) and a missing clamp in
    upsample_flow.

    Coarse sample k sits at fine coordinate 2k, so a coarse ramp f(k) = k
    upsamples to u(x) = 2 * (x / 2) = x until x/2 passes the last coarse
    sample, and 2 * (Wc - 1) after it; likewise in y."""
    Wc, Hc, W, H = 6, 4, 12, 7
    ramp_x = np.tile(np.arange(Wc, dtype=np.float64), (Hc, 1))
    up = hs.upsample_flow(ramp_x, H, W)
    exp = 2.0 * np.minimum(np.arange(W) / 2.0, Wc - 1.0)
    assert np.array_equal(up, np.tile(exp, (H, 1)))
    ramp_y = np.tile(np.arange(Hc, dtype=np.float64)[:, None], (1, Wc))
    upy = hs.upsample_flow(ramp_y, H, W)
    expy = 2.0 * np.minimum(np.arange(H) / 2.0, Hc - 1.0)
    assert np.array_equal(upy, np.tile(expy[:, None], (1, W)))


def test_bilinear_is_exact_on_bilinear_functions_and_clamps():
    """Catches swapped or mirrored interpolation weights, a wrong corner, and a
    missing or wrong clamp in bilinear.

    Bilinear interpolation reproduces every function in span{1, x, y, xy}
    exactly, so sampling f = 2 + 3x - 5y + 0.25xy at fractional points inside
    the image gives f there; points outside sample f at the clamped
    coordinates."""
    H, W = 7, 9
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)

    def f(x, y):
        return 2.0 + 3.0 * x - 5.0 * y + 0.25 * x * y

    img = f(xs, ys)
    rng = np.random.default_rng(11)
    X = rng.uniform(-3.0, W + 2.0, 400)
    Y = rng.uniform(-3.0, H + 2.0, 400)
    got = hs.bilinear(img, X, Y)
    exp = f(np.clip(X, 0, W - 1), np.clip(Y, 0, H - 1))
    assert np.abs(got - exp).max() < 1e-12
    # exactly on the last row/column the upper neighbour is the sample itself
    assert hs.bilinear(img, np.array([W - 1.0]), np.array([H - 1.0]))[0] == img[H - 1, W - 1]
    # a warp by a fractional constant flow is a fractional shift of the ramp
    w = hs.warp(img, np.full(img.shape, 0.25), np.full(img.shape, -0.5))
    inner = (slice(1, H), slice(0, W - 1))
    assert np.abs(w[inner] - f(xs + 0.25, ys - 0.5)[inner]).max() < 1e-12
