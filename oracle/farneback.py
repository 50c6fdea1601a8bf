"""Farnebäck optical flow by polynomial expansion, FP64 (oracle; test
infrastructure only).

Scanner's FLOW microbenchmark computes dense optical flow between the frames
of each pair with Farnebäck's method (Sec. 5.1.2; a two-frame stencil
S[0,1], Sec. 3.2).  This module writes out that method as published by
Farnebäck ("Two-frame motion estimation based on polynomial expansion",
SCIA 2003; thesis "Polynomial expansion for orientation and motion
estimation", 2002), in whole-array numpy, with the readings below.  The
flow w = (u, v) of a pair (I1, I2) satisfies I1(x) ~ I2(x + w(x)), in pixels
of the level it is expressed at (the convention of the Horn-Schunck oracle).

1. I = float(Y) of the NV12 luma plane, code values 0..255.
2. Pyramid: the same 2x binomial pyramid as the Horn-Schunck oracle (level
   l+1 keeps the even samples of the separable [1,4,6,4,1]/16 blur of level
   l, clamp-to-edge).  Reading: the method's coarse-to-fine scheme with
   scale factor 1/2 uses this pyramid.
3. Polynomial expansion of each level image: at every pixel x the
   neighbourhood is modelled as f(x + t) ~ t'A t + b't + c, fitted by
   weighted least squares over t in {-n..n}^2 with the Gaussian applicability
   a(t) = exp(-|t|^2 / (2 sigma^2)); basis order 1, tx, ty, tx^2, ty^2,
   tx ty, so c = r1, b = (r2, r3), A = [[r4, r6/2], [r6/2, r5]].  Reading:
   samples outside the image take the value of the nearest pixel
   (clamp-to-edge), so the normal matrix is the same at every pixel.
4. Displacement estimation, repeated `iters` times per level from a prior
   displacement d~ (the coarser level's result upsampled at the first
   iteration, the previous iteration's result after that):
     A2w, b2w = bilinear interpolation of frame 2's A and b at x + d~(x),
                sample coordinates clamped to the image (the Horn-Schunck
                warp convention);
     A  = (A1 + A2w) / 2,   db = -(b2w - b1) / 2 + A d~;
     G  = A'A,  h = A'db  (per pixel);
     Gm, hm = means of G and h over the (2m+1)^2 box around x (values
              outside the image: the nearest pixel's, clamp-to-edge);
     d  = (Gm + lambda I)^-1 hm.
   Reading: the local averaging is a box window; lambda > 0 keeps the 2x2
   system solvable where the window holds no structure (constant image:
   Gm = 0, hm = 0, d = 0).
5. Coarse to fine: the coarsest level starts from d~ = 0; a finer level
   starts from 2 * bilinear(d_coarse, x/2, y/2) (coordinates clamped), the
   Horn-Schunck upsampling convention.
6. Parameters (reading; the paper gives none): n = 2 (5 x 5 expansion),
   sigma = 1.1, m = 7 (15 x 15 averaging), lambda = 1e-3, 3 iterations per
   level; the pyramid depth as for Horn-Schunck (4 levels at 1080p).

Pins (tests): the expansion is exact on quadratic images and equals a
per-pixel weighted least-squares solve (numpy lstsq) everywhere, borders
included; on a translated quadratic the displacement is the closed form
(Gm + lambda I)^-1 Gm d at every interior pixel and further iterations keep
it; identical frames give exactly zero flow, constant frames zero;
sub-pixel translations of band-limited textures are recovered, with the
right sign; transposing both frames swaps u and v; at one level a mirror
negates u; the box mean equals explicit window loops.  A mutation test
plants a mistake in each step and checks that a pin fails.  Parity pinned.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from oracle import hs as _hs

POLY_N = 2
POLY_SIGMA = 1.1
WIN = 7
LAMBDA = 1e-3
ITERS = 3


def basis(n: int = POLY_N) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Window offsets (tx, ty) in row-major order and the basis matrix B
    [(2n+1)^2, 6] with columns 1, tx, ty, tx^2, ty^2, tx ty."""
    ty, tx = np.mgrid[-n:n + 1, -n:n + 1]
    tx = tx.ravel().astype(np.float64)
    ty = ty.ravel().astype(np.float64)
    B = np.stack([np.ones_like(tx), tx, ty, tx * tx, ty * ty, tx * ty], axis=1)
    return tx, ty, B


def applicability(n: int = POLY_N, sigma: float = POLY_SIGMA) -> np.ndarray:
    """Gaussian weights a(t) over the window, row-major."""
    tx, ty, _ = basis(n)
    return np.exp(-(tx * tx + ty * ty) / (2.0 * sigma * sigma))


def poly_exp(img: np.ndarray, n: int = POLY_N, sigma: float = POLY_SIGMA) -> np.ndarray:
    """Weighted least-squares coefficients r[6][H][W] (c, b1, b2, a11, a22, 2 a12)
    of every pixel's clamped (2n+1)^2 neighbourhood."""
    H, W = img.shape
    tx, ty, B = basis(n)
    a = applicability(n, sigma)
    p = np.pad(img.astype(np.float64), n, mode="edge")
    # window samples f(x + t), one row per offset t
    F = np.stack([p[n + int(dy):n + int(dy) + H, n + int(dx):n + int(dx) + W] for dx, dy in zip(tx, ty)])
    G = B.T @ (a[:, None] * B)                      # normal matrix (the same at every pixel)
    rhs = (B * a[:, None]).T @ F.reshape(len(a), -1)  # B' W f per pixel
    r = np.linalg.solve(G, rhs)
    return r.reshape(6, H, W)


def coeffs(r: np.ndarray):
    """(A11, A22, A12, b1, b2) planes from the expansion."""
    return r[3], r[4], 0.5 * r[5], r[1], r[2]


def box_mean(img: np.ndarray, m: int = WIN) -> np.ndarray:
    """Mean over the (2m+1)^2 box around each pixel, clamp-to-edge (the window
    sum of the 2m+1 row neighbours, then of the 2m+1 column neighbours)."""
    H, W = img.shape
    k = 2 * m + 1
    p = np.pad(img, ((0, 0), (m, m)), mode="edge")
    rows = sum(p[:, i:i + W] for i in range(k))
    p = np.pad(rows, ((m, m), (0, 0)), mode="edge")
    return sum(p[i:i + H, :] for i in range(k)) / float(k * k)


def displacement(r1: np.ndarray, r2: np.ndarray, du: np.ndarray, dv: np.ndarray, m: int = WIN,
                 lam: float = LAMBDA) -> Tuple[np.ndarray, np.ndarray]:
    """One displacement estimate from the expansions of both frames and the
    prior displacement (du, dv) (step 4)."""
    A11a, A22a, A12a, b1a, b2a = coeffs(r1)
    H, W = du.shape
    xs, ys = _hs.grid(H, W)
    X, Y = xs + du, ys + dv
    A11b, A22b, A12b, b1b, b2b = (_hs.bilinear(q, X, Y) for q in coeffs(r2))
    A11 = 0.5 * (A11a + A11b)
    A22 = 0.5 * (A22a + A22b)
    A12 = 0.5 * (A12a + A12b)
    db1 = -0.5 * (b1b - b1a) + (A11 * du + A12 * dv)
    db2 = -0.5 * (b2b - b2a) + (A12 * du + A22 * dv)
    # G = A'A and h = A'db (A symmetric)
    G11 = A11 * A11 + A12 * A12
    G12 = A11 * A12 + A12 * A22
    G22 = A12 * A12 + A22 * A22
    h1 = A11 * db1 + A12 * db2
    h2 = A12 * db1 + A22 * db2
    G11, G12, G22, h1, h2 = (box_mean(q, m) for q in (G11, G12, G22, h1, h2))
    G11 = G11 + lam
    G22 = G22 + lam
    det = G11 * G22 - G12 * G12
    u = (G22 * h1 - G12 * h2) / det
    v = (G11 * h2 - G12 * h1) / det
    return u, v


def fb_flow(Y1: np.ndarray, Y2: np.ndarray, levels: int = 4, iters: int = ITERS, n: int = POLY_N,
            sigma: float = POLY_SIGMA, m: int = WIN, lam: float = LAMBDA):
    """Level-0 Farnebäck flow (u, v) of the pair (Y1, Y2)."""
    p1 = _hs.pyramid(_hs.luma_float(Y1), levels)
    p2 = _hs.pyramid(_hs.luma_float(Y2), levels)
    u = v = None
    for lv in range(levels - 1, -1, -1):
        H, W = p1[lv].shape
        if u is None:
            u, v = np.zeros((H, W)), np.zeros((H, W))
        else:
            u, v = _hs.upsample_flow(u, H, W), _hs.upsample_flow(v, H, W)
        r1 = poly_exp(p1[lv], n, sigma)
        r2 = poly_exp(p2[lv], n, sigma)
        for _ in range(iters):
            u, v = displacement(r1, r2, u, v, m, lam)
    return u, v
