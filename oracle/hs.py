"""Pyramidal Horn-Schunck optical flow in FP64 (oracle; test infrastructure only).

Scanner's FLOW microbenchmark runs an optical-flow kernel over every frame
pair with a two-frame stencil S[0,1] (Sec. 3.2 "Stencil operations",
Sec. 5.1.2).  The paper's kernel is a third-party library routine; this
build fixes the textbook Horn & Schunck (1981) method in a coarse-to-fine
pyramid instead.  The flow w = (u, v) of a pair (I1, I2) satisfies
I1(x) ~ I2(x + w(x)), in pixels of the level it is expressed at.

Steps (this module follows them in this order, in whole-array numpy):

1. I = float(Y) of the NV12 luma plane, code values 0..255.
2. Pyramid: level 0 = I; level l+1 keeps the even samples of level l blurred
   by the separable [1,4,6,4,1]/16 filter (horizontal pass, then vertical),
   clamp-to-edge; size ceil(W/2) x ceil(H/2).
3. The coarsest level starts from u = v = 0.
4. Finer levels start from u0(x, y) = 2 * bilinear(u_coarse, x/2, y/2)
   (coordinates clamped), likewise v0.
5. I2 is warped by the start flow: I2w(x, y) = bilinear(I2, x + u0, y + v0),
   sample coordinates clamped to the image.
6. Ix = (Dx I1 + Dx I2w) / 2 with Dx I(x) = (I(x+1) - I(x-1)) / 2 under
   clamp-to-edge; Iy likewise; It = I2w - I1.
7. The brightness-constancy constraint is linearised about the start flow,
   so smoothness acts on the total flow: It' = It - Ix u0 - Iy v0 and the
   iteration starts from (u0, v0).
8. Neighbour average: weight 1/6 on the four edge neighbours and 1/12 on the
   four diagonal neighbours, clamp-to-edge.
9. Jacobi update, all reads from the previous iterate:
   u <- ubar - Ix (Ix ubar + Iy vbar + It') / (alpha^2 + Ix^2 + Iy^2),
   v <- vbar - Iy (same).
10. alpha and the iteration count are the same at every level; one warp per
    level; no median filtering or robust penalty.

Pins (tests): identical and constant frames give exactly zero flow;
sub-pixel translations of band-limited textures are recovered, with the
right sign; transposing both frames swaps u and v; at one level a horizontal
mirror negates u; the Jacobi fixed point equals a sparse direct solve of the
Horn-Schunck normal equations; the blur of an impulse is the binomial
outer product; an integer warp is an exact shift; upsampling a constant c
gives 2c.  The border and coordinate conventions are pinned by values worked
out by hand: the clamped blur of a corner impulse and of a ramp, the even
samples of a clamped ramp, half one-sided differences of x^2 + 5 at both
ends, the upsampling of a coarse ramp (coarse sample k at fine 2k), and
bilinear sampling of a function in span{1, x, y, xy} (exact inside,
clamped outside).  A mutation test plants a mistake at each of these places
and checks that a pin fails.  Parity pinned.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def luma_float(y_u8: np.ndarray) -> np.ndarray:
    return y_u8.astype(np.float64)


def blur5(img: np.ndarray) -> np.ndarray:
    """Separable [1,4,6,4,1]/16 blur, horizontal then vertical, clamp-to-edge."""
    k = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0
    H, W = img.shape
    p = np.pad(img, ((0, 0), (2, 2)), mode="edge")
    h = sum(k[i] * p[:, i:i + W] for i in range(5))
    p = np.pad(h, ((2, 2), (0, 0)), mode="edge")
    return sum(k[i] * p[i:i + H, :] for i in range(5))


def pyr_down(img: np.ndarray) -> np.ndarray:
    return blur5(img)[0::2, 0::2]


def pyramid(img: np.ndarray, levels: int) -> List[np.ndarray]:
    out = [img]
    for _ in range(levels - 1):
        out.append(pyr_down(out[-1]))
    return out


def bilinear(img: np.ndarray, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Bilinear sample of img at (X, Y), coordinates clamped to the image."""
    H, W = img.shape
    X = np.clip(X, 0.0, W - 1.0)
    Y = np.clip(Y, 0.0, H - 1.0)
    x0 = np.floor(X).astype(np.int64)
    y0 = np.floor(Y).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    fx = X - x0
    fy = Y - y0
    top = (1.0 - fx) * img[y0, x0] + fx * img[y0, x1]
    bot = (1.0 - fx) * img[y1, x0] + fx * img[y1, x1]
    return (1.0 - fy) * top + fy * bot


def grid(H: int, W: int) -> Tuple[np.ndarray, np.ndarray]:
    ys, xs = np.mgrid[0:H, 0:W]
    return xs.astype(np.float64), ys.astype(np.float64)


def upsample_flow(f_coarse: np.ndarray, H: int, W: int) -> np.ndarray:
    xs, ys = grid(H, W)
    return 2.0 * bilinear(f_coarse, xs / 2.0, ys / 2.0)


def warp(img: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    xs, ys = grid(*img.shape)
    return bilinear(img, xs + u, ys + v)


def dx(img: np.ndarray) -> np.ndarray:
    p = np.pad(img, ((0, 0), (1, 1)), mode="edge")
    return (p[:, 2:] - p[:, :-2]) / 2.0


def dy(img: np.ndarray) -> np.ndarray:
    p = np.pad(img, ((1, 1), (0, 0)), mode="edge")
    return (p[2:, :] - p[:-2, :]) / 2.0


def neighbour_avg(f: np.ndarray) -> np.ndarray:
    H, W = f.shape
    p = np.pad(f, 1, mode="edge")
    edge = p[0:H, 1:W + 1] + p[2:H + 2, 1:W + 1] + p[1:H + 1, 0:W] + p[1:H + 1, 2:W + 2]
    diag = p[0:H, 0:W] + p[0:H, 2:W + 2] + p[2:H + 2, 0:W] + p[2:H + 2, 2:W + 2]
    return edge / 6.0 + diag / 12.0


def level_setup(I1: np.ndarray, I2: np.ndarray, u0: np.ndarray, v0: np.ndarray):
    """Steps 5-7: warped image and the linearised constraint's coefficients."""
    I2w = warp(I2, u0, v0)
    Ix = 0.5 * (dx(I1) + dx(I2w))
    Iy = 0.5 * (dy(I1) + dy(I2w))
    It = I2w - I1
    Itp = It - Ix * u0 - Iy * v0
    return Ix, Iy, Itp


def jacobi(u: np.ndarray, v: np.ndarray, Ix: np.ndarray, Iy: np.ndarray, Itp: np.ndarray,
           alpha: float, iters: int):
    """Steps 8-9 repeated `iters` times."""
    den = alpha * alpha + Ix * Ix + Iy * Iy
    for _ in range(iters):
        ub = neighbour_avg(u)
        vb = neighbour_avg(v)
        t = (Ix * ub + Iy * vb + Itp) / den
        u = ub - Ix * t
        v = vb - Iy * t
    return u, v


def hs_flow(Y1: np.ndarray, Y2: np.ndarray, levels: int = 4, alpha: float = 10.0, iters: int = 50,
            return_levels: bool = False):
    """Level-0 flow (u, v) of the pair (Y1, Y2) (uint8 luma planes or float images)."""
    p1 = pyramid(luma_float(Y1), levels)
    p2 = pyramid(luma_float(Y2), levels)
    u = v = None
    per_level = []
    for lv in range(levels - 1, -1, -1):
        H, W = p1[lv].shape
        if u is None:
            u0 = np.zeros((H, W))
            v0 = np.zeros((H, W))
        else:
            u0 = upsample_flow(u, H, W)
            v0 = upsample_flow(v, H, W)
        Ix, Iy, Itp = level_setup(p1[lv], p2[lv], u0, v0)
        u, v = jacobi(u0, v0, Ix, Iy, Itp, alpha, iters)
        per_level.append((lv, u, v))
    if return_levels:
        return u, v, per_level
    return u, v


def level_sizes(width: int, height: int, levels: int) -> List[Tuple[int, int]]:
    out = [(width, height)]
    for _ in range(levels - 1):
        w, h = out[-1]
        out.append(((w + 1) // 2, (h + 1) // 2))
    return out
