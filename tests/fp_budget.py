"""FP32 error budget of pyramidal Horn-Schunck on the 14-camera rig pair
(test infrastructure: numpy only, no GPU).

The flow kernels compute in FP32; the oracle in FP64.  On the 2048 x 2048
rig pairs (5 levels, up to 64 px of disparity between neighbouring cameras,
hard occlusion edges) a few pixels are ill-conditioned: a perturbation of the
images by one FP32 rounding moves their flow by 1e-3 px or more.  This module
re-evaluates the oracle's steps with each step's arithmetic in FP32 or FP64,
so that the share of every step in the deviation from the FP64 result can be
measured:

  pyramid  the [1,4,6,4,1]/16 blur and decimation of each level;
  setup0   warp, gradients and the linearised constraint at level 0;
  setup    the same at the coarser levels;
  upsample the x2 bilinear upsampling of the coarser level's flow;
  jacobi   the 50 Jacobi iterations of each level.

The flow itself is kept in FP32 between steps whenever a step that reads it
is FP32 (the kernels store it in FP32).  The kernels' precision choices --
an exact pyramid (FP64 above level 0), setup in FP64 above level 0, FP32
elsewhere -- are the `kernels` policy.  Run as a script for the full table:

    python tests/fp_budget.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

STEPS = ("pyramid", "setup0", "setup", "upsample", "jacobi")
KERNELS = {"setup0", "upsample", "jacobi"}  # the steps the kernels evaluate in FP32


def rig_pair():
    """Luma planes of cameras 12 and 13 at time step 7 of the seeded rig."""
    import synth
    S = 2048
    rig = synth.rig_scene(5, S, S, 14)
    rows = synth.rig_batch_nv12(rig, [(12, 7), (13, 7)], "cpu").reshape(2, -1).numpy()
    return rows[0].reshape(S * 3 // 2, S)[:S], rows[1].reshape(S * 3 // 2, S)[:S]


def _blur_down(img, dt):
    k = (np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0).astype(dt)
    H, W = img.shape
    p = np.pad(img, ((0, 0), (2, 2)), mode="edge")
    h = sum(k[i] * p[:, i:i + W] for i in range(5))
    p = np.pad(h, ((2, 2), (0, 0)), mode="edge")
    return sum(k[i] * p[i:i + H, :] for i in range(5))[0::2, 0::2]


def _bilinear(img, X0, fx, Y0, fy, dt):
    """Clamped bilinear sample at (X0 + fx, Y0 + fy), integer parts X0, Y0
    and fractions fx, fy in [0, 1) given separately."""
    H, W = img.shape
    one = dt(1)
    fx = np.where((X0 < 0) | (X0 >= W - 1), dt(0), fx).astype(dt)
    fy = np.where((Y0 < 0) | (Y0 >= H - 1), dt(0), fy).astype(dt)
    x0 = np.clip(X0, 0, W - 1)
    y0 = np.clip(Y0, 0, H - 1)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    top = (one - fx) * img[y0, x0] + fx * img[y0, x1]
    bot = (one - fx) * img[y1, x0] + fx * img[y1, x1]
    return (one - fy) * top + fy * bot


def _dx(a):
    p = np.pad(a, ((0, 0), (1, 1)), mode="edge")
    return (p[:, 2:] - p[:, :-2]) * a.dtype.type(0.5)


def _dy(a):
    p = np.pad(a, ((1, 1), (0, 0)), mode="edge")
    return (p[2:, :] - p[:-2, :]) * a.dtype.type(0.5)


def _avg(f):
    H, W = f.shape
    p = np.pad(f, 1, mode="edge")
    t = f.dtype.type
    edge = p[0:H, 1:W + 1] + p[2:H + 2, 1:W + 1] + p[1:H + 1, 0:W] + p[1:H + 1, 2:W + 2]
    diag = p[0:H, 0:W] + p[0:H, 2:W + 2] + p[2:H + 2, 0:W] + p[2:H + 2, 2:W + 2]
    return edge / t(6) + diag / t(12)


def flow(Y1, Y2, fp32_steps, levels=5, alpha=10.0, iters=50):
    """Horn-Schunck flow with the named steps in FP32 and the others in FP64."""
    f32, f64 = np.float32, np.float64
    dt = {s: (f32 if s in fp32_steps else f64) for s in STEPS}
    p1, p2 = [Y1.astype(f64)], [Y2.astype(f64)]
    for _ in range(levels - 1):
        p1.append(_blur_down(p1[-1].astype(dt["pyramid"]), dt["pyramid"]))
        p2.append(_blur_down(p2[-1].astype(dt["pyramid"]), dt["pyramid"]))
    u = v = None
    for lv in range(levels - 1, -1, -1):
        H, W = p1[lv].shape
        if u is None:
            u0 = np.zeros((H, W), f64)
            v0 = np.zeros((H, W), f64)
        else:
            t = dt["upsample"]
            ys, xs = np.mgrid[0:H, 0:W]
            half = np.where(xs & 1, t(0.5), t(0)), np.where(ys & 1, t(0.5), t(0))
            u0 = t(2) * _bilinear(u.astype(t), xs >> 1, half[0], ys >> 1, half[1], t)
            v0 = t(2) * _bilinear(v.astype(t), xs >> 1, half[0], ys >> 1, half[1], t)
        t = dt["setup0"] if lv == 0 else dt["setup"]
        if t == f32 or dt["jacobi"] == f32 or dt["upsample"] == f32:
            u0, v0 = u0.astype(f32), v0.astype(f32)  # the flow the kernels store
        ys, xs = np.mgrid[0:H, 0:W]
        fu, fv = np.floor(u0), np.floor(v0)
        I1 = p1[lv].astype(t)
        I2w = _bilinear(p2[lv].astype(t), xs + fu.astype(np.int64), (u0 - fu).astype(t), ys + fv.astype(np.int64),
                        (v0 - fv).astype(t), t)
        Ix = t(0.5) * (_dx(I1) + _dx(I2w))
        Iy = t(0.5) * (_dy(I1) + _dy(I2w))
        Itp = (I2w - I1) - Ix * u0.astype(t) - Iy * v0.astype(t)
        t = dt["jacobi"]
        Ix, Iy, Itp = Ix.astype(t), Iy.astype(t), Itp.astype(t)
        u, v = u0.astype(t), v0.astype(t)
        den = t(alpha * alpha) + Ix * Ix + Iy * Iy
        for _ in range(iters):
            ub, vb = _avg(u), _avg(v)
            s = (Ix * ub + Iy * vb + Itp) / den
            u, v = ub - Ix * s, vb - Iy * s
    return u.astype(f64), v.astype(f64)


def deviation(ref, got):
    e = np.maximum(np.abs(got[0] - ref[0]), np.abs(got[1] - ref[1]))
    return float(e.max()), int((e > 1e-3).sum()), float(np.quantile(e, 0.9999))


def main():
    from oracle import hs as OH
    Y1, Y2 = rig_pair()
    t0 = time.time()
    ref = OH.hs_flow(Y1, Y2, levels=5, alpha=10.0, iters=50)
    print("FP64 oracle: %.0f s" % (time.time() - t0))
    assert deviation(ref, flow(Y1, Y2, set())) [0] < 1e-9  # this module's FP64 path is the oracle
    rows = [("all FP32", set(STEPS)), ("kernels (FP32: %s)" % ", ".join(sorted(KERNELS)), KERNELS)]
    rows += [("only %s in FP32" % s, {s}) for s in STEPS]
    rows += [("all but %s in FP32" % s, set(STEPS) - {s}) for s in STEPS]
    print("%-44s %10s %8s %12s" % ("policy", "max |d|", "> 1e-3", "99.99th pct"))
    for name, pol in rows:
        mx, n, q = deviation(ref, flow(Y1, Y2, pol))
        print("%-44s %10.3g %8d %12.3g" % (name, mx, n, q), flush=True)


if __name__ == "__main__":
    main()
