"""BF16 conv encoder-decoder flow surrogate, its training step, the residual
gate and EPE (oracle; test infrastructure only).

The Scanner paper runs learned models as ordinary graph operations
(Sec. 3.1, Sec. 5.1.2 DNN) and shows, in its hyperlapse application
(Sec. 5.2.2), a cheap per-pair cost with a conditional fallback to the full
computation when the cheap result is not good enough.  The flow
surrogate is that pattern applied to FLOW: a small network predicts the
flow, a brightness-constancy residual decides per pair whether to keep it
or to fall back to the plain Horn-Schunck solver.  The paper gives no
network; the readings below fix it.

Readings:
* Input: the 2x2 mean of each frame's luma (round half up), as
  (Y - 128) / 64 in BF16, channels (frame 1, frame 2).  Full-resolution width
  and height must be multiples of 8.
* Layers (all 3x3, zero padding 1, BF16 weights and activations, FP32
  accumulation, FP32 bias, ReLU after 1-5):
  conv1 2->32 s1; conv2 32->64 s2; conv3 64->96 s2; nearest x2 up, conv4
  96->64; nearest x2 up, conv5 64->32; conv6 32->2 (linear, FP32 output).
  An activation is bf16(relu(acc + bias)).
* Output: half-resolution flow in half-resolution pixels; full-resolution
  flow = 2 * bilinear(half, (x + 0.5)/2 - 0.5, (y + 0.5)/2 - 0.5), clamped.
* Loss: mean over full-resolution pixels of sqrt(du^2 + dv^2 + eps^2),
  eps = 0.01, against the plain solver's flow.
* ReLU derivative: 1 where the stored activation is > 0.
* Adam with bias correction on FP32 master weights; the BF16 copy used by
  the forward pass is the RNE rounding of the master weights.
* Gate: r = mean over full-resolution pixels of |I2(x + w) - I1(x)| on luma
  (clamped bilinear warp); the pair falls back to the plain solver if
  r > tau.
* EPE: per-pixel sqrt(du^2 + dv^2) against plain flow, mean over pixels.

Pins (tests): forward of each layer against torch.nn.functional.conv2d in
FP64 on the same BF16-rounded inputs; backward against torch FP64 autograd
and against central finite differences; Adam on a linear objective against
its closed form; BF16 rounding against torch's bfloat16 conversion; the
upsampling operator against its transpose (adjoint identity); EPE against
closed forms (constant offsets, half-image offsets).  The trained
network's quality is parity unpinned (only the EPE measurement judges it).
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

LAYERS = [  # (name, c_in, c_out, stride, upsample_input, relu)
    ("conv1", 2, 32, 1, False, True),
    ("conv2", 32, 64, 2, False, True),
    ("conv3", 64, 96, 2, False, True),
    ("conv4", 96, 64, 1, True, True),
    ("conv5", 64, 32, 1, True, True),
    ("conv6", 32, 2, 1, False, False),
]
CHARB_EPS = 0.01


def n_params() -> int:
    return sum(co * ci * 9 + co for _, ci, co, _, _, _ in LAYERS)


def bf16_rne(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest BF16 value (8 significant bits), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)               # x = m * 2^e, 0.5 <= |m| < 1
    scaled = m * 256.0               # 8 significant bits -> integer part
    r = np.round(scaled)             # numpy rounds half to even
    return np.ldexp(r / 256.0, e)


def half_gray(y: np.ndarray) -> np.ndarray:
    """2x2 mean of luma (round half up) as (v - 128) / 64."""
    a = y.astype(np.int64)
    s = a[0::2, 0::2] + a[0::2, 1::2] + a[1::2, 0::2] + a[1::2, 1::2]
    v = (s + 2) >> 2
    return (v - 128) / 64.0


def net_input(y1: np.ndarray, y2: np.ndarray) -> np.ndarray:
    return bf16_rne(np.stack([half_gray(y1), half_gray(y2)]))


def upsample2(x: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_adjoint(g: np.ndarray) -> np.ndarray:
    C, H, W = g.shape
    return g.reshape(C, H // 2, 2, W // 2, 2).sum(axis=(2, 4))


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """out[co, y, x] = b[co] + sum_{ci,ky,kx} w[co,ci,ky,kx] xpad[ci, s*y+ky, s*x+kx] (FP64)."""
    C, H, W = x.shape
    Ho = (H - 1) // stride + 1
    Wo = (W - 1) // stride + 1
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    out = np.zeros((w.shape[0], Ho, Wo)) + b[:, None, None]
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            # the channel contraction of one tap, as a library matrix product
            out += np.tensordot(w[:, :, ky, kx], patch, axes=([1], [0]))
    return out


def conv3x3_backward(x: np.ndarray, w: np.ndarray, stride: int, gout: np.ndarray):
    """Gradients of conv3x3 w.r.t. its input, weights and bias."""
    C, H, W = x.shape
    Ho, Wo = gout.shape[1:]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride),
                  slice(kx, kx + stride * (Wo - 1) + 1, stride))
            gw[:, :, ky, kx] = np.tensordot(gout, xp[sl], axes=([1, 2], [1, 2]))
            gxp[sl] += np.tensordot(w[:, :, ky, kx], gout, axes=([0], [0]))
    gb = gout.sum(axis=(1, 2))
    return gxp[:, 1:H + 1, 1:W + 1], gw, gb


def init_params(seed: int) -> Dict[str, np.ndarray]:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, from SplitMix64 + Box-Muller."""
    from synth import SplitMix64
    rng = SplitMix64(seed)
    p = {}
    for name, ci, co, _, _, _ in LAYERS:
        std = math.sqrt(2.0 / (ci * 9))
        if name == "conv6":
            std *= 0.1
        p[name + ".w"] = np.array([rng.normal() * std for _ in range(co * ci * 9)]).reshape(co, ci, 3, 3)
        p[name + ".b"] = np.zeros(co)
    return p


def _identity(x):
    return x


def forward(params: Dict[str, np.ndarray], x: np.ndarray, rounding: bool = True):
    """Returns (half-res FP64 flow [2, h, w], saved (layer input, activation) pairs).
    rounding=False drops the BF16 rounding (for derivative checks)."""
    rnd = bf16_rne if rounding else _identity
    saved = []
    a = x
    for name, ci, co, stride, up, relu in LAYERS:
        inp = upsample2(a) if up else a
        w = rnd(params[name + ".w"])
        z = conv3x3(inp, w, params[name + ".b"], stride)
        a = rnd(np.maximum(z, 0.0)) if relu else z
        saved.append((inp, a))
    return a, saved


def backward(params: Dict[str, np.ndarray], saved, g_out: np.ndarray, rounding: bool = True) -> Dict[str, np.ndarray]:
    """Gradients of every parameter given dLoss/d(half-res flow); the BF16
    rounding of weights and activations passes gradients through unchanged."""
    rnd = bf16_rne if rounding else _identity
    grads = {}
    g = g_out
    for (name, ci, co, stride, up, relu), (inp, act) in zip(reversed(LAYERS), reversed(saved)):
        if relu:
            g = g * (act > 0)
        w = rnd(params[name + ".w"])
        gx, gw, gb = conv3x3_backward(inp, w, stride, g)
        grads[name + ".w"] = gw
        grads[name + ".b"] = gb
        g = upsample2_adjoint(gx) if up else gx
    return grads


def upsample_flow_matrix_1d(n_half: int) -> np.ndarray:
    """Linear map half-res -> full-res samples of bilinear with half-pixel centres (clamped)."""
    n = 2 * n_half
    M = np.zeros((n, n_half))
    for x in range(n):
        X = min(max((x + 0.5) / 2.0 - 0.5, 0.0), n_half - 1.0)
        x0 = int(math.floor(X))
        x1 = min(x0 + 1, n_half - 1)
        f = X - x0
        M[x, x0] += 1.0 - f
        M[x, x1] += f
    return M


def flow_full(half: np.ndarray) -> np.ndarray:
    """Full-resolution flow in full-resolution pixels: 2 * bilinear upsample."""
    _, h, w = half.shape
    My = upsample_flow_matrix_1d(h)
    Mx = upsample_flow_matrix_1d(w)
    # separable: rows with My, columns with Mx (library matrix products)
    return 2.0 * np.stack([My @ half[c] @ Mx.T for c in range(half.shape[0])])


def flow_full_adjoint(g_full: np.ndarray, h: int, w: int) -> np.ndarray:
    My = upsample_flow_matrix_1d(h)
    Mx = upsample_flow_matrix_1d(w)
    return 2.0 * np.stack([My.T @ g_full[c] @ Mx for c in range(g_full.shape[0])])


def charbonnier_loss(full: np.ndarray, target: np.ndarray):
    """(loss, dloss/dfull) of mean sqrt(du^2 + dv^2 + eps^2)."""
    d = full - target
    r = np.sqrt(d[0] ** 2 + d[1] ** 2 + CHARB_EPS ** 2)
    n = r.size
    return r.mean(), d / r[None] / n


def train_step_grads(params, y1, y2, target_full, rounding: bool = True):
    """Loss and gradients of one sample (y1, y2 full-resolution luma; target [2, H, W])."""
    x = net_input(y1, y2)
    return loss_and_grads(params, x, target_full, rounding)


def loss_and_grads(params, x, target_full, rounding: bool = True):
    half, saved = forward(params, x, rounding)
    full = flow_full(half)
    loss, g_full = charbonnier_loss(full, target_full)
    g_half = flow_full_adjoint(g_full, half.shape[1], half.shape[2])
    return loss, backward(params, saved, g_half, rounding)


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        for k in params:
            g = grads[k]
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g * g
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            params[k] = params[k] - lr * mh / (np.sqrt(vh) + self.eps)


def warp_residual(y1: np.ndarray, y2: np.ndarray, flow: np.ndarray) -> float:
    """Gate statistic: mean |I2(x + w) - I1(x)| with a clamped bilinear warp of luma."""
    from oracle.hs import warp
    I1 = y1.astype(np.float64)
    I2 = y2.astype(np.float64)
    return float(np.abs(warp(I2, flow[0], flow[1]) - I1).mean())


def epe(flow: np.ndarray, ref: np.ndarray) -> float:
    return float(np.sqrt(((flow - ref) ** 2).sum(axis=0)).mean())
