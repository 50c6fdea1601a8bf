"""Seeded synthetic NV12 video sources.

This module only *generates inputs*: textures, layered scenes, camera rigs,
sampling lists.  It contains none of the pixel-stage arithmetic (colour
conversion, histograms, pyramids, optical flow, the surrogate network); both
the CPU oracle and the GPU path consume the bytes it produces.

Design of the stand-in data (the paper's 1080p film, TV clips and camera-rig
footage are not available; the shapes follow the paper's workloads):

* Scalar parameters (frequencies, phases, layer shapes, motion) come from
  SplitMix64 (Steele, Lea & Flood 2014) seeded per object, followed by
  Box-Muller for normals, so they are identical on every machine.
* A texture is 128 + sum_k a cos(2 pi f_k . x + phi_k) over 64 plane waves
  with |f_k| uniform in [1/64, 1/16] cycles/px, uniform directions and
  a = sigma * sqrt(2/64).  It is band-limited and evaluated analytically, so a
  sub-pixel translation or any affine map of it is exact.  A plane wave under
  an affine map is again a plane wave, and cos(a x + b y + c) splits into
  products of 1-D cos/sin tables, so a whole frame is one small matrix
  product per texture.
* Per-pixel sensor noise N(0, sigma_n^2) comes from torch's seeded
  generator on the generating device, then rint and clamp to 0..255.  Bytes
  therefore depend on the device that generated them; every consumer takes
  its bytes from one generation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import torch

_M64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 stream (public-domain reference constants)."""

    def __init__(self, seed: int):
        self.s = seed & _M64

    def u64(self) -> int:
        self.s = (self.s + 0x9E3779B97F4A7C15) & _M64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.u64() >> 11) * 2.0 ** -53)

    def normal(self) -> float:
        u1 = max(self.uniform(), 2.0 ** -60)
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)

    def randint(self, n: int) -> int:
        return self.u64() % n


# --------------------------------------------------------------------------
# textures


@dataclass
class Texture:
    mean: float
    amp: float
    fx: List[float]
    fy: List[float]
    phase: List[float]

    @staticmethod
    def random(rng: SplitMix64, mean: float = 128.0, sigma: float = 40.0, k: int = 64,
               fmin: float = 1.0 / 64, fmax: float = 1.0 / 16) -> "Texture":
        fx, fy, ph = [], [], []
        for _ in range(k):
            mag = rng.uniform(fmin, fmax)
            ang = rng.uniform(0.0, 2.0 * math.pi)
            fx.append(mag * math.cos(ang))
            fy.append(mag * math.sin(ang))
            ph.append(rng.uniform(0.0, 2.0 * math.pi))
        return Texture(mean, sigma * math.sqrt(2.0 / k), fx, fy, ph)

    def eval_grid(self, xs: torch.Tensor, ys: torch.Tensor, M=((1.0, 0.0), (0.0, 1.0)),
                  c=(0.0, 0.0)) -> torch.Tensor:
        """T(M @ (x, y) + c) on the grid ys x xs (float64, shape [len(ys), len(xs)])."""
        dev = xs.device
        fx = torch.tensor(self.fx, dtype=torch.float64, device=dev)
        fy = torch.tensor(self.fy, dtype=torch.float64, device=dev)
        ph = torch.tensor(self.phase, dtype=torch.float64, device=dev)
        two_pi = 2.0 * math.pi
        # f . (M p + c) = (M^T f) . p + f . c
        gx = two_pi * (M[0][0] * fx + M[1][0] * fy)
        gy = two_pi * (M[0][1] * fx + M[1][1] * fy)
        gam = two_pi * (fx * c[0] + fy * c[1]) + ph
        ax = gx[:, None] * xs[None, :] + gam[:, None]          # [K, W]
        ay = gy[:, None] * ys[None, :]                           # [K, H]
        left = torch.cat([torch.cos(ay), -torch.sin(ay)], 0).t()  # [H, 2K]
        right = torch.cat([torch.cos(ax), torch.sin(ax)], 0)      # [2K, W]
        return self.mean + self.amp * (left @ right)


# --------------------------------------------------------------------------
# layered scenes


@dataclass
class Layer:
    tex_y: Texture
    tex_u: Texture
    tex_v: Texture
    shape: str                 # "full", "ellipse", "rect"
    cx: float = 0.0
    cy: float = 0.0
    rx: float = 1.0
    ry: float = 1.0
    rot: float = 0.0
    # motion: image = A_t q + b_t, A_t = I + eps * sin(2 pi t / period + phi) * E, b_t = B sin(...)
    bx: float = 0.0
    by: float = 0.0
    period: float = 100.0
    phi: float = 0.0
    eps: float = 0.0
    E: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    # optional explicit per-frame translation list (pure translation scenes)
    shifts: Optional[List[Tuple[float, float]]] = None

    def inverse_map(self, t: float):
        """Return (M, c) with q = M @ x_img + c."""
        if self.shifts is not None:
            dx, dy = self.shifts[int(t)]
            return ((1.0, 0.0), (0.0, 1.0)), (-dx, -dy)
        s = math.sin(2.0 * math.pi * t / self.period + self.phi)
        a00 = 1.0 + self.eps * s * self.E[0]
        a01 = self.eps * s * self.E[1]
        a10 = self.eps * s * self.E[2]
        a11 = 1.0 + self.eps * s * self.E[3]
        det = a00 * a11 - a01 * a10
        m = ((a11 / det, -a01 / det), (-a10 / det, a00 / det))
        b = (self.bx * s, self.by * s)
        # about the layer centre so that the affine part does not drift the whole frame
        cxi, cyi = self.cx, self.cy
        # image = A (q - ctr) + ctr + b  =>  q = M (image - ctr - b) + ctr
        ox = -(cxi + b[0])
        oy = -(cyi + b[1])
        c = (m[0][0] * ox + m[0][1] * oy + cxi, m[1][0] * ox + m[1][1] * oy + cyi)
        return m, c

    def mask(self, qx: torch.Tensor, qy: torch.Tensor) -> torch.Tensor:
        if self.shape == "full":
            return torch.ones_like(qx, dtype=torch.bool)
        dx = qx - self.cx
        dy = qy - self.cy
        cr, sr = math.cos(self.rot), math.sin(self.rot)
        lx = cr * dx + sr * dy
        ly = -sr * dx + cr * dy
        if self.shape == "ellipse":
            return (lx / self.rx) ** 2 + (ly / self.ry) ** 2 <= 1.0
        return (lx.abs() <= self.rx) & (ly.abs() <= self.ry)


@dataclass
class Scene:
    width: int
    height: int
    layers: List[Layer]
    seed: int
    noise_sigma: float = 2.0

    def planes(self, t: int, device="cpu") -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
        """Noise-free float64 Y [H,W], U and V [H/2,W/2] of frame t."""
        W, H = self.width, self.height
        dev = torch.device(device)
        xs = torch.arange(W, dtype=torch.float64, device=dev)
        ys = torch.arange(H, dtype=torch.float64, device=dev)
        cxs = 2.0 * torch.arange(W // 2, dtype=torch.float64, device=dev) + 0.5
        cys = 2.0 * torch.arange(H // 2, dtype=torch.float64, device=dev) + 0.5
        Y = torch.zeros(H, W, dtype=torch.float64, device=dev)
        U = torch.zeros(H // 2, W // 2, dtype=torch.float64, device=dev)
        V = torch.zeros_like(U)
        for lay in self.layers:
            M, c = lay.inverse_map(t)
            ty = lay.tex_y.eval_grid(xs, ys, M, c)
            tu = lay.tex_u.eval_grid(cxs, cys, M, c)
            tv = lay.tex_v.eval_grid(cxs, cys, M, c)
            if lay.shape == "full":
                Y, U, V = ty, tu, tv
                continue
            qx = M[0][0] * xs[None, :] + M[0][1] * ys[:, None] + c[0]
            qy = M[1][0] * xs[None, :] + M[1][1] * ys[:, None] + c[1]
            m = lay.mask(qx, qy)
            Y = torch.where(m, ty, Y)
            qcx = M[0][0] * cxs[None, :] + M[0][1] * cys[:, None] + c[0]
            qcy = M[1][0] * cxs[None, :] + M[1][1] * cys[:, None] + c[1]
            mc = lay.mask(qcx, qcy)
            U = torch.where(mc, tu, U)
            V = torch.where(mc, tv, V)
        return Y, U, V

    def nv12(self, t: int, device="cpu", pitch: Optional[int] = None) -> torch.Tensor:
        """uint8 NV12 frame [H*3/2, pitch]: Y rows then interleaved U,V rows."""
        W, H = self.width, self.height
        pitch = W if pitch is None else pitch
        Y, U, V = self.planes(t, device)
        dev = Y.device
        g = torch.Generator(device=dev)
        g.manual_seed((self.seed * 1_000_003 + 7919 * t + 17) & 0x7FFFFFFFFFFFFFFF)
        s = self.noise_sigma
        if s > 0:
            Y = Y + s * torch.randn(Y.shape, generator=g, dtype=torch.float64, device=dev)
            U = U + s * torch.randn(U.shape, generator=g, dtype=torch.float64, device=dev)
            V = V + s * torch.randn(V.shape, generator=g, dtype=torch.float64, device=dev)
        q = lambda a: torch.clamp(torch.round(a), 0, 255).to(torch.uint8)
        out = torch.zeros(H * 3 // 2, pitch, dtype=torch.uint8, device=dev)
        out[:H, :W] = q(Y)
        uv = torch.stack([q(U), q(V)], dim=-1).reshape(H // 2, W)
        out[H:, :W] = uv
        return out


def eval_grid_batch(tex: Texture, xs: torch.Tensor, ys: torch.Tensor, Ms, cs) -> torch.Tensor:
    """tex(M_b @ (x, y) + c_b) for a batch of maps (float64 [B, len(ys), len(xs)])."""
    dev = xs.device
    fx = torch.tensor(tex.fx, dtype=torch.float64, device=dev)
    fy = torch.tensor(tex.fy, dtype=torch.float64, device=dev)
    ph = torch.tensor(tex.phase, dtype=torch.float64, device=dev)
    M = torch.tensor(Ms, dtype=torch.float64, device=dev)          # [B, 2, 2]
    c = torch.tensor(cs, dtype=torch.float64, device=dev)          # [B, 2]
    two_pi = 2.0 * math.pi
    gx = two_pi * (M[:, 0, 0, None] * fx + M[:, 1, 0, None] * fy)  # [B, K]
    gy = two_pi * (M[:, 0, 1, None] * fx + M[:, 1, 1, None] * fy)
    gam = two_pi * (c[:, 0, None] * fx + c[:, 1, None] * fy) + ph
    ax = gx[:, :, None] * xs[None, None, :] + gam[:, :, None]      # [B, K, W]
    ay = gy[:, :, None] * ys[None, None, :]                        # [B, K, H]
    left = torch.cat([torch.cos(ay), -torch.sin(ay)], 1).transpose(1, 2)  # [B, H, 2K]
    right = torch.cat([torch.cos(ax), torch.sin(ax)], 1)                   # [B, 2K, W]
    return tex.mean + tex.amp * torch.bmm(left, right)


def _layers_batch_nv12(layers, maps, W: int, H: int, dev, gen_seed: int, sigma: float) -> torch.Tensor:
    """Compose hard-edged layers for a batch of frames: maps[l] lists the (M, c)
    inverse maps of layer l, one per frame; the first layer is the background."""
    B = len(maps[0])
    xs = torch.arange(W, dtype=torch.float64, device=dev)
    ys = torch.arange(H, dtype=torch.float64, device=dev)
    cxs = 2.0 * torch.arange(W // 2, dtype=torch.float64, device=dev) + 0.5
    cys = 2.0 * torch.arange(H // 2, dtype=torch.float64, device=dev) + 0.5
    Y = U = V = None
    for lay, lm in zip(layers, maps):
        Ms = [m for m, _ in lm]
        cs = [c for _, c in lm]
        ty = eval_grid_batch(lay.tex_y, xs, ys, Ms, cs)
        tu = eval_grid_batch(lay.tex_u, cxs, cys, Ms, cs)
        tv = eval_grid_batch(lay.tex_v, cxs, cys, Ms, cs)
        if Y is None:
            Y, U, V = ty, tu, tv
            continue
        M = torch.tensor(Ms, dtype=torch.float64, device=dev)
        c = torch.tensor(cs, dtype=torch.float64, device=dev)

        def qmap(px, py):
            qx = M[:, 0, 0, None, None] * px[None, None, :] + M[:, 0, 1, None, None] * py[None, :, None] + c[:, 0, None, None]
            qy = M[:, 1, 0, None, None] * px[None, None, :] + M[:, 1, 1, None, None] * py[None, :, None] + c[:, 1, None, None]
            return qx, qy
        m = lay.mask(*qmap(xs, ys))
        Y = torch.where(m, ty, Y)
        mc = lay.mask(*qmap(cxs, cys))
        U = torch.where(mc, tu, U)
        V = torch.where(mc, tv, V)
    g = torch.Generator(device=dev)
    g.manual_seed(gen_seed & 0x7FFFFFFFFFFFFFFF)
    if sigma > 0:
        Y = Y + sigma * torch.randn(Y.shape, generator=g, dtype=torch.float64, device=dev)
        U = U + sigma * torch.randn(U.shape, generator=g, dtype=torch.float64, device=dev)
        V = V + sigma * torch.randn(V.shape, generator=g, dtype=torch.float64, device=dev)
    q = lambda a: torch.clamp(torch.round(a), 0, 255).to(torch.uint8)
    out = torch.empty(B, H * 3 // 2, W, dtype=torch.uint8, device=dev)
    out[:, :H] = q(Y)
    out[:, H:] = torch.stack([q(U), q(V)], dim=-1).reshape(B, H // 2, W)
    return out


def scene_batch_nv12(scene: "Scene", ts: Sequence[int], device="cpu", seed_salt: int = 0) -> torch.Tensor:
    """uint8 NV12 frames [B, H*3/2, W] of one layered scene at time steps ts,
    evaluated for all time steps at once (same model as Scene.nv12; the noise
    stream differs)."""
    maps = [[lay.inverse_map(t) for t in ts] for lay in scene.layers]
    seed = scene.seed * 1_000_003 + 104729 * (seed_salt + 1) + int(ts[0])
    return _layers_batch_nv12(scene.layers, maps, scene.width, scene.height, torch.device(device), seed,
                              scene.noise_sigma)


def translation_scene(seed: int, width: int, height: int, n_frames: int, max_shift: float = 2.0,
                      noise_sigma: float = 2.0) -> Tuple[Scene, List[Tuple[float, float]]]:
    """One texture translated per frame: frame t = T(x - sum_{k<t} d_k), |d_k| <= max_shift.

    Returns the scene and the per-pair shifts d_0..d_{n-2}."""
    rng = SplitMix64(seed)
    tex = Texture.random(rng)
    tu = Texture.random(rng, sigma=20.0)
    tv = Texture.random(rng, sigma=20.0)
    ds, cum = [], [(0.0, 0.0)]
    for _ in range(n_frames - 1):
        r = max_shift * math.sqrt(rng.uniform())
        a = rng.uniform(0.0, 2.0 * math.pi)
        ds.append((r * math.cos(a), r * math.sin(a)))
        cum.append((cum[-1][0] + ds[-1][0], cum[-1][1] + ds[-1][1]))
    lay = Layer(tex, tu, tv, "full", shifts=cum)
    return Scene(width, height, [lay], seed, noise_sigma), ds


def layered_scene(seed: int, width: int, height: int, n_layers: int = 4, max_disp: float = 8.0,
                  noise_sigma: float = 2.0) -> Scene:
    """Background plus n_layers hard-edged ellipse/rectangle layers, each with its own
    textures and a bounded-excursion affine trajectory: any two frames differ by at
    most about max_disp px at any pixel."""
    rng = SplitMix64(seed)
    W, H = width, height
    diag = math.hypot(W, H)
    layers = []
    for i in range(n_layers + 1):
        ty = Texture.random(rng)
        tu = Texture.random(rng, sigma=20.0)
        tv = Texture.random(rng, sigma=20.0)
        # translation excursion amplitude (half the bound, since sin spans [-1, 1])
        amp = max_disp * 0.5 * (0.35 + 0.4 * rng.uniform())
        ang = rng.uniform(0.0, 2.0 * math.pi)
        # affine excursion: eps * |q - ctr| <= about 0.1 * max_disp over the frame
        eps = 0.1 * max_disp / diag * rng.uniform()
        E = tuple(rng.uniform(-1.0, 1.0) for _ in range(4))
        period = rng.uniform(60.0, 600.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        if i == 0:
            lay = Layer(ty, tu, tv, "full", cx=W / 2, cy=H / 2, bx=0.5 * amp * math.cos(ang),
                        by=0.5 * amp * math.sin(ang), period=period, phi=phi, eps=eps, E=E)
        else:
            shape = "ellipse" if rng.uniform() < 0.5 else "rect"
            lay = Layer(ty, tu, tv, shape, cx=rng.uniform(0.15, 0.85) * W, cy=rng.uniform(0.15, 0.85) * H,
                        rx=rng.uniform(0.08, 0.25) * W, ry=rng.uniform(0.08, 0.25) * H,
                        rot=rng.uniform(0.0, math.pi), bx=amp * math.cos(ang), by=amp * math.sin(ang),
                        period=period, phi=phi, eps=eps, E=E)
        layers.append(lay)
    return Scene(W, H, layers, seed, noise_sigma)


def rig_scene(seed: int, width: int, height: int, n_cams: int, max_disp: float = 64.0,
              noise_sigma: float = 2.0) -> "RigScene":
    return RigScene(seed, width, height, n_cams, max_disp, noise_sigma)


@dataclass
class RigScene:
    """Camera-rig stand-in: camera c sees layer l shifted horizontally by c * delta_l(x, t),
    with delta_l an affine function of x in [0, max_disp / (n_cams - 1)] per camera step,
    and a vertical offset of at most 1 px across the rig."""
    seed: int
    width: int
    height: int
    n_cams: int
    max_disp: float
    noise_sigma: float
    scene: Scene = field(init=False)
    disp: List[Tuple[float, float, float]] = field(init=False)

    def __post_init__(self):
        self.scene = layered_scene(self.seed, self.width, self.height, 4, 0.0, self.noise_sigma)
        rng = SplitMix64(self.seed ^ 0xA5A5)
        step = self.max_disp / max(self.n_cams - 1, 1)
        self.disp = []
        for _ in self.scene.layers:
            d0 = rng.uniform(0.0, step)
            d1 = rng.uniform(0.0, step)
            self.disp.append((d0, d1, rng.uniform(-1.0, 1.0) / max(self.n_cams - 1, 1)))

    def nv12(self, cam: int, t: int, device="cpu") -> torch.Tensor:
        """uint8 NV12 frame of camera `cam` at time step `t`."""
        return _rig_frame(self, cam, t, device)


def _rig_frame(rig: "RigScene", cam: int, t: int, device) -> torch.Tensor:
    sc = rig.scene
    W, H = sc.width, sc.height
    dev = torch.device(device)
    xs = torch.arange(W, dtype=torch.float64, device=dev)
    ys = torch.arange(H, dtype=torch.float64, device=dev)
    cxs = 2.0 * torch.arange(W // 2, dtype=torch.float64, device=dev) + 0.5
    cys = 2.0 * torch.arange(H // 2, dtype=torch.float64, device=dev) + 0.5
    Y = U = V = None
    tt = 0.35 * math.sin(2.0 * math.pi * t / 150.0)  # slow common drift over time
    for lay, (d0, d1, vyc) in zip(sc.layers, rig.disp):
        # camera c sees the layer shifted by c * (d0 + (d1 - d0) x / W) horizontally
        off, k, vy = cam * d0, cam * (d1 - d0) / W, cam * vyc
        # x_img = (1 + k) x_q + off + tt  =>  x_q = (x_img - off - tt) / (1 + k)
        M = ((1.0 / (1.0 + k), 0.0), (0.0, 1.0))
        c = (-(off + tt) / (1.0 + k), -vy)
        ty = lay.tex_y.eval_grid(xs, ys, M, c)
        tu = lay.tex_u.eval_grid(cxs, cys, M, c)
        tv = lay.tex_v.eval_grid(cxs, cys, M, c)
        if Y is None:
            Y, U, V = ty, tu, tv
            continue
        qx = M[0][0] * xs[None, :] + c[0] + 0.0 * ys[:, None]
        qy = ys[:, None] + c[1] + 0.0 * xs[None, :]
        m = lay.mask(qx, qy)
        Y = torch.where(m, ty, Y)
        qcx = M[0][0] * cxs[None, :] + c[0] + 0.0 * cys[:, None]
        qcy = cys[:, None] + c[1] + 0.0 * cxs[None, :]
        mc = lay.mask(qcx, qcy)
        U = torch.where(mc, tu, U)
        V = torch.where(mc, tv, V)
    g = torch.Generator(device=dev)
    g.manual_seed((sc.seed * 1_000_003 + 7919 * (t * 64 + cam) + 29) & 0x7FFFFFFFFFFFFFFF)
    s = sc.noise_sigma
    Y = Y + s * torch.randn(Y.shape, generator=g, dtype=torch.float64, device=dev)
    U = U + s * torch.randn(U.shape, generator=g, dtype=torch.float64, device=dev)
    V = V + s * torch.randn(V.shape, generator=g, dtype=torch.float64, device=dev)
    q = lambda a: torch.clamp(torch.round(a), 0, 255).to(torch.uint8)
    out = torch.empty(H * 3 // 2, W, dtype=torch.uint8, device=dev)
    out[:H] = q(Y)
    out[H:] = torch.stack([q(U), q(V)], dim=-1).reshape(H // 2, W)
    return out


def rig_batch_nv12(rig: "RigScene", frames: Sequence[Tuple[int, int]], device="cpu") -> torch.Tensor:
    """uint8 NV12 frames [B, H*3/2, W] of (camera, time step) pairs, evaluated at
    once (same geometry as RigScene.nv12; the noise stream differs)."""
    sc = rig.scene
    W = sc.width
    maps = []
    for (d0, d1, vyc) in rig.disp:
        lm = []
        for cam, t in frames:
            tt = 0.35 * math.sin(2.0 * math.pi * t / 150.0)
            off, k, vy = cam * d0, cam * (d1 - d0) / W, cam * vyc
            lm.append((((1.0 / (1.0 + k), 0.0), (0.0, 1.0)), (-(off + tt) / (1.0 + k), -vy)))
        maps.append(lm)
    cam0, t0 = frames[0]
    seed = sc.seed * 1_000_003 + 7919 * (t0 * 64 + cam0) + 31
    return _layers_batch_nv12(sc.layers, maps, W, sc.height, torch.device(device), seed, sc.noise_sigma)


# --------------------------------------------------------------------------
# tables and sampling lists


def frame_bytes(width: int, height: int, pitch: Optional[int] = None) -> int:
    pitch = width if pitch is None else pitch
    return pitch * (height * 3 // 2)


def make_table(frame_fn, rows: Sequence[int], n_frames: int, width: int, height: int,
               pitch: Optional[int] = None, poison: int = 0xFF, device="cpu") -> torch.Tensor:
    """uint8 table [n_frames, frame_bytes]; `rows` are synthesised via frame_fn(row, device),
    every other row is filled with the poison byte."""
    pitch = width if pitch is None else pitch
    fb = frame_bytes(width, height, pitch)
    tab = torch.full((n_frames, fb), poison, dtype=torch.uint8, device=device)
    for r in rows:
        f = frame_fn(r, device)
        full = torch.full((height * 3 // 2, pitch), poison, dtype=torch.uint8, device=device)
        full[:, : f.shape[1]] = f[:, : min(f.shape[1], pitch)]
        tab[r] = full.reshape(-1)
    return tab


def gather_list(seed: int, n_frames: int, fraction: float) -> List[int]:
    """Seeded sorted index list of round(fraction * n_frames) distinct rows."""
    k = int(round(fraction * n_frames))
    rng = SplitMix64(seed)
    pool = list(range(n_frames))
    for i in range(k):  # partial Fisher-Yates
        j = i + rng.randint(n_frames - i)
        pool[i], pool[j] = pool[j], pool[i]
    return sorted(pool[:k])


def range_windows(seed: int, n_frames: int, window: int, count: int = 1) -> List[Tuple[int, int]]:
    """`count` disjoint half-open windows of `window` rows at seeded offsets."""
    rng = SplitMix64(seed)
    span = n_frames // count
    out = []
    for i in range(count):
        off = i * span + rng.randint(max(span - window + 1, 1))
        out.append((off, min(off + window, n_frames)))
    return out


def uniform_bytes(seed: int, shape, device="cpu") -> torch.Tensor:
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(seed)
    return torch.randint(0, 256, shape, generator=g, dtype=torch.uint8, device=device)
