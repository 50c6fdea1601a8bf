"""Pins of the surrogate oracle: BF16 rounding vs torch, conv forward vs
torch conv2d (FP64), backward vs torch FP64 autograd and central finite
differences, Adam vs its closed form on a linear objective, the upsampling
operator vs its adjoint, the Charbonnier gradient vs finite differences."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import surrogate as S


def test_bf16_rne_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e3, 2000), rng.normal(0, 1e-3, 2000)])
    x32 = x.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x32).float().to(torch.bfloat16).double().numpy()
    assert np.array_equal(S.bf16_rne(x32), ref)
    assert S.bf16_rne(np.array([1 + 2 ** -8]))[0] == 1.0
    assert S.bf16_rne(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    assert S.bf16_rne(np.array([-(1 + 2 ** -8)]))[0] == -1.0
    # the network input is exact in BF16
    v = np.arange(256)
    assert np.array_equal(S.bf16_rne((v - 128) / 64.0), (v - 128) / 64.0)


def test_half_gray_round_half_up():
    y = np.array([[0, 1, 2, 3], [1, 1, 2, 2]], np.uint8)
    # block sums 3 and 9 -> (3+2)>>2 = 1, (9+2)>>2 = 2
    assert np.array_equal(S.half_gray(y), (np.array([[1, 2]]) - 128) / 64.0)


@pytest.mark.parametrize("stride,H,W", [(1, 7, 9), (2, 8, 10), (2, 9, 7), (1, 2, 2)])
def test_conv_forward_matches_torch(stride, H, W):
    rng = np.random.default_rng(stride * 100 + H)
    x = S.bf16_rne(rng.normal(size=(5, H, W)))
    w = S.bf16_rne(rng.normal(size=(4, 5, 3, 3)))
    b = rng.normal(size=4)
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w), torch.from_numpy(b), stride=stride,
                   padding=1)[0].numpy()
    out = S.conv3x3(x, w, b, stride)
    assert out.shape == ref.shape
    assert np.abs(out - ref).max() < 1e-12


def _torch_net(params, x):
    """The same network in torch FP64 without rounding (autograd reference)."""
    a = torch.from_numpy(x)[None]
    for name, ci, co, stride, up, relu in S.LAYERS:
        if up:
            a = a.repeat_interleave(2, dim=2).repeat_interleave(2, dim=3)
        a = F.conv2d(a, params[name + ".w"], params[name + ".b"], stride=stride, padding=1)
        if relu:
            a = torch.relu(a)
    return a[0]


def _small_problem(seed=3, H=24, W=32):
    rng = np.random.default_rng(seed)
    params = S.init_params(seed)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng.normal(0, 0.05, params[k].shape)
    y1 = rng.integers(0, 256, (H, W)).astype(np.uint8)
    y2 = rng.integers(0, 256, (H, W)).astype(np.uint8)
    target = rng.normal(0, 1.0, (2, H, W))
    return params, y1, y2, target


def test_backward_matches_torch_autograd():
    params, y1, y2, target = _small_problem()
    x = S.net_input(y1, y2)
    loss, grads = S.loss_and_grads(params, x, target, rounding=False)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in params.items()}
    half = _torch_net(tp, x)
    # full-resolution flow through the same linear upsampling
    My = torch.from_numpy(S.upsample_flow_matrix_1d(half.shape[1]))
    Mx = torch.from_numpy(S.upsample_flow_matrix_1d(half.shape[2]))
    full = 2.0 * torch.einsum("yh,chw,xw->cyx", My, half, Mx)
    d = full - torch.from_numpy(target)
    tl = torch.sqrt(d[0] ** 2 + d[1] ** 2 + S.CHARB_EPS ** 2).mean()
    tl.backward()
    assert abs(float(tl) - loss) < 1e-12
    for k in params:
        ref = tp[k].grad.numpy()
        assert np.abs(grads[k] - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max()), k


def test_backward_matches_central_differences():
    params, y1, y2, target = _small_problem(seed=5)
    x = S.net_input(y1, y2)
    _, grads = S.loss_and_grads(params, x, target, rounding=False)
    rng = np.random.default_rng(9)
    for name in ["conv1.w", "conv3.w", "conv4.b", "conv6.w", "conv2.b"]:
        p = params[name]
        for _ in range(4):
            idx = tuple(rng.integers(0, n) for n in p.shape)
            h = 1e-5 * max(1.0, abs(p[idx]))
            old = p[idx]
            p[idx] = old + h
            lp, _ = S.loss_and_grads(params, x, target, rounding=False)
            p[idx] = old - h
            lm, _ = S.loss_and_grads(params, x, target, rounding=False)
            p[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, grads[name][idx])


def test_upsample_operators_are_adjoint_and_exact():
    rng = np.random.default_rng(1)
    h, w = 6, 10
    half = rng.normal(size=(2, h, w))
    g = rng.normal(size=(2, 2 * h, 2 * w))
    assert abs((S.flow_full(half) * g).sum() - (half * S.flow_full_adjoint(g, h, w)).sum()) < 1e-10
    assert np.allclose(S.flow_full(np.full((2, h, w), 1.5)), 3.0)
    ramp = np.broadcast_to(np.arange(w, dtype=float), (2, h, w)).copy()
    full = S.flow_full(ramp)
    xs = np.arange(2 * w)
    exp = 2.0 * np.clip((xs + 0.5) / 2 - 0.5, 0, w - 1)
    assert np.allclose(full[0, 3], exp)
    x = rng.normal(size=(3, h, w))
    y = rng.normal(size=(3, 2 * h, 2 * w))
    assert abs((S.upsample2(x) * y).sum() - (x * S.upsample2_adjoint(y)).sum()) < 1e-10


def test_charbonnier_gradient_fd():
    rng = np.random.default_rng(2)
    full = rng.normal(size=(2, 5, 6))
    tgt = rng.normal(size=(2, 5, 6))
    _, g = S.charbonnier_loss(full, tgt)
    for _ in range(10):
        idx = tuple(rng.integers(0, n) for n in full.shape)
        h = 1e-6
        a = full.copy(); a[idx] += h
        b = full.copy(); b[idx] -= h
        fd = (S.charbonnier_loss(a, tgt)[0] - S.charbonnier_loss(b, tgt)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-8


def test_adam_linear_objective_closed_form():
    # constant gradient c: bias-corrected moments are exactly c and c^2, so every
    # step moves by lr * c / (|c| + eps)
    c, lr, eps = 0.37, 1e-2, 1e-8
    params = {"w": np.array([2.0])}
    opt = S.Adam(params, lr=lr, eps=eps)
    for t in range(1, 51):
        opt.step(params, {"w": np.array([c])})
        assert abs(params["w"][0] - (2.0 - t * lr * c / (abs(c) + eps))) < 1e-12


def test_param_count():
    assert S.n_params() == 148898


def test_residual_gate_statistic():
    import synth
    s, ds = synth.translation_scene(4, 64, 48, 2, noise_sigma=0.0)
    y1 = s.nv12(0).numpy()[:48]
    assert S.warp_residual(y1, y1, np.zeros((2, 48, 64))) == 0.0
    # an integer shift warped back by its exact flow leaves only the border
    y2 = np.zeros_like(y1)
    y2[:, 3:] = y1[:, :-3]
    flow = np.zeros((2, 48, 64)); flow[0] = 3.0
    r_full = S.warp_residual(y1, y2, flow)
    r_zero = S.warp_residual(y1, y2, np.zeros((2, 48, 64)))
    assert r_full < r_zero
    from oracle.hs import warp
    assert np.array_equal(warp(y2.astype(float), flow[0], flow[1])[:, :-3], y1[:, :-3].astype(float))


def test_epe_closed_forms():
    """EPE (per-pixel endpoint distance, mean over pixels): zero against
    itself; a constant (3, 4) offset gives exactly 5; half the pixels off by
    (0, 2) and half exact gives 1 (catches a squared, summed or per-component
    error measure)."""
    rng = np.random.default_rng(3)
    f = rng.normal(size=(2, 6, 8))
    assert S.epe(f, f) == 0.0
    off = f.copy()
    off[0] += 3.0
    off[1] += 4.0
    assert abs(S.epe(off, f) - 5.0) < 1e-12
    half = f.copy()
    half[1, :3] += 2.0
    assert abs(S.epe(half, f) - 1.0) < 1e-12
