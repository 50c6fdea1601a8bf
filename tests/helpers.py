"""Shared helpers for the GPU parity tests: seeded tables on the host, copied
to the device, and the oracle run on the same bytes."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synth


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def table_from_frames(frames, n_frames, rows, width, height, pitch=None, poison=0xFF, device="cuda"):
    """uint8 [n_frames, frame_bytes] with frames[k] at rows[k]; other rows poison-filled."""
    pitch = width if pitch is None else pitch
    fb = pitch * height * 3 // 2
    tab = torch.full((n_frames, fb), poison, dtype=torch.uint8)
    for r, f in zip(rows, frames):
        full = torch.full((height * 3 // 2, pitch), poison, dtype=torch.uint8)
        full[:, :width] = f[:, :width]
        tab[r] = full.reshape(-1)
    return tab.to(device)


def c1_frames(n=16, noise=2.0, w=320, h=240, seed=1):
    s, ds = synth.translation_scene(seed, w, h, n, noise_sigma=noise)
    return [s.nv12(t) for t in range(n)], ds


def frame_np(tab: torch.Tensor, row: int, width: int, height: int, pitch: int) -> np.ndarray:
    return tab[row].cpu().numpy().reshape(height * 3 // 2, pitch)


def _oracle_flow_job(args):
    from oracle import hs as OH
    y1, y2, levels, alpha, iters = args
    u, v = OH.hs_flow(y1, y2, levels=levels, alpha=alpha, iters=iters)
    return np.stack([u, v])


def oracle_flows(luma_pairs, levels, alpha=10.0, iters=50):
    """FP64 oracle flow of each (Y1, Y2) luma pair, one pair per process
    (spawned interpreters that never touch the GPU)."""
    import multiprocessing as mp
    import os
    jobs = [(a, b, levels, alpha, iters) for a, b in luma_pairs]
    if len(jobs) <= 1:
        return [_oracle_flow_job(j) for j in jobs]
    n = max(1, min(len(jobs), len(os.sched_getaffinity(0)), 16))
    with mp.get_context("spawn").Pool(n) as pool:
        return pool.map(_oracle_flow_job, jobs, chunksize=1)
