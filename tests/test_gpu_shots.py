"""Shot-boundary cue on the GPU (HIST, then the histogram distance of each
S[0,1] pair and the cut flag) against the oracle, bit-exact: streams made of
several synthetic shots with hard cuts, RANGE windows (no pair across a
window), threshold extremes, no cut output, a single row, and a 1080p
stream."""
import numpy as np
import pytest
import torch

import paper_1805_07339_amd as scn
import synth
from oracle import color as OC
from oracle import sampling as OS
from oracle import shots as SH
from tests.helpers import frame_np, need_gpu, table_from_frames

pytestmark = pytest.mark.gpu


def _shots_stream(w, h, n, cuts, seed, pitch=None):
    """n frames: a new layered scene starts at each frame index in `cuts`."""
    frames, scene, k = [], None, 0
    for t in range(n):
        if t == 0 or t in cuts:
            scene = synth.layered_scene(seed + 101 * k, w, h)
            k += 1
        frames.append(scene.nv12(t))
    tab = table_from_frames(frames, n, list(range(n)), w, h, pitch=pitch)
    return tab


def _oracle_d(tab, slices, w, h, pitch):
    rows = [r for s in slices for r in s]
    hs = np.stack([OC.hist_frame(frame_np(tab, r, w, h, pitch), w, h) for r in rows])
    return SH.pair_distances(hs, SH.pair_slots(slices)), hs


def test_cuts_of_a_three_shot_stream():
    need_gpu()
    w, h, n, cuts = 320, 240, 12, (4, 9)
    tab = _shots_stream(w, h, n, cuts, 7)
    job = scn.Job(scn.Table.from_tensor(tab, w, h), scn.Sampling.stride(1, 0, n))
    hist = scn.hist(job)
    exp, hs = _oracle_d(tab, OS.slices("stride", n, start=0, step=1, stop=n), w, h, w)
    assert np.array_equal(hist.cpu().numpy().astype(np.int64), hs.astype(np.int64))
    inner = np.delete(exp, [c - 1 for c in cuts])
    thr = (int(inner.max()) + int(min(exp[c - 1] for c in cuts))) // 2
    assert inner.max() < thr < min(exp[c - 1] for c in cuts)
    d, cut = scn.hist_diff(job, hist, thr)
    assert d.cpu().numpy().tolist() == exp.tolist()
    assert cut.cpu().numpy().tolist() == [1 if k + 1 in cuts else 0 for k in range(n - 1)]
    assert cut.cpu().numpy().tolist() == SH.cuts(exp, thr).tolist()


def test_range_windows_threshold_extremes_and_no_cut_output():
    need_gpu()
    w, h, n = 160, 96, 14
    pitch = 171  # odd pitch: the HIST reads take the scalar path
    tab = _shots_stream(w, h, n, (3, 8), 11, pitch=pitch)
    windows = [(0, 4), (6, 12)]
    job = scn.Job(scn.Table.from_tensor(tab, w, h, pitch), scn.Sampling.range(windows))
    hist = scn.hist(job)
    sl = OS.slices("range", n, idx=[v for wnd in windows for v in wnd])
    exp, _ = _oracle_d(tab, sl, w, h, pitch)
    assert len(exp) == scn.count_pairs(job) == 3 + 5
    for thr in (0, 1, int(np.median(exp)), 0xFFFFFFFF):
        d, cut = scn.hist_diff(job, hist, thr)
        assert d.cpu().numpy().tolist() == exp.tolist()
        assert cut.cpu().numpy().tolist() == SH.cuts(exp, thr).tolist()
    d, cut = scn.hist_diff(job, hist, 0, with_cut=False)
    assert cut is None and d.cpu().numpy().tolist() == exp.tolist()
    # a single sampled row: no pairs, nothing to do
    one = scn.Job(scn.Table.from_tensor(tab, w, h, pitch), scn.Sampling.gather([5]))
    d, cut = scn.hist_diff(one, scn.hist(one), 0)
    assert d.numel() == 0 and cut.numel() == 0


def test_1080p_stream_every_pair():
    need_gpu()
    w, h, n = 1920, 1080, 6
    tab = _shots_stream(w, h, n, (3,), 23)
    job = scn.Job(scn.Table.from_tensor(tab, w, h), scn.Sampling.stride(1, 0, n))
    thr = 50_000  # between the within-shot distances (~1.2e4) and the cut's (~1e5) on this stream
    d, cut = scn.hist_diff(job, scn.hist(job), thr)
    exp, _ = _oracle_d(tab, OS.slices("stride", n, start=0, step=1, stop=n), w, h, w)
    print("1080p distances:", exp.tolist(), flush=True)
    assert d.cpu().numpy().tolist() == exp.tolist()
    assert cut.cpu().numpy().tolist() == SH.cuts(exp, thr).tolist() == [0, 0, 1, 0, 0]
