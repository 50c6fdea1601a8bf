"""Pins of the shot-boundary oracle (histogram differences over the S[0,1]
pairs) against closed forms, invariants, brute-force counts and a synthetic
hard cut."""
import numpy as np

import synth
from oracle import color as C
from oracle import sampling as OS
from oracle import shots as SH


def _const_frame(w, h, y, u, v):
    f = np.empty((h * 3 // 2, w), dtype=np.uint8)
    f[:h] = y
    f[h:, 0::2] = u
    f[h:, 1::2] = v
    return f


def _random_frame(rng, w, h):
    return rng.integers(0, 256, size=(h * 3 // 2, w), dtype=np.uint8)


def test_identical_frames_give_zero():
    rng = np.random.default_rng(1)
    f = _random_frame(rng, 16, 8)
    h = C.hist_frame(f, 16, 8)
    assert SH.hist_l1(h, h) == 0


def test_black_to_white_is_six_w_h():
    # (16, 128, 128) -> (0, 0, 0): bin 0 of each channel; (235, 128, 128) ->
    # (255, 255, 255): bin 15.  Every pixel leaves one bin and enters another
    # in all three channels: 3 channels x 2 w h.
    w, h = 12, 6
    a = C.hist_frame(_const_frame(w, h, 16, 128, 128), w, h)
    b = C.hist_frame(_const_frame(w, h, 235, 128, 128), w, h)
    assert SH.hist_l1(a, b) == 6 * w * h


def test_half_frame_cut_is_three_w_h():
    w, h = 16, 8
    a = _const_frame(w, h, 16, 128, 128)
    b = a.copy()
    b[:h, w // 2:] = 235  # right half white (chroma stays neutral)
    assert SH.hist_l1(C.hist_frame(a, w, h), C.hist_frame(b, w, h)) == 3 * w * h


def test_symmetry_triangle_and_parity():
    rng = np.random.default_rng(2)
    w, h = 10, 6
    hs = [C.hist_frame(_random_frame(rng, w, h), w, h) for _ in range(6)]
    for i in range(6):
        for j in range(6):
            dij = SH.hist_l1(hs[i], hs[j])
            assert dij == SH.hist_l1(hs[j], hs[i])
            # both histograms hold w h pixels per channel: the distance is even
            assert dij % 2 == 0
            for k in range(6):
                assert dij <= SH.hist_l1(hs[i], hs[k]) + SH.hist_l1(hs[k], hs[j])


def test_brute_force_counts_on_tiny_frames():
    """Per-pixel interval counting (no bincount, no shifts) and an explicit
    double loop over channels and bins give the same distance."""
    rng = np.random.default_rng(3)
    for w, h in [(2, 2), (4, 2), (6, 4)]:
        f1, f2 = _random_frame(rng, w, h), _random_frame(rng, w, h)
        rgb1 = C.nv12_to_rgb(*C.split_nv12(f1, w, h))
        rgb2 = C.nv12_to_rgb(*C.split_nv12(f2, w, h))

        def counts(rgb):
            out = [[0] * 16 for _ in range(3)]
            for px in rgb.reshape(-1, 3):
                for c in range(3):
                    for k in range(16):
                        if 16 * k <= int(px[c]) < 16 * k + 16:
                            out[c][k] += 1
            return out

        c1, c2 = counts(rgb1), counts(rgb2)
        d = 0
        for c in range(3):
            for k in range(16):
                d += abs(c1[c][k] - c2[c][k])
        assert SH.hist_l1(C.hist_frame(f1, w, h), C.hist_frame(f2, w, h)) == d


def test_pairs_stay_within_range_windows():
    sl = OS.slices("range", 20, idx=[0, 3, 5, 8])
    assert SH.pair_slots(sl) == [(0, 1), (1, 2), (3, 4), (4, 5)]
    assert len(SH.pair_slots(sl)) == len(OS.pairs("range", 20, idx=[0, 3, 5, 8]))
    assert SH.pair_slots(OS.slices("stride", 10, start=0, step=3, stop=10)) == [(0, 1), (1, 2), (2, 3)]
    assert SH.pair_slots([[4]]) == []


def test_cuts_threshold_is_strict():
    d = np.array([0, 5, 6, 7])
    assert SH.cuts(d, 6).tolist() == [0, 0, 0, 1]
    assert SH.cuts(d, -1).tolist() == [1, 1, 1, 1]


def test_synthetic_hard_cut_is_found():
    """Two different layered scenes back to back: the pair across the cut is
    the only one above any threshold between the largest within-shot
    distance and the cut distance."""
    w, h, n, cut = 64, 48, 8, 5
    s1, s2 = synth.layered_scene(71, w, h), synth.layered_scene(72, w, h)
    frames = [(s1 if t < cut else s2).nv12(t).numpy() for t in range(n)]
    hs = np.stack([C.hist_frame(f, w, h) for f in frames])
    d = SH.pair_distances(hs, SH.pair_slots([list(range(n))]))
    inner = np.delete(d, cut - 1)
    assert d[cut - 1] > inner.max()
    thr = (int(inner.max()) + int(d[cut - 1])) // 2
    assert SH.cuts(d, thr).tolist() == [1 if k == cut - 1 else 0 for k in range(n - 1)]
