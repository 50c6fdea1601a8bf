"""GPU parity of gather + NV12->RGB convert (+ resize) and HIST against the
oracle: bit-exact on every pixel and bin."""
import numpy as np
import pytest
import torch

import paper_1805_07339_amd as scn
import synth
from oracle import color as OC
from oracle import sampling as OS
from tests.helpers import c1_frames, frame_np, need_gpu, table_from_frames

pytestmark = pytest.mark.gpu


def _oracle_hist(tab, rows, w, h, pitch):
    return np.stack([OC.hist_frame(frame_np(tab, r, w, h, pitch), w, h) for r in rows])


def _oracle_convert(tab, rows, w, h, pitch, ow, oh, fmt):
    return np.stack([OC.convert(frame_np(tab, r, w, h, pitch), w, h, ow, oh, "gray8" if fmt else "rgb24")
                     for r in rows])


def test_hist_and_convert_c1_bitexact():
    need_gpu()
    frames, _ = c1_frames()
    tab = table_from_frames(frames, 16, list(range(16)), 320, 240)
    t = scn.Table.from_tensor(tab, 320, 240)
    job = scn.Job(t, scn.Sampling.stride(1, 0, 16))
    h = scn.hist(job)
    rgb = scn.sample_convert(job)
    torch.cuda.synchronize()
    exp = _oracle_hist(tab, range(16), 320, 240, 320)
    assert np.array_equal(h.cpu().numpy().astype(np.int64), exp.astype(np.int64))
    assert (h.cpu().numpy().sum(axis=2) == 320 * 240).all()
    assert np.array_equal(rgb.cpu().numpy(), _oracle_convert(tab, range(16), 320, 240, 320, 320, 240, 0))


def test_exhaustive_triples_frame_bitexact():
    need_gpu()
    from tests.test_oracle_color import exhaustive_frame
    y, u, v = exhaustive_frame()
    uv = np.stack([u, v], -1).reshape(2048, 4096)
    fr = torch.from_numpy(np.concatenate([y, uv], 0))
    tab = table_from_frames([fr], 1, [0], 4096, 4096)
    job = scn.Job(scn.Table.from_tensor(tab, 4096, 4096), scn.Sampling.stride(1, 0, 1))
    h = scn.hist(job).cpu().numpy()
    rgb = scn.sample_convert(job).cpu().numpy()
    exp_rgb = OC.nv12_to_rgb(y, u, v)
    assert np.array_equal(rgb[0], exp_rgb)
    assert np.array_equal(h[0].astype(np.int64), OC.hist16(exp_rgb).astype(np.int64))


@pytest.mark.parametrize("w,h,pitch", [(328, 240, 336), (330, 242, 330), (18, 4, 32), (2, 2, 2), (64, 2, 64)])
def test_ragged_and_unaligned_geometry(w, h, pitch):
    need_gpu()
    g = torch.Generator().manual_seed(w * 1000 + h)
    frames = [torch.randint(0, 256, (h * 3 // 2, pitch), generator=g, dtype=torch.uint8) for _ in range(5)]
    tab = table_from_frames(frames, 9, [0, 2, 4, 6, 8], w, h, pitch)
    job = scn.Job(scn.Table.from_tensor(tab, w, h, pitch), scn.Sampling.stride(2, 0, 9))
    hh = scn.hist(job).cpu().numpy()
    rgb = scn.sample_convert(job).cpu().numpy()
    gray = scn.sample_convert(job, fmt=scn.SCN_GRAY8).cpu().numpy()
    rows = [0, 2, 4, 6, 8]
    assert np.array_equal(hh.astype(np.int64), _oracle_hist(tab, rows, w, h, pitch).astype(np.int64))
    assert np.array_equal(rgb, _oracle_convert(tab, rows, w, h, pitch, w, h, 0))
    assert np.array_equal(gray, _oracle_convert(tab, rows, w, h, pitch, w, h, 1))


@pytest.mark.parametrize("ow,oh", [(160, 120), (224, 224), (640, 480), (97, 33), (1, 1)])
@pytest.mark.parametrize("fmt", [scn.SCN_RGB24, scn.SCN_GRAY8])
def test_resize_bitexact(ow, oh, fmt):
    need_gpu()
    frames, _ = c1_frames(n=3)
    tab = table_from_frames(frames, 3, [0, 1, 2], 320, 240)
    job = scn.Job(scn.Table.from_tensor(tab, 320, 240), scn.Sampling.gather([0, 2]))
    out = scn.sample_convert(job, ow, oh, fmt).cpu().numpy()
    assert np.array_equal(out, _oracle_convert(tab, [0, 2], 320, 240, 320, ow, oh, fmt))


def test_unsampled_rows_are_never_read():
    """Poison test (Sec. 4.2): changing every unsampled row leaves outputs bitwise unchanged."""
    need_gpu()
    frames, _ = c1_frames(n=6)
    rows = [3, 10, 11, 30]
    outs = []
    for poison in (0x00, 0xFF, 0x5A):
        tab = table_from_frames(frames[:4], 40, rows, 320, 240, poison=poison)
        job = scn.Job(scn.Table.from_tensor(tab, 320, 240), scn.Sampling.gather(rows))
        outs.append((scn.hist(job).cpu(), scn.sample_convert(job).cpu(), scn.sample_convert(job, 100, 50).cpu()))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


def test_sampling_kinds_and_empty():
    need_gpu()
    frames, _ = c1_frames(n=8)
    tab = table_from_frames(frames, 8, list(range(8)), 320, 240)
    t = scn.Table.from_tensor(tab, 320, 240)
    full = scn.hist(scn.Job(t, scn.Sampling.stride(1, 0, 8))).cpu()
    for samp, rows in [(scn.Sampling.stride(3, 1, 8), [1, 4, 7]), (scn.Sampling.gather([0, 5, 6]), [0, 5, 6]),
                       (scn.Sampling.range([(2, 4), (6, 8)]), [2, 3, 6, 7])]:
        h = scn.hist(scn.Job(t, samp)).cpu()
        assert torch.equal(h, full[rows])
    e = scn.hist(scn.Job(t, scn.Sampling.gather([])))
    assert e.shape == (0, 3, 16)


def test_hist_c2_1080p_stride24_sampled_parity():
    """1080p, 2400-row table, STRIDE-24 (100 rows): bin sums for every row,
    bit-exact oracle comparison on a seeded sample of rows."""
    need_gpu()
    W, H, N = 1920, 1080, 2400
    scene = synth.layered_scene(2, W, H)
    rows = OS.rows("stride", N, start=0, step=24, stop=N)
    fb = W * H * 3 // 2
    tab = torch.full((N, fb), 0xFF, dtype=torch.uint8, device="cuda")
    for r in rows:
        tab[r] = scene.nv12(r, device="cuda").reshape(-1)
    job = scn.Job(scn.Table.from_tensor(tab, W, H), scn.Sampling.stride(24, 0, N))
    h = scn.hist(job).cpu().numpy()
    assert (h.sum(axis=2) == W * H).all()
    for k in [0, 37, 99]:
        exp = OC.hist_frame(frame_np(tab, rows[k], W, H, W), W, H)
        assert np.array_equal(h[k].astype(np.int64), exp.astype(np.int64))
    rgb = scn.sample_convert(scn.Job(scn.Table.from_tensor(tab, W, H), scn.Sampling.gather([rows[5]])))
    assert np.array_equal(rgb[0].cpu().numpy(), OC.convert(frame_np(tab, rows[5], W, H, W), W, H))
