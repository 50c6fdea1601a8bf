"""GPU parity of pyramidal Horn-Schunck flow against the FP64 oracle:
max |du|, |dv| <= 1e-3 px on every pixel of every pair."""
import numpy as np
import pytest
import torch

import paper_1805_07339_amd as scn
import synth
from oracle import hs as OH
from oracle import sampling as OS
from oracle import warm as OW
from tests.helpers import c1_frames, frame_np, need_gpu, oracle_flows, table_from_frames

pytestmark = pytest.mark.gpu

TOL = 1e-3


def _oracle_pairs(tab, pairs, w, h, pitch, levels, alpha=10.0, iters=50):
    out = []
    for r1, r2 in pairs:
        y1 = frame_np(tab, r1, w, h, pitch)[:h, :w]
        y2 = frame_np(tab, r2, w, h, pitch)[:h, :w]
        u, v = OH.hs_flow(y1, y2, levels=levels, alpha=alpha, iters=iters)
        out.append(np.stack([u, v]))
    return np.stack(out)


def _maxdiff(gpu, exp):
    return float(np.abs(gpu.astype(np.float64) - exp).max())


def test_flow_c1_parity():
    need_gpu()
    frames, _ = c1_frames()
    tab = table_from_frames(frames, 16, list(range(16)), 320, 240)
    job = scn.Job(scn.Table.from_tensor(tab, 320, 240), scn.Sampling.stride(1, 0, 16))
    (f,) = scn.flow([job], scn.flow_params(levels=3))
    f = f.cpu().numpy()
    assert f.shape == (15, 2, 240, 320)
    exp = _oracle_pairs(tab, [(i, i + 1) for i in range(15)], 320, 240, 320, 3)
    d = _maxdiff(f, exp)
    print("C1 max |d| = %.3g" % d)
    assert d <= TOL


def test_identical_frames_give_exact_zero():
    need_gpu()
    frames, _ = c1_frames(n=2)
    tab = table_from_frames([frames[0], frames[0]], 2, [0, 1], 320, 240)
    job = scn.Job(scn.Table.from_tensor(tab, 320, 240), scn.Sampling.stride(1, 0, 2))
    (f,) = scn.flow([job], scn.flow_params(levels=3))
    assert (f == 0).all()


@pytest.mark.parametrize("w,h,levels,iters", [(250, 186, 4, 50), (66, 34, 2, 7), (2 * 17, 2 * 9, 1, 3),
                                              (128, 96, 3, 0), (96, 64, 5, 1)])
def test_ragged_sizes_levels_iters(w, h, levels, iters):
    need_gpu()
    frames, _ = c1_frames(n=3, w=w, h=h, seed=w + h)
    tab = table_from_frames(frames, 3, [0, 1, 2], w, h)
    job = scn.Job(scn.Table.from_tensor(tab, w, h), scn.Sampling.stride(1, 0, 3))
    (f,) = scn.flow([job], scn.flow_params(levels=levels, iters=iters))
    exp = _oracle_pairs(tab, [(0, 1), (1, 2)], w, h, w, levels, iters=iters)
    assert _maxdiff(f.cpu().numpy(), exp) <= TOL


def test_uneven_jobs_and_slices_one_call():
    need_gpu()
    fa, _ = c1_frames(n=6, w=160, h=120, seed=3)
    fb, _ = c1_frames(n=6, w=96, h=64, seed=4)
    ta = table_from_frames(fa, 20, [0, 2, 4, 6, 8, 10], 160, 120)
    tb = table_from_frames(fb, 10, [1, 2, 3, 6, 7, 8], 96, 64, pitch=112)
    ja = scn.Job(scn.Table.from_tensor(ta, 160, 120), scn.Sampling.stride(2, 0, 11))
    jb = scn.Job(scn.Table.from_tensor(tb, 96, 64, 112), scn.Sampling.range([(1, 4), (6, 9)]))
    fa_out, fb_out = scn.flow([ja, jb], scn.flow_params(levels=3))
    assert fa_out.shape[0] == 5 and fb_out.shape[0] == 4
    ea = _oracle_pairs(ta, OS.pairs("stride", 20, start=0, step=2, stop=11), 160, 120, 160, 3)
    eb = _oracle_pairs(tb, OS.pairs("range", 10, idx=[1, 4, 6, 9]), 96, 64, 112, 3)
    assert _maxdiff(fa_out.cpu().numpy(), ea) <= TOL
    assert _maxdiff(fb_out.cpu().numpy(), eb) <= TOL


def test_stencil_before_sampling_flow():
    """Stencil before sampling: each sampled row s gives the pair (s, s+1) of
    original rows.  Only the sampled rows and their successors hold frames
    (every other row is poison); the sampled last row of the table has no
    pair; each pair matches the oracle on its two frames; the same frames as
    an after-sampling job of consecutive rows give bitwise the same flow."""
    need_gpu()
    w, h, n = 160, 120, 40
    sampled = [3, 17, 25, 39]
    pairs = OS.pairs_before("gather", n, idx=sampled)
    assert pairs == [(3, 4), (17, 18), (25, 26)]
    rows = sorted({r for p in pairs for r in p} | set(sampled))
    frames, _ = c1_frames(n=len(rows), w=w, h=h, seed=77)
    tab = table_from_frames(frames, n, rows, w, h)
    job = scn.Job(scn.Table.from_tensor(tab, w, h), scn.Sampling.gather(sampled).before())
    assert scn.count_pairs(job) == 3
    (f,) = scn.flow([job], scn.flow_params(levels=3))
    assert f.shape == (3, 2, h, w)
    d = _maxdiff(f.cpu().numpy(), _oracle_pairs(tab, pairs, w, h, w, 3))
    print("stencil-before max |d| = %.3g" % d, flush=True)
    assert d <= TOL
    # pair (17, 18) as a RANGE window of the after-sampling stencil: same work, same bits
    (g,) = scn.flow([scn.Job(scn.Table.from_tensor(tab, w, h), scn.Sampling.range([(17, 19)]))],
                    scn.flow_params(levels=3))
    assert torch.equal(g[0], f[1])


def _constant_motion_frames(n, d, w, h, seed, noise=2.0):
    rng = synth.SplitMix64(seed)
    tex = synth.Texture.random(rng)
    tu = synth.Texture.random(rng, sigma=20.0)
    tv = synth.Texture.random(rng, sigma=20.0)
    lay = synth.Layer(tex, tu, tv, "full", shifts=[(t * d[0], t * d[1]) for t in range(n)])
    sc = synth.Scene(w, h, [lay], seed, noise)
    return [sc.nv12(t) for t in range(n)]


def test_warm_start_chain_matches_the_oracle():
    """Temporal warm start, packets of 3 pairs over two RANGE slices (pairs
    0-4 and 6-7): every pair within 1e-3 px of the oracle's chain; a
    workspace that forces chunking gives the same bits; packets of 1 are
    the cold solve bit for bit."""
    need_gpu()
    w, h, n = 160, 120, 9
    frames = _constant_motion_frames(n, (0.8, -0.45), w, h, 31)
    tab = table_from_frames(frames, n, list(range(n)), w, h)
    job = scn.Job(scn.Table.from_tensor(tab, w, h), scn.Sampling.range([(0, 6), (6, 9)]))
    prm = scn.flow_params(3, 10.0, 50, warm_packet=3, warm_iters=10)
    (f,) = scn.flow([job], prm)
    ys = [frame_np(tab, r, w, h, w)[:h, :w] for r in range(n)]
    slices = [[(ys[r], ys[r + 1]) for r in range(0, 5)], [(ys[r], ys[r + 1]) for r in range(6, 8)]]
    exp = OW.warm_chain(slices, 3, 3, 10.0, 50, 10)
    exp = np.stack([np.stack([u, v]) for u, v in exp])
    d = _maxdiff(f.cpu().numpy(), exp)
    print("warm chain max |d| = %.3g" % d, flush=True)
    assert d <= TOL
    # the cold pairs of each packet are the plain solve
    (plain,) = scn.flow([job], scn.flow_params(3, 10.0, 50))
    for k in (0, 3, 5):
        assert torch.equal(f[k], plain[k])
    # chunked workspace: the same bits
    need = scn.workspace_bytes(scn.SCN_OP_FLOW, [job], prm)
    small = need // 3
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    (g,) = scn.flow([job], prm, ws=ws, ws_bytes=small)
    assert torch.equal(f, g)
    (one,) = scn.flow([job], scn.flow_params(3, 10.0, 50, warm_packet=1, warm_iters=10))
    assert torch.equal(one, plain)
    # zero warm iterations: a later pair returns its start, its predecessor's
    # flow, bit for bit; a packet longer than a slice restarts at the next slice
    (z,) = scn.flow([job], scn.flow_params(3, 10.0, 50, warm_packet=100, warm_iters=0))
    for k in range(1, 5):
        assert torch.equal(z[k], z[0])
    assert torch.equal(z[5], plain[5]) and torch.equal(z[6], z[5])


def test_odd_pitch_rows_unaligned():
    """An odd pitch puts every odd row at an odd address: the level-0
    pyramid's word loads and the setup's paired-column warp loads then run
    unaligned; the flow still matches the oracle."""
    need_gpu()
    w, h, pitch = 320, 240, 333
    frames, _ = c1_frames(n=3, w=w, h=h, seed=41)
    tab = table_from_frames(frames, 3, [0, 1, 2], w, h, pitch=pitch)
    job = scn.Job(scn.Table.from_tensor(tab, w, h, pitch), scn.Sampling.stride(1, 0, 3))
    (f,) = scn.flow([job], scn.flow_params(levels=3))
    exp = _oracle_pairs(tab, [(0, 1), (1, 2)], w, h, pitch, 3)
    assert _maxdiff(f.cpu().numpy(), exp) <= TOL


def test_chunked_workspace_is_bitwise_identical():
    need_gpu()
    frames, _ = c1_frames(n=9, w=128, h=96)
    tab = table_from_frames(frames, 9, list(range(9)), 128, 96)
    job = scn.Job(scn.Table.from_tensor(tab, 128, 96), scn.Sampling.stride(1, 0, 9))
    p = scn.flow_params(levels=3)
    (full,) = scn.flow([job], p)
    full = full.clone()
    # workspace for about 2 pairs at a time
    need = scn.workspace_bytes(scn.SCN_OP_FLOW, [job], p)
    small = need // 4
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    (chunked,) = scn.flow([job], p, ws=ws)
    assert torch.equal(full, chunked)


def test_unsampled_rows_are_never_read():
    need_gpu()
    frames, _ = c1_frames(n=4, w=128, h=96)
    rows = [2, 9, 10, 17]
    res = []
    for poison in (0x00, 0xFF):
        tab = table_from_frames(frames, 20, rows, 128, 96, poison=poison)
        job = scn.Job(scn.Table.from_tensor(tab, 128, 96), scn.Sampling.gather(rows))
        (f,) = scn.flow([job], scn.flow_params(levels=3))
        res.append(f.cpu())
    assert torch.equal(res[0], res[1])


def test_flow_c2_1080p_sampled_pairs():
    """The benchmark's 1080p call: the layered-affine stream sampled STRIDE-24
    (99 pairs) and by the seeded 1% GATHER (23 pairs), both jobs in one call
    as the benchmark times them; three STRIDE pairs and two GATHER pairs
    against the oracle."""
    need_gpu()
    W, H, N = 1920, 1080, 2400
    scene = synth.layered_scene(2, W, H)
    rows = OS.rows("stride", N, start=0, step=24, stop=N)
    grows = synth.gather_list(2, N, 0.01)
    fb = W * H * 3 // 2
    tab = torch.full((N, fb), 0xFF, dtype=torch.uint8, device="cuda")
    for r in sorted(set(rows) | set(grows)):
        tab[r] = scene.nv12(r, device="cuda").reshape(-1)
    t = scn.Table.from_tensor(tab, W, H)
    js, jg = scn.Job(t, scn.Sampling.stride(24, 0, N)), scn.Job(t, scn.Sampling.gather(grows))
    fs, fg = scn.flow([js, jg], scn.flow_params(levels=4))
    assert fs.shape == (99, 2, H, W) and fg.shape == (23, 2, H, W)
    prs = OS.pairs("stride", N, start=0, step=24, stop=N)
    pgs = OS.pairs("gather", N, idx=grows)
    cases = [("stride", k, fs, prs[k]) for k in (0, 50, 98)] + [("gather", k, fg, pgs[k]) for k in (0, 22)]
    exp = oracle_flows([(frame_np(tab, a, W, H, W)[:H], frame_np(tab, b, W, H, W)[:H]) for *_, (a, b) in cases], 4)
    for (kind, k, f, pr), e in zip(cases, exp):
        d = _maxdiff(f[k].cpu().numpy(), e)
        print("C2 %s pair %d %s max |d| = %.3g" % (kind, k, pr, d))
        assert d <= TOL


@pytest.mark.parametrize("w,h,levels", [(320, 240, 3), (250, 186, 4), (130, 34, 2)])
def test_jacobi_schedules_are_bitwise_identical(w, h, levels):
    """Every Jacobi schedule (one sweep per launch, or k sweeps per launch on
    each register-tile variant, or the autotuned choice) gives the same bits."""
    need_gpu()
    frames, _ = c1_frames(n=3, w=w, h=h, seed=7 + w)
    tab = table_from_frames(frames, 3, [0, 1, 2], w, h)
    job = scn.Job(scn.Table.from_tensor(tab, w, h), scn.Sampling.stride(1, 0, 3))
    (ref,) = scn.flow([job], scn.flow_params(levels=levels, sweeps_per_pass=1))
    ref = ref.clone()
    exp = _oracle_pairs(tab, [(0, 1), (1, 2)], w, h, w, levels)
    assert _maxdiff(ref.cpu().numpy(), exp) <= TOL
    for variant in range(1, 19):
        for k in (2, 5, 8, 13, 17):
            (f,) = scn.flow([job], scn.flow_params(levels=levels, sweeps_per_pass=k, tile_variant=variant))
            assert torch.equal(f, ref), (variant, k)
    (f,) = scn.flow([job], scn.flow_params(levels=levels))
    assert torch.equal(f, ref)


def test_jobs_without_pairs_in_a_batch():
    """Degenerate jobs -- a single sampled row (no pair), an empty gather and
    a RANGE of one-row windows -- in one call with a normal job: the call
    succeeds, the empty jobs get no work and the normal job's flow equals
    its solo call bit for bit."""
    need_gpu()
    frames, _ = c1_frames(n=4, w=96, h=64, seed=5)
    tab = table_from_frames(frames, 4, [0, 1, 2, 3], 96, 64)
    t = scn.Table.from_tensor(tab, 96, 64)
    full = scn.Job(t, scn.Sampling.stride(1, 0, 4))
    single = scn.Job(t, scn.Sampling.stride(5, 2, 3))
    empty = scn.Job(t, scn.Sampling.gather([]))
    ones = scn.Job(t, scn.Sampling.range([(0, 1), (2, 3)]))
    for j in (single, empty, ones):
        assert scn.count_pairs(j) == 0
    p = scn.flow_params(levels=2)
    (solo,) = scn.flow([full], p)
    outs = scn.flow([single, full, empty, ones], p)
    assert [o.shape[0] for o in outs] == [0, 3, 0, 0]
    assert torch.equal(outs[1], solo)


def test_timing_units_count_pixel_passes():
    """The Jacobi timers' work units are the level's pixels x the pairs of
    every pass over the planes (the benchmark forms algorithmic bytes per
    launch from them): 5 passes of 10 sweeps on the streaming kernel, 50
    one-sweep launches on the reference schedule."""
    need_gpu()
    w, h, levels = 160, 120, 3
    frames, _ = c1_frames(n=3, w=w, h=h, seed=3)
    tab = table_from_frames(frames, 3, [0, 1, 2], w, h)
    job = scn.Job(scn.Table.from_tensor(tab, w, h), scn.Sampling.stride(1, 0, 3))
    sizes = [(160, 120), (80, 60), (40, 30)]
    for variant, k, passes in ((9, 10, 5), (0, 1, 50)):
        p = scn.flow_params(levels=levels, sweeps_per_pass=k, tile_variant=variant)
        scn.flow([job], p)
        torch.cuda.synchronize()
        scn.timing_enable(True, 4096)
        scn.timing_reset()
        scn.flow([job], p)
        torch.cuda.synchronize()
        for lv, (lw, lh) in enumerate(sizes):
            assert scn.timing_units("hs_jacobi_l%d" % lv) == lw * lh * 2 * passes, (variant, lv)
        assert scn.timing_units("hs_jacobi") == sum(lw * lh for lw, lh in sizes) * 2 * passes
        assert scn.timing_units("hs_setup") == 0
        scn.timing_enable(False)


@pytest.mark.parametrize("warm", [0, 2])
def test_graph_capture_replays_match_eager(warm):
    """After one eager call (plan upload, tuning), the flow and HIST calls of an
    uneven multi-job batch are captured into a HIP graph; every replay, with
    eager work in between, reproduces the eager result bit for bit (also with
    the warm start, whose later pairs read their predecessors' outputs)."""
    need_gpu()
    fa, _ = c1_frames(n=4, w=160, h=120, seed=21)
    fb, _ = c1_frames(n=4, w=96, h=64, seed=22)
    ta = table_from_frames(fa, 4, [0, 1, 2, 3], 160, 120)
    tb = table_from_frames(fb, 4, [0, 1, 2, 3], 96, 64)
    ja = scn.Job(scn.Table.from_tensor(ta, 160, 120), scn.Sampling.stride(1, 0, 4))
    jb = scn.Job(scn.Table.from_tensor(tb, 96, 64), scn.Sampling.range([(0, 4)]))
    p = scn.flow_params(levels=3, warm_packet=warm, warm_iters=5)
    outs = [torch.empty((3, 2, 120, 160), device="cuda"), torch.empty((3, 2, 64, 96), device="cuda")]
    hist = torch.empty((4, 3, 16), dtype=torch.int32, device="cuda")
    ws = torch.empty(scn.workspace_bytes(scn.SCN_OP_FLOW, [ja, jb], p), dtype=torch.uint8, device="cuda")
    wsh = torch.empty(scn.workspace_bytes(scn.SCN_OP_HIST, [ja]), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        scn.flow([ja, jb], p, outs=outs, ws=ws)
        scn.hist(ja, out=hist, ws=wsh)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    href = hist.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        scn.flow([ja, jb], p, outs=outs, ws=ws)
        scn.hist(ja, out=hist, ws=wsh)
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        hist.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(o, r) for o, r in zip(outs, ref)), rep
        assert torch.equal(hist, href), rep
        _ = torch.randn(1000, device="cuda").sum()  # eager work between replays
