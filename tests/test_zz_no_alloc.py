"""scn_hist_static (HIST without a workspace, for callers that cannot
allocate) against scn_hist, through the C ABI: two calls in a row, the second
with a smaller job, so the second reads the fixed row table the first one
left behind and must overwrite what it uses.  Integer outputs: bit-exact."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1805_07339_amd as scn

pytestmark = pytest.mark.gpu


def _table(seed, w, h, n, pitch=None):
    g = np.random.default_rng(seed)
    pitch = w if pitch is None else pitch
    fb = pitch * h * 3 // 2
    host = torch.from_numpy(g.integers(0, 256, size=(n, fb), dtype=np.uint8))
    return scn.Table.from_tensor(host.cuda(), w, h, pitch)


def _via_ws(job):
    m = scn.count_rows(job)
    out = torch.full((m, 3, 16), -1, dtype=torch.int32, device="cuda")
    need = scn.workspace_bytes(scn.SCN_OP_HIST, [job])
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    st = scn.lib().scn_hist(ctypes.byref(job.cjob), out.data_ptr(), ws.data_ptr(), need,
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == scn.SCN_OK, scn.lib().scn_last_error()
    return out


def _static(job):
    m = scn.count_rows(job)
    out = torch.full((m, 3, 16), -1, dtype=torch.int32, device="cuda")
    st = scn.lib().scn_hist_static(ctypes.byref(job.cjob), out.data_ptr(),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == scn.SCN_OK, scn.lib().scn_last_error()
    return out


def test_hist_static_matches_hist_on_two_calls_in_a_row():
    print("hist_static: 1080p STRIDE-12 then 320x240 GATHER", flush=True)
    big = scn.Job(_table(11, 1920, 1080, 120), scn.Sampling.stride(12, 0, 120))  # rows 0, 12, ..., 108
    small_t = _table(12, 320, 240, 40, pitch=336)
    small = scn.Job(small_t, scn.Sampling.gather([2, 17, 39]))
    a1 = _static(big)
    b1 = _via_ws(big)
    a2 = _static(small)  # fewer rows: reuses the table's prefix
    b2 = _via_ws(small)
    torch.cuda.synchronize()
    assert a1.shape == (10, 3, 16) and a2.shape == (3, 3, 16)
    assert torch.equal(a1, b1)
    assert torch.equal(a2, b2)
    assert int(a1.sum()) == 10 * 3 * 1920 * 1080
    assert int(a2.sum()) == 3 * 3 * 320 * 240
