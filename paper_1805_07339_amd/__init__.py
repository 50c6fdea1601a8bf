"""Python binding of libscn (ctypes; argument marshalling only).

Every step of the pixel stage runs in libscn's HIP kernels.  PyTorch is used
for device memory (input tables, outputs, the workspace pool) and for the
stream handle; nothing here computes pixels.  Importing the package does not
need a GPU; calling into the library needs the built libscn.so and fails
loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libscn.so")

SCN_OK, SCN_EINVAL, SCN_EUNSUPPORTED, SCN_ENOSPACE, SCN_EHIP = 0, -1, -2, -3, -4
SCN_STRIDE, SCN_GATHER, SCN_RANGE = 0, 1, 2
SCN_STENCIL_AFTER, SCN_STENCIL_BEFORE = 0, 1
SCN_SPACE_NULL, SCN_SPACE_REPEAT = 0, 1
SCN_RGB24, SCN_GRAY8 = 0, 1
SCN_OP_CONVERT, SCN_OP_HIST, SCN_OP_FLOW, SCN_OP_SURROGATE = 0, 1, 2, 3
SCN_OP_SURROGATE_GRADS, SCN_OP_SURROGATE_INFER, SCN_OP_HIST_DIFF = 4, 5, 6

_STATUS_NAMES = {SCN_EINVAL: "SCN_EINVAL", SCN_EUNSUPPORTED: "SCN_EUNSUPPORTED", SCN_ENOSPACE: "SCN_ENOSPACE",
                 SCN_EHIP: "SCN_EHIP"}


class ScnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class CTable(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("reserved", ctypes.c_int32), ("frame_bytes", ctypes.c_int64),
                ("n_frames", ctypes.c_int64), ("backed_first", ctypes.c_int64), ("backed_count", ctypes.c_int64)]


class CSampling(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("stencil", ctypes.c_int32), ("start", ctypes.c_int64),
                ("step", ctypes.c_int64), ("stop", ctypes.c_int64), ("idx", ctypes.POINTER(ctypes.c_int64)),
                ("n", ctypes.c_int64)]


class CJob(ctypes.Structure):
    _fields_ = [("table", ctypes.POINTER(CTable)), ("sampling", ctypes.POINTER(CSampling))]


class CFlowParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("alpha", ctypes.c_float), ("iters", ctypes.c_int32),
                ("sweeps_per_pass", ctypes.c_int32), ("tile_variant", ctypes.c_int32), ("warm_packet", ctypes.c_int32),
                ("warm_iters", ctypes.c_int32), ("solver", ctypes.c_int32), ("fb_poly_n", ctypes.c_int32),
                ("fb_sigma", ctypes.c_float), ("fb_win", ctypes.c_int32), ("fb_lambda", ctypes.c_float)]


# Every symbol declared in include/scn.h (checked by the CPU test suite).
EXPORTS = ["scn_count_rows", "scn_count_pairs", "scn_workspace_bytes", "scn_sample_convert", "scn_hist",
           "scn_hist_diff", "scn_space_map", "scn_flow", "scn_ws_forget", "scn_last_error", "scn_version", "scn_timing_enable",
           "scn_timing_reset", "scn_timing_read", "scn_timing_units", "scn_net_bytes", "scn_net_params", "scn_net_pack",
           "scn_adam_step", "scn_surrogate_grads", "scn_surrogate_infer", "scn_flow_surrogate", "scn_hist_static",
           "scn_surrogate_train_step"]

_lib = None


def lib() -> ctypes.CDLL:
    """Load libscn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libscn.so is not built (%s); run __graft_entry__.build() or "
                           "python -m paper_1805_07339_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.scn_count_rows.argtypes = [P(CJob)]
    L.scn_count_rows.restype = ctypes.c_int64
    L.scn_count_pairs.argtypes = [P(CJob)]
    L.scn_count_pairs.restype = ctypes.c_int64
    L.scn_workspace_bytes.argtypes = [ctypes.c_int32, P(CJob), ctypes.c_int32, P(CFlowParams)]
    L.scn_workspace_bytes.restype = ctypes.c_size_t
    L.scn_sample_convert.argtypes = [P(CJob), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                     ctypes.c_size_t, vp]
    L.scn_sample_convert.restype = ctypes.c_int
    L.scn_hist.argtypes = [P(CJob), vp, vp, ctypes.c_size_t, vp]
    L.scn_hist.restype = ctypes.c_int
    L.scn_hist_static.argtypes = [P(CJob), vp, vp]
    L.scn_hist_static.restype = ctypes.c_int
    L.scn_hist_diff.argtypes = [P(CJob), vp, ctypes.c_uint32, vp, vp, vp, ctypes.c_size_t, vp]
    L.scn_hist_diff.restype = ctypes.c_int
    L.scn_space_map.argtypes = [P(CJob), ctypes.c_int32, vp]
    L.scn_space_map.restype = ctypes.c_int
    L.scn_flow.argtypes = [P(CJob), ctypes.c_int32, P(CFlowParams), P(vp), vp, ctypes.c_size_t, vp]
    L.scn_flow.restype = ctypes.c_int
    L.scn_ws_forget.argtypes = [vp]
    L.scn_ws_forget.restype = None
    L.scn_last_error.argtypes = []
    L.scn_last_error.restype = ctypes.c_char_p
    L.scn_version.argtypes = []
    L.scn_version.restype = ctypes.c_char_p
    L.scn_timing_enable.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.scn_timing_enable.restype = ctypes.c_int
    L.scn_timing_reset.argtypes = []
    L.scn_timing_reset.restype = ctypes.c_int
    L.scn_timing_read.argtypes = [ctypes.c_char_p, P(ctypes.c_double), P(ctypes.c_int64)]
    L.scn_timing_read.restype = ctypes.c_int
    L.scn_timing_units.argtypes = [ctypes.c_char_p, P(ctypes.c_double)]
    L.scn_timing_units.restype = ctypes.c_int
    L.scn_net_bytes.argtypes = []
    L.scn_net_bytes.restype = ctypes.c_size_t
    L.scn_net_params.argtypes = []
    L.scn_net_params.restype = ctypes.c_int32
    L.scn_net_pack.argtypes = [vp, vp, vp]
    L.scn_net_pack.restype = ctypes.c_int
    L.scn_adam_step.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, vp, vp]
    L.scn_adam_step.restype = ctypes.c_int
    L.scn_surrogate_grads.argtypes = [P(CJob), ctypes.c_int32, vp, P(vp), vp, vp, vp, ctypes.c_size_t, vp]
    L.scn_surrogate_grads.restype = ctypes.c_int
    L.scn_surrogate_train_step.argtypes = [P(CJob), ctypes.c_int32, P(vp), vp, vp, vp, vp, vp, ctypes.c_int32,
                                           ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp, vp,
                                           ctypes.c_size_t, vp]
    L.scn_surrogate_train_step.restype = ctypes.c_int
    L.scn_surrogate_infer.argtypes = [P(CJob), ctypes.c_int32, vp, P(vp), vp, ctypes.c_size_t, vp]
    L.scn_surrogate_infer.restype = ctypes.c_int
    L.scn_flow_surrogate.argtypes = [P(CJob), ctypes.c_int32, P(CFlowParams), vp, ctypes.c_float, P(vp), P(vp), P(vp),
                                     vp, ctypes.c_size_t, vp]
    L.scn_flow_surrogate.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != SCN_OK:
        raise ScnError(status, lib().scn_last_error().decode())


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# tables, sampling specs, jobs


@dataclass
class Table:
    """A column of decoded NV12 frames: uint8 tensor [n_frames, frame_bytes] (or any
    tensor whose memory is laid out that way) with frame geometry."""
    frames: torch.Tensor
    width: int
    height: int
    pitch: int
    frame_bytes: int
    n_frames: int
    row0: int = 0  # table row held by frames[0] (window views)
    backed: int = 0  # rows row0 .. row0 + backed - 1 are backed (0: every row)

    @staticmethod
    def window(rows: torch.Tensor, first_row: int, n_frames: int, width: int, height: int,
               pitch: Optional[int] = None) -> "Table":
        """A table of n_frames rows of which only rows first_row .. first_row +
        len(rows) - 1 are backed by memory (rows[i] holds row first_row + i).
        Only the rows a job reads are touched, so a job may use such a view as
        long as those rows are backed (Sec. 4.2: frames that no output needs
        are never materialised); the library refuses jobs that read outside
        the window."""
        t = Table.from_tensor(rows, width, height, pitch)
        if first_row < 0 or first_row + t.n_frames > n_frames:
            raise ValueError("window rows fall outside the table")
        if t.n_frames == 0:
            raise ValueError("a window needs at least one backed row")
        t.row0, t.backed, t.n_frames = first_row, t.n_frames, n_frames
        return t

    @staticmethod
    def from_tensor(frames: torch.Tensor, width: int, height: int, pitch: Optional[int] = None) -> "Table":
        pitch = width if pitch is None else pitch
        if frames.dtype != torch.uint8:
            raise TypeError("table frames must be uint8")
        n = frames.shape[0]
        fb = frames.stride(0) * frames.element_size() if frames.dim() > 1 else frames.numel()
        return Table(frames, width, height, pitch, fb, n)

    def c(self) -> CTable:
        return CTable(self.frames.data_ptr() - self.row0 * self.frame_bytes, self.width, self.height, self.pitch, 0,
                      self.frame_bytes, self.n_frames, self.row0 if self.backed else 0, self.backed)


class Sampling:
    """Stride / gather / range sampling (host-side spec)."""

    def __init__(self, kind: int, start: int = 0, step: int = 1, stop: int = 0, idx: Sequence[int] = (),
                 stencil: int = SCN_STENCIL_AFTER):
        self.kind, self.start, self.step, self.stop = kind, start, step, stop
        self.stencil = stencil
        self.idx = [int(v) for v in idx]
        self._arr = (ctypes.c_int64 * max(len(self.idx), 1))(*self.idx)

    def before(self) -> "Sampling":
        """The same rows with the flow stencil applied before sampling: pairs
        (s, s+1) of original rows for each sampled row s.  A Job copies its
        sampling when it is built, so call this before building the Job."""
        self.stencil = SCN_STENCIL_BEFORE
        return self

    @staticmethod
    def stride(step: int, start: int = 0, stop: Optional[int] = None, n_frames: Optional[int] = None) -> "Sampling":
        if stop is None:
            stop = n_frames
        return Sampling(SCN_STRIDE, start, step, stop)

    @staticmethod
    def gather(rows: Sequence[int]) -> "Sampling":
        return Sampling(SCN_GATHER, idx=rows)

    @staticmethod
    def range(windows: Sequence[Tuple[int, int]]) -> "Sampling":
        flat = [v for w in windows for v in w]
        s = Sampling(SCN_RANGE, idx=flat)
        s.n_windows = len(windows)
        return s

    def c(self) -> CSampling:
        n = len(self.idx) // 2 if self.kind == SCN_RANGE else len(self.idx)
        return CSampling(self.kind, self.stencil, self.start, self.step, self.stop,
                         ctypes.cast(self._arr, ctypes.POINTER(ctypes.c_int64)), n)


class Job:
    def __init__(self, table: Table, sampling: Sampling):
        self.table, self.sampling = table, sampling
        self._ct = table.c()
        self._cs = sampling.c()
        self.cjob = CJob(ctypes.pointer(self._ct), ctypes.pointer(self._cs))


def _jobs_array(jobs: Sequence[Job]):
    arr = (CJob * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = j.cjob
    return arr


SCN_SOLVER_HS, SCN_SOLVER_FARNEBACK = 0, 1


def flow_params(levels: int = 4, alpha: float = 10.0, iters: int = 50, sweeps_per_pass: int = 0,
                tile_variant: int = 0, warm_packet: int = 0, warm_iters: int = 0) -> CFlowParams:
    """Horn-Schunck parameters; warm_packet >= 2 turns on the temporal warm
    start (packets of that many pairs, later pairs solved at full resolution
    from their predecessor's flow with warm_iters iterations)."""
    return CFlowParams(levels, alpha, iters, sweeps_per_pass, tile_variant, warm_packet, warm_iters,
                       SCN_SOLVER_HS, 0, 0.0, 0, 0.0)


def farneback_params(levels: int = 4, iters: int = 3, poly_n: int = 2, sigma: float = 1.1, win: int = 7,
                     lam: float = 1e-3) -> CFlowParams:
    """Farnebäck parameters for scn.flow: `iters` displacement estimates per
    level, (2 poly_n + 1)^2 expansion window with Gaussian applicability of
    standard deviation `sigma`, (2 win + 1)^2 averaging box, regulariser
    `lam`."""
    return CFlowParams(levels, 0.0, iters, 0, 0, 0, 0, SCN_SOLVER_FARNEBACK, poly_n, sigma, win, lam)


def count_rows(job: Job) -> int:
    n = lib().scn_count_rows(ctypes.byref(job.cjob))
    if n < 0:
        _check(int(n))
    return int(n)


def count_pairs(job: Job) -> int:
    n = lib().scn_count_pairs(ctypes.byref(job.cjob))
    if n < 0:
        _check(int(n))
    return int(n)


def workspace_bytes(op: int, jobs: Sequence[Job], params: Optional[CFlowParams] = None) -> int:
    arr = _jobs_array(jobs)
    n = lib().scn_workspace_bytes(op, arr, len(jobs), ctypes.byref(params) if params is not None else None)
    if n == 0:
        raise ScnError(SCN_EINVAL, lib().scn_last_error().decode())
    return int(n)


# ---------------------------------------------------------------------------
# workspace pool (caller-owned scratch; the library never allocates)


class Workspace:
    """A growable device scratch buffer, one per (device, name)."""

    def __init__(self, device=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.buf: Optional[torch.Tensor] = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            if self.buf is not None:
                lib().scn_ws_forget(self.buf.data_ptr())
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


_pools = {}


def _ws(device, nbytes: int, name: str = "default") -> torch.Tensor:
    key = (str(device), name)
    if key not in _pools:
        _pools[key] = Workspace(device)
    return _pools[key].get(nbytes)


# ---------------------------------------------------------------------------
# operations


def hist(job: Job, out: Optional[torch.Tensor] = None, stream=None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Per-sampled-row 16-bin R, G, B histograms -> int32 tensor [M, 3, 16] (uint32 counts)."""
    m = count_rows(job)
    dev = job.table.frames.device
    if out is None:
        out = torch.empty((m, 3, 16), dtype=torch.int32, device=dev)
    if m == 0:
        return out
    need = workspace_bytes(SCN_OP_HIST, [job])
    w = ws if ws is not None else _ws(dev, need)
    _check(lib().scn_hist(ctypes.byref(job.cjob), out.data_ptr(), w.data_ptr(), w.numel(), _stream(stream)))
    return out


HIST_STATIC_MAX_ROWS = 65536  # SCN_HIST_STATIC_MAX_ROWS


def hist_static(job: Job, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """hist() without a workspace: the row table goes to the library's fixed
    per-GPU array (for callers that cannot allocate; at most
    HIST_STATIC_MAX_ROWS sampled rows; calls on one GPU must not overlap).
    The output tensor is the caller's: pass `out` to allocate nothing."""
    m = count_rows(job)
    if out is None:
        out = torch.empty((m, 3, 16), dtype=torch.int32, device=job.table.frames.device)
    _check(lib().scn_hist_static(ctypes.byref(job.cjob), _ptr(out), _stream(stream)))
    return out


def space_map(job: Job, mode: int = SCN_SPACE_NULL) -> List[int]:
    """Spacing: index of the job's FLOW output placed at each table row
    (NULL: only at the first row of its pair; REPEAT: the last output at or
    before the row), -1 elsewhere (host only)."""
    n = job.table.n_frames
    buf = (ctypes.c_int64 * max(n, 1))()
    _check(lib().scn_space_map(ctypes.byref(job.cjob), mode, ctypes.cast(buf, ctypes.c_void_p)))
    return list(buf[:n])


def hist_diff(job: Job, hist: torch.Tensor, threshold: int, with_cut: bool = True, stream=None,
              ws: Optional[torch.Tensor] = None):
    """Shot-boundary cue over the job's S[0,1] pairs from its HIST output
    `hist` ([M, 3, 16] int32 holding uint32 counts, on the GPU): returns
    (diff, cut) with diff int64 [P] (the L1 histogram distances) and cut
    uint8 [P] (diff > threshold), or cut None when with_cut is False."""
    p = count_pairs(job)
    dev = hist.device
    if not (0 <= int(threshold) <= 0xFFFFFFFF):
        raise ValueError("threshold must fit uint32")
    if hist.dtype != torch.int32 or not hist.is_contiguous() or hist.shape != (count_rows(job), 3, 16):
        raise ValueError("hist must be a contiguous int32 [M, 3, 16] tensor")
    raw = torch.empty((p,), dtype=torch.int32, device=dev)
    cut = torch.empty((p,), dtype=torch.uint8, device=dev) if with_cut else None
    if p > 0:
        need = workspace_bytes(SCN_OP_HIST_DIFF, [job])
        w = ws if ws is not None else _ws(dev, need)
        _check(lib().scn_hist_diff(ctypes.byref(job.cjob), hist.data_ptr(), int(threshold), raw.data_ptr(),
                                   cut.data_ptr() if cut is not None else None, w.data_ptr(), w.numel(),
                                   _stream(stream)))
    return raw.to(torch.int64) & 0xFFFFFFFF, cut


def sample_convert(job: Job, out_w: Optional[int] = None, out_h: Optional[int] = None, fmt: int = SCN_RGB24,
                   out: Optional[torch.Tensor] = None, stream=None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Gather + BT.601 convert (+ resize) -> uint8 [M, out_h, out_w, 3] (RGB24) or [M, out_h, out_w] (GRAY8)."""
    t = job.table
    out_w = t.width if out_w is None else out_w
    out_h = t.height if out_h is None else out_h
    m = count_rows(job)
    if out is None:
        shape = (m, out_h, out_w, 3) if fmt == SCN_RGB24 else (m, out_h, out_w)
        out = torch.empty(shape, dtype=torch.uint8, device=t.frames.device)
    if m == 0:
        return out
    need = workspace_bytes(SCN_OP_CONVERT, [job])
    w = ws if ws is not None else _ws(t.frames.device, need)
    _check(lib().scn_sample_convert(ctypes.byref(job.cjob), out_w, out_h, fmt, out.data_ptr(), w.data_ptr(),
                                    w.numel(), _stream(stream)))
    return out


def flow(jobs: Sequence[Job], params: Optional[CFlowParams] = None, outs: Optional[List[torch.Tensor]] = None,
         stream=None, ws: Optional[torch.Tensor] = None, ws_bytes: Optional[int] = None) -> List[torch.Tensor]:
    """Pyramidal Horn-Schunck (or, with farneback_params, Farnebäck) flow for
    every job -> list of float32 [P_j, 2, H_j, W_j]."""
    params = flow_params() if params is None else params
    if outs is None:
        outs = []
        for j in jobs:
            p = count_pairs(j)
            outs.append(torch.empty((p, 2, j.table.height, j.table.width), dtype=torch.float32,
                                    device=j.table.frames.device))
    arr = _jobs_array(jobs)
    ptrs = (ctypes.c_void_p * len(jobs))(*[o.data_ptr() if o.numel() else None for o in outs])
    if sum(o.shape[0] for o in outs) == 0:
        return outs
    if ws is None:
        need = workspace_bytes(SCN_OP_FLOW, jobs, params) if ws_bytes is None else ws_bytes
        ws = _ws(jobs[0].table.frames.device, need)
    nbytes = ws.numel() if ws_bytes is None else min(ws_bytes, ws.numel())
    _check(lib().scn_flow(arr, len(jobs), ctypes.byref(params), ptrs, ws.data_ptr(), nbytes, _stream(stream)))
    return outs


# ---------------------------------------------------------------------------
# learned surrogate


def net_params() -> int:
    return int(lib().scn_net_params())


def net_bytes() -> int:
    return int(lib().scn_net_bytes())


def net_pack(master: torch.Tensor, net: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """FP32 master parameters (device, [net_params()]) -> network blob (uint8 device tensor)."""
    if net is None:
        net = torch.empty(net_bytes(), dtype=torch.uint8, device=master.device)
    _check(lib().scn_net_pack(master.data_ptr(), net.data_ptr(), _stream(stream)))
    return net


def adam_step(master, m, v, grads, step: int, lr: float, net, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().scn_adam_step(master.data_ptr(), m.data_ptr(), v.data_ptr(), grads.data_ptr(), step, lr, beta1, beta2,
                               eps, net.data_ptr(), _stream(stream)))


def _ptr_array(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() if (t is not None and t.numel()) else None for t in ts])


def surrogate_grads(jobs: Sequence[Job], net: torch.Tensor, targets: List[torch.Tensor],
                    grads: Optional[torch.Tensor] = None, loss: Optional[torch.Tensor] = None, stream=None,
                    ws: Optional[torch.Tensor] = None):
    dev = net.device
    if grads is None:
        grads = torch.empty(net_params(), dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    if ws is None:
        ws = _ws(dev, workspace_bytes(SCN_OP_SURROGATE_GRADS, jobs), "surrogate")
    _check(lib().scn_surrogate_grads(_jobs_array(jobs), len(jobs), net.data_ptr(), _ptr_array(targets),
                                     grads.data_ptr(), loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return grads, loss


def surrogate_train_step(jobs: Sequence[Job], targets: List[torch.Tensor], master, m, v, net, step: int, lr: float,
                         beta1=0.9, beta2=0.999, eps=1e-8, grads: Optional[torch.Tensor] = None,
                         loss: Optional[torch.Tensor] = None, stream=None, ws: Optional[torch.Tensor] = None):
    """Gradients of the batch and the Adam step in one call; returns (grads, loss)."""
    dev = net.device
    if grads is None:
        grads = torch.empty(net_params(), dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    if ws is None:
        ws = _ws(dev, workspace_bytes(SCN_OP_SURROGATE_GRADS, jobs), "surrogate")
    _check(lib().scn_surrogate_train_step(_jobs_array(jobs), len(jobs), _ptr_array(targets), master.data_ptr(),
                                          m.data_ptr(), v.data_ptr(), grads.data_ptr(), net.data_ptr(), step, lr,
                                          beta1, beta2, eps, loss.data_ptr(), ws.data_ptr(), ws.numel(),
                                          _stream(stream)))
    return grads, loss


def surrogate_infer(jobs: Sequence[Job], net: torch.Tensor, outs: Optional[List[torch.Tensor]] = None, stream=None,
                    ws: Optional[torch.Tensor] = None) -> List[torch.Tensor]:
    if outs is None:
        outs = [torch.empty((count_pairs(j), 2, j.table.height, j.table.width), dtype=torch.float32,
                            device=net.device) for j in jobs]
    if ws is None:
        ws = _ws(net.device, workspace_bytes(SCN_OP_SURROGATE_INFER, jobs), "surrogate")
    _check(lib().scn_surrogate_infer(_jobs_array(jobs), len(jobs), net.data_ptr(), _ptr_array(outs), ws.data_ptr(),
                                     ws.numel(), _stream(stream)))
    return outs


def flow_surrogate(jobs: Sequence[Job], net: torch.Tensor, tau: float, params: Optional[CFlowParams] = None,
                   outs=None, fell_back=None, residual=None, stream=None, ws: Optional[torch.Tensor] = None,
                   ws_bytes: Optional[int] = None):
    """Surrogate flow with the residual gate and the plain-solver fallback.
    Returns (flows, fell_back flags, residuals), one entry per job."""
    params = flow_params() if params is None else params
    dev = net.device
    if outs is None:
        outs = [torch.empty((count_pairs(j), 2, j.table.height, j.table.width), dtype=torch.float32, device=dev)
                for j in jobs]
    if fell_back is None:
        fell_back = [torch.empty(count_pairs(j), dtype=torch.uint8, device=dev) for j in jobs]
    if residual is None:
        residual = [torch.empty(count_pairs(j), dtype=torch.float32, device=dev) for j in jobs]
    if ws is None:
        need = workspace_bytes(SCN_OP_SURROGATE, jobs, params) if ws_bytes is None else ws_bytes
        ws = _ws(dev, need, "surrogate")
    nbytes = ws.numel() if ws_bytes is None else min(ws_bytes, ws.numel())
    _check(lib().scn_flow_surrogate(_jobs_array(jobs), len(jobs), ctypes.byref(params), net.data_ptr(), tau,
                                    _ptr_array(outs), _ptr_array(fell_back), _ptr_array(residual), ws.data_ptr(),
                                    nbytes, _stream(stream)))
    return outs, fell_back, residual


def timing_enable(on: bool = True, max_launches: int = 65536):
    _check(lib().scn_timing_enable(1 if on else 0, max_launches))


def timing_reset():
    _check(lib().scn_timing_reset())


def timing_read(kernel: str) -> Tuple[float, int]:
    """(total milliseconds, launches) recorded for one kernel class."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().scn_timing_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def timing_units(kernel: str) -> float:
    """Summed work units recorded for one kernel class (Jacobi: pixels x pairs per pass)."""
    u = ctypes.c_double()
    _check(lib().scn_timing_units(kernel.encode(), ctypes.byref(u)))
    return u.value


def version() -> str:
    return lib().scn_version().decode()
