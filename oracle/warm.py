"""Temporal warm start of the flow, a bounded-state operation (oracle; test
infrastructure only).

Sec. 3.2 lets an operation carry state from one output element to the next
as long as the dependence is bounded by a warmup W; the runtime then cuts a
sequence into work packets and replays W elements at each packet start
(Sec. 4.1).  For FLOW the natural state is the previous pair's result: a
pair's solve can start from its predecessor's flow instead of from the
coarse levels (W = 1), which cuts work when motion is coherent in time.
The paper gives no algorithm for it; the readings below fix one.

Readings:
* Work packets hold G consecutive pairs of one slice, counted from the
  slice's first pair.  The first pair of a packet is solved cold: the full
  pyramidal method of hs.py (levels, alpha, iters).  No packet crosses a
  slice boundary, so results depend on G but not on how pairs are batched.
* Each later pair of the packet is solved at full resolution only, from its
  predecessor's final flow (u_p, v_p): I2 warped by it, the constraint
  linearised about it (steps 5-7 of hs.py with start flow (u_p, v_p)), then
  `warm_iters` Jacobi iterations (steps 8-9).

Pins (tests): from a zero start the warm solve is the one-level method of
hs.py; G = 1 is the cold method for every pair; packets restart at slice
boundaries; on a constant-velocity translation the warm chain recovers the
motion with far fewer iterations than a cold one-level solve, and as well as
the cold pyramid.  Parity pinned.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import hs


def level0_from(Y1: np.ndarray, Y2: np.ndarray, u0: np.ndarray, v0: np.ndarray, alpha: float,
                iters: int) -> Tuple[np.ndarray, np.ndarray]:
    """Full-resolution solve of (Y1, Y2) started from the flow (u0, v0)."""
    I1, I2 = hs.luma_float(Y1), hs.luma_float(Y2)
    Ix, Iy, Itp = hs.level_setup(I1, I2, u0, v0)
    return hs.jacobi(u0, v0, Ix, Iy, Itp, alpha, iters)


def warm_chain(slices: Sequence[Sequence[Tuple[np.ndarray, np.ndarray]]], packet: int, levels: int, alpha: float,
               iters: int, warm_iters: int) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Flows of every pair, in order; `slices` lists the (Y1, Y2) pairs of each slice."""
    if packet < 1:
        raise ValueError("packet must be >= 1")
    out = []
    for pairs in slices:
        u = v = None
        for k, (Y1, Y2) in enumerate(pairs):
            if k % packet == 0:
                u, v = hs.hs_flow(Y1, Y2, levels=levels, alpha=alpha, iters=iters)
            else:
                u, v = level0_from(Y1, Y2, u, v, alpha, warm_iters)
            out.append((u, v))
    return out
