"""The FP32 error budget of Horn-Schunck on the 2048 x 2048 rig pair (CPU):
with the kernels' precision choices (exact pyramid, setup in FP64 above level
0, FP32 elsewhere) the oracle's steps stay within 2.5e-4 px of the FP64 flow
on every pixel, while an FP32 pyramid alone moves pixels by more than the
1e-3 px contract."""
import numpy as np

from oracle import hs as OH
from tests import fp_budget as B


def test_kernel_precision_choices_meet_the_flow_bound_on_the_rig():
    Y1, Y2 = B.rig_pair()
    ref = OH.hs_flow(Y1, Y2, levels=5, alpha=10.0, iters=50)
    mx, n, _ = B.deviation(ref, B.flow(Y1, Y2, B.KERNELS))
    print("kernels' precision: max |d| = %.3g px" % mx)
    assert mx <= 2.5e-4 and n == 0
    mx_pyr, n_pyr, _ = B.deviation(ref, B.flow(Y1, Y2, {"pyramid"}))
    print("FP32 pyramid: max |d| = %.3g px on %d pixels over 1e-3" % (mx_pyr, n_pyr))
    assert mx_pyr > 1e-3 and n_pyr > 0


def test_fp64_policy_is_the_oracle():
    """The budget's all-FP64 evaluation is the oracle itself (small pair)."""
    import synth
    s, _ = synth.translation_scene(3, 96, 64, 2)
    a, b = (s.nv12(t).numpy()[:64] for t in range(2))
    ref = OH.hs_flow(a, b, levels=3, alpha=10.0, iters=20)
    got = B.flow(a, b, set(), levels=3, iters=20)
    assert max(np.abs(got[0] - ref[0]).max(), np.abs(got[1] - ref[1]).max()) < 1e-12
