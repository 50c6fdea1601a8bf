"""Pins of the warm-start oracle: the zero-start special case, G = 1, slice
restarts, and the iteration saving on a constant-velocity translation."""
import numpy as np

import synth
from oracle import hs as OH
from oracle import warm as OW


def _frames(n, d, w=96, h=64, seed=5, noise=0.0):
    rng = synth.SplitMix64(seed)
    tex = synth.Texture.random(rng)
    tu = synth.Texture.random(rng, sigma=20.0)
    tv = synth.Texture.random(rng, sigma=20.0)
    lay = synth.Layer(tex, tu, tv, "full", shifts=[(t * d[0], t * d[1]) for t in range(n)])
    sc = synth.Scene(w, h, [lay], seed, noise)
    return [sc.nv12(t).numpy()[:h, :w] for t in range(n)]


def test_zero_start_is_the_one_level_method():
    f = _frames(2, (0.7, -0.4))
    z = np.zeros(f[0].shape)
    u, v = OW.level0_from(f[0], f[1], z, z, 10.0, 30)
    u1, v1 = OH.hs_flow(f[0], f[1], levels=1, alpha=10.0, iters=30)
    assert np.array_equal(u, u1) and np.array_equal(v, v1)


def test_packet_of_one_is_cold_and_slices_restart():
    f = _frames(5, (0.5, 0.3))
    pairs = list(zip(f[:-1], f[1:]))
    cold = [OH.hs_flow(a, b, levels=2, alpha=10.0, iters=20) for a, b in pairs]
    got = OW.warm_chain([pairs], 1, 2, 10.0, 20, 5)
    for (u, v), (uc, vc) in zip(got, cold):
        assert np.array_equal(u, uc) and np.array_equal(v, vc)
    # two slices, G = 3: pairs 0 and 3 of slice 1 and pair 0 of slice 2 are cold
    got = OW.warm_chain([pairs, pairs[:2]], 3, 2, 10.0, 20, 5)
    for idx, ref in ((0, 0), (3, 3), (4, 0)):
        assert np.array_equal(got[idx][0], cold[ref][0])
    for idx in (1, 2, 5):
        assert not np.array_equal(got[idx][0], cold[idx if idx < 4 else 1][0])


def test_warm_start_cuts_iterations_on_constant_motion():
    d = (0.8, -0.45)
    f = _frames(5, d, noise=0.0)
    pairs = list(zip(f[:-1], f[1:]))
    m = 16  # interior margin

    def err(u, v):
        return float(np.hypot(u[m:-m, m:-m] - d[0], v[m:-m, m:-m] - d[1]).mean())

    warm = OW.warm_chain([pairs], 4, 3, 10.0, 50, 10)
    cold1 = [OH.hs_flow(a, b, levels=1, alpha=10.0, iters=10) for a, b in pairs]
    cold3 = [OH.hs_flow(a, b, levels=3, alpha=10.0, iters=50) for a, b in pairs]
    for k in (1, 2, 3):
        ew, e1, e3 = err(*warm[k]), err(*cold1[k]), err(*cold3[k])
        assert ew < 0.5 * e1
        assert ew < e3 + 0.02
