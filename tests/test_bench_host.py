"""Host logic of bench.py (no GPU): the multi-GPU refusal, the Jacobi
roofline arithmetic and the thresholds of the forced-fallback leg."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_jacobi_roofline_from_work_units():
    import bench
    # 10 launches over 1000 ms in total, 1e9 pixel-passes, 5e9 pixel-sweeps
    r = bench._jacobi_roofline(1000.0, 10, 1e9, 5e9, traffic=3.0e9)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["algorithmic_bytes_per_launch"] - 28e9 / 10) < 1
    assert abs(r["achieved"] - 28.0) < 1e-9          # 28e9 B in 1 s
    assert abs(r["frac"] - 28.0 / bench.HBM_PEAK_GBS) < 1e-12
    assert abs(r["alu"]["achieved_TFLOPs"] - 27 * 5e9 / 1e12) < 1e-9
    assert r["traffic"] == 3.0e9 and r["avg_launch_ms"] == 100.0


def test_fallback_thresholds_select_the_quantiles():
    import bench
    import random
    rng = random.Random(3)
    for n in (1, 7, 122):
        r = sorted(rng.uniform(0.5, 4.0) for _ in range(n))
        for frac in (0.25, 0.5, 1.0):
            t = bench.fallback_threshold(r, frac)
            failing = sum(x > t for x in r)  # the gate's rule: residual above the threshold
            assert failing == int(round(frac * n)), (n, frac, t)
            assert t >= 0.0
