"""Host-side pieces of bench.py (no GPU): the one-GPU guard and the
per-launch work figures its roofline divides by."""
import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_launch_work_per_unit_figures():
    N, m, T = 65536, 1024, 50
    fl, by = bench.launch_work("forward_layer", N, m, T)
    assert fl == 2.0 * N * m * m * T                 # T contractions of 2 m^2 flops per sample
    assert by == 4.0 * m * N * (T + 3)               # c once, T kept iterates, z^T, the seed
    fl, by = bench.launch_work("backward_layer", N, m, T)
    assert fl == 2.0 * N * m * m * (T - 1)
    assert by == 4.0 * m * N * (T + 1)               # the seed, z^T, z^t for 1 <= t < T
    # both launches sit above the BF16 ridge (2.5 PFLOP/s over 8 TB/s) at m = 1024
    for kind in ("forward_layer", "backward_layer"):
        fl, by = bench.launch_work(kind, N, m, T)
        assert fl / by > 2.5e15 / 8e12
