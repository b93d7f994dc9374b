"""bench.py's command line on the CPU: the one-GPU contract (more GPUs exit
with a message before touching a device) and the operation counts behind
the LDS solvers' roofline (linear in the iteration counts, the reaction term
heavier than the diffusion stencil alone)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_lds_flop_counts_are_linear_in_iterations():
    for n in (8, 16, 32, 64, 128):
        for reaction in (False, True):
            f0 = bench.lds_update_flops(n, 9, 0, reaction)
            f1 = bench.lds_update_flops(n, 9, 1, reaction)
            assert bench.lds_update_flops(n, 9, 7, reaction) == f0 + 7 * (f1 - f0)
            assert f1 > f0 > 0
            r0 = bench.rqi_sample_flops(n, 9, 0, 0, reaction)
            assert bench.rqi_sample_flops(n, 9, 3, 5, reaction) > r0 > 0
        assert bench.lds_update_flops(n, 9, 1, True) > bench.lds_update_flops(n, 9, 1, False)
