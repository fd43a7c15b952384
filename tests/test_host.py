"""Host-side contracts of the benchmark and the input generators (no GPU)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1509_08197_amd import scenes  # noqa: E402


def test_bench_refuses_several_gpus():
    # one GPU only: asked for more, the bench says so and exits before any GPU call
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2, r.stderr[-2000:]
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_forked_and_serial_draws_agree():
    # the batched pairs drawn by the forked host pool are the serially drawn ones
    # (the pool is used only before the first GPU call; both must give the same input)
    forked = scenes._draw_batch(5, 3, processes=3)
    serial = scenes._draw_batch(5, 3, processes=1)
    assert len(forked) == len(serial) == 3
    for a, b in zip(forked, serial):
        assert a.shape == b.shape and a.dmax == b.dmax
        assert np.array_equal(a.left, b.left) and np.array_equal(a.right, b.right)


def test_no_fork_after_gpu_flag():
    # without torch initialised on a device the pool may fork
    assert scenes._gpu_initialised() is False
