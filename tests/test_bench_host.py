"""Host logic of bench.py that runs without a GPU: the autotuning choice
over several passes, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pick_tuning_keeps_each_candidates_best_pass():
    a = np.full((3, 3), 9.0)
    b = np.full((3, 3), 9.0)
    a[1, 1] = 7.5  # 2 groups, 512 lanes: fast in one pass only
    b[1, 1] = 8.5
    a[2, 1] = 7.8  # 4 groups, 512 lanes: steady
    b[2, 1] = 7.7
    threads, groups, best = bench.pick_tuning([a, b])
    assert (threads, groups) == (512, 2)
    assert best[1, 1] == 7.5 and best[2, 1] == 7.7


def test_pick_tuning_skips_candidates_never_run():
    a = np.full((3, 3), 5.0)
    a[2, :] = -1.0  # more groups than filters: not run
    a[0, 2] = 1.0
    threads, groups, best = bench.pick_tuning([a, a.copy()])
    assert (threads, groups) == (1024, 1)
    assert (best[2] == -1.0).all()
    with pytest.raises(ValueError):
        bench.pick_tuning([np.full((3, 3), -1.0)])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
