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


def test_model_flop_counts():
    """30 d K + 4 |O| FLOP per particle-step for Lorenz '96: 1,952 at d = 8
    (all 8 observed, K = 8) and 9,680 at d = 40 (20 observed)."""
    import workloads as W
    assert bench.model_flop_per_particle_step(W.MODEL_L96, 8, 8, 8) == 1952
    assert bench.model_flop_per_particle_step(W.MODEL_L96, 40, 8, 20) == 9680


def test_tf_summary_counts_pairs_over_the_bound():
    err = np.array([[1e-6, 2e-4], [5e-5, 3e-4]])
    ell = np.array([[-10.0, -250.0], [-12.0, -300.0]])
    ess = np.array([[900.0, 1.2], [800.0, 1.0]])
    s = bench.tf_summary(err, ell, ess, 1e-4)
    assert s["pairs"] == 4 and s["pairs_over_bound"] == 2
    assert s["frac_within_bound"] == 0.5
    assert s["max_abs_where_ess_ge_2"] == 5e-5 and s["pairs_over_bound_where_ess_ge_2"] == 0
    assert s["worst"][0]["err"] == 3e-4 and s["worst"][0]["ess"] == 1.0


def test_oracle_worker_is_pinned(tmp_path):
    """The CPU baseline's oracle process runs on the one core it is given."""
    import oracle
    import workloads as W
    pb = W.config("lorenz96_d8_batched")
    _, y = oracle.simulate(pb)
    path = str(tmp_path / "obs.npy")
    np.save(path, y, allow_pickle=False)
    core = sorted(os.sched_getaffinity(0))[-1]
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-worker", "0",
                        "512", "0.01", path, str(core)],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    import json
    d = json.loads(r.stdout.strip().splitlines()[-1])
    assert d["affinity"] == [core] and d["filters"] == 1 and d["ps"] > 0
