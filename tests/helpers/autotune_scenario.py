"""Run as a child process by test_autotune_keeps_results: a batched handle
steps T intervals, is autotuned (which must leave it re-initialised), steps
again; the two likelihood-increment traces must agree.  Prints "ok" and the
choice, or raises."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import dataclasses  # noqa: E402

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402
import paper_1306_3277_amd as pfm  # noqa: E402


def main():
    torch.cuda.set_device(0)
    pfm.load()
    th, n = W.batched_thetas(40, seed=9)
    base = W.lorenz96(d=8, N=1, T=6)
    _, y = oracle.simulate(base)
    pb = dataclasses.replace(base.with_obs(y), theta=np.asarray(th, dtype=np.float64),
                             n_particles=np.asarray(n, dtype=np.int64))
    f = pfm.Filter(pb, layout=pfm.PF_LAYOUT_BATCHED)
    f.advance(pb.T)
    e0, _ = f.trace()
    threads, groups, ms = f.autotune(steps=3)
    assert threads in (256, 512, 1024) and groups in (1, 2, 4), (threads, groups)
    assert np.all(ms[ms >= 0] > 0)
    f.advance(pb.T)  # autotune leaves the filters re-initialised
    e1, _ = f.trace()
    np.testing.assert_allclose(e1, e0, rtol=1e-12, atol=1e-12)
    f.close()
    print(f"ok {threads} {groups}", flush=True)


if __name__ == "__main__":
    main()
