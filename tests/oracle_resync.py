"""Resynchronising a GPU handle on the oracle after an in-band ancestor flip.

Where a cumulative weight lies within 1e-9 (normalised) of a stratum
boundary, the GPU and the oracle may legitimately pick different ancestors
(the two sums are rounded in different orders).  From then on that filter's
particles differ, so a parity test puts the oracle's equally weighted
particles of that time into the handle (pf_set_state) and carries on: the
later likelihood increments, log-weights and particles are then again
deterministic functions of the same state and generator counters, and are
compared as before.  Not a test module (no test_ prefix)."""
import numpy as np

import oracle


def oracle_state_after(pb, b, t, scheme=0, steps=0, ess_frac=float("inf")):
    """The oracle's particles of filter b after t intervals (resampled at t)."""
    r = oracle.pf_run_ex(pb, theta=pb.theta[b], N=int(pb.n_particles[b]), b=b, T=t,
                         resampler=scheme, steps=steps, ess_frac=ess_frac)
    return r["x"]


def resync(f, pb, flipped, t, scheme=0, steps=0, ess_frac=float("inf")):
    """Replace the particles of the filters in `flipped` by the oracle's after
    interval t; the other filters keep the handle's own particles."""
    x = f.get_state()
    off = np.concatenate([[0], np.cumsum(pb.n_particles)])
    for b in sorted(set(flipped)):
        x[:, off[b]:off[b + 1]] = oracle_state_after(pb, b, t, scheme, steps, ess_frac)
    f.set_state(x)
