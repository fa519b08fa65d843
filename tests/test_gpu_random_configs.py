"""GPU parity with the oracle over fixed-seed sweeps of batched and plain
configurations that the hand-picked tests do not combine: the three models
(Lorenz '96 at d = 4/8/16/32/40, the paper's stage-noise form, the windkessel),
particle counts at the edges of the 64-lane waves, 256-particle chunks and
the 8192-particle collective (batched) or of the propagation, scan and
merge-path blocks (plain: 255..257, 1023..1025, 2047..2049), every
resampler with and without the ESS trigger, every collective workgroup size
and 1-4 filter groups (batched).  FP64 throughout: log-weights bit for bit at every
time, ancestors bit for bit or (for FP64 comparisons of sums taken in
another order) a flip within 1e-9 of a stratum edge, likelihood increments
within 1e-10 relative, ESS within 1e-9, final particles bit for bit; then a
graph-replayed run of the same configuration gives the same bits as the
eager one."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle_resync import resync
import workloads as W

pytestmark = pytest.mark.gpu

REL64 = 1e-10
BAND = 1e-9
EDGE_COUNTS = [1, 2, 63, 64, 65, 255, 256, 257, 1000, 4095, 8192]
# the plain layout's 256-particle propagation blocks, 1024-particle scan
# blocks and 2048-diagonal merge-path blocks
PLAIN_EDGE_COUNTS = [1, 2, 255, 256, 257, 1023, 1024, 1025, 2047, 2048, 2049, 4097, 20000]


@pytest.fixture(scope="module")
def pfm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_3277_amd as pfm
    pfm.load()
    return pfm


def _config(i, plain=False):
    """Configuration i of the sweep (numpy's generator, seed 2026 + i, or
    3026 + i for the plain layout)."""
    rng = np.random.default_rng((3026 if plain else 2026) + i)
    kind = ["l96", "l96", "stage", "wk"][i % 4]
    B = int(rng.integers(1, 4 if plain else 8))
    T = int(rng.integers(2, 6))
    d = [4, 16, 40, 8, 32][(i // 2) % 5] if kind == "l96" else 8
    edges = PLAIN_EDGE_COUNTS if plain else EDGE_COUNTS
    counts = [c for c in edges if d < 16 or c <= 2049]
    n = rng.choice(counts, size=B).astype(np.int64)
    if kind == "wk":
        base = W.windkessel(N=1, T=T)
        th = np.stack([W.wk_theta(1.0, 1.5, 0.03, float(rng.uniform(0.3, 0.8)),
                                  float(rng.uniform(80, 100)), float(rng.uniform(5, 20)), 0.01)
                       for _ in range(B)])
    else:
        base = W.lorenz96(d=d, N=1, T=T, stage_noise=(kind == "stage"))
        th, _ = W.batched_thetas(B, seed=100 + i)
    _, y = oracle.simulate(base)
    pb = dataclasses.replace(base.with_obs(y), theta=th, n_particles=n)
    scheme = int(rng.integers(0, 4))
    steps = int(rng.integers(1, 10)) if scheme == oracle.RESAMPLE_METROPOLIS else 0
    ess_frac = float(rng.choice([np.inf, 0.5, 0.9]))
    nt = int(rng.choice([256, 512, 1024]))
    groups = int(rng.integers(1, 5))
    return pb, scheme, steps, ess_frac, nt, groups


def _edge_flip(lw, k, ref_u, band=BAND):
    w = np.exp(lw - lw.max())
    cw = np.cumsum(w) / w.sum()
    return np.min(np.abs(cw - ref_u)) < band


def _ancestors_agree(pb, scheme, lw, ag, ar, t, b):
    """True if equal; False if every difference is a legitimate flip at an
    edge (the caller then resynchronises this filter on the oracle); fails
    otherwise."""
    mism = np.flatnonzero(ag != ar)
    if mism.size == 0:
        return True
    assert scheme != oracle.RESAMPLE_METROPOLIS, (t, b, mism[:8])
    N = lw.size
    for k in mism:
        if scheme == oracle.RESAMPLE_MULTINOMIAL:
            ref_u = oracle.multi_u(pb.seed, t, b, 0, int(k))
        elif scheme == oracle.RESAMPLE_STRATIFIED:
            ref_u = (oracle.strat_u(pb.seed, t, b, 0, int(k)) + k) / N
        else:
            ref_u = (oracle.resample_u(pb.seed, t, b) + k) / N
        assert _edge_flip(lw, int(k), ref_u), (t, b, int(k))
    return False


def _run_config(pfm, i, layout):
    pb, scheme, steps, ess_frac, nt, groups = _config(i, plain=layout == pfm.PF_LAYOUT_PLAIN)
    n = pb.n_particles
    off = np.concatenate([[0], np.cumsum(n)])
    refs = [oracle.pf_run_ex(pb, theta=pb.theta[b], N=int(n[b]), b=b, resampler=scheme,
                             steps=steps, ess_frac=ess_frac, traces=True) for b in range(pb.B)]
    f = pfm.Filter(pb, precision=pfm.PF_FP64, layout=layout)
    f.set_tuning(nt, groups)
    f.set_resampler(scheme, steps, ess_frac)
    flips = 0
    for t in range(1, pb.T + 1):
        f.step()
        lw = f.logweights()
        for b in range(pb.B):
            np.testing.assert_array_equal(lw[off[b]:off[b + 1]], refs[b]["lw"][t - 1],
                                          err_msg=f"config {i}, filter {b}, t = {t}")
        f.resample()
        a = f.ancestors()
        flipped = [b for b in range(pb.B)
                   if not _ancestors_agree(pb, scheme, refs[b]["lw"][t - 1],
                                           a[off[b]:off[b + 1]], refs[b]["anc"][t - 1], t, b)]
        if flipped:
            flips += len(flipped)
            resync(f, pb, flipped, t, scheme, steps, ess_frac)
    ell, ess = f.trace()
    x = f.get_state()
    for b in range(pb.B):
        r = refs[b]
        np.testing.assert_array_less(np.abs(ell[b] - r["ell"]),
                                     REL64 * np.maximum(1.0, np.abs(r["ell"])))
        np.testing.assert_allclose(ess[b], r["ess"], rtol=1e-9)
        np.testing.assert_array_equal(x[:, off[b]:off[b + 1]], r["x"])
    f.close()
    if flips:
        print(f"config {i}: {flips} in-band ancestor flips, resynchronised on the oracle")
    # graph replay against eager launches of the same handle type (no resync)
    e = pfm.Filter(pb, precision=pfm.PF_FP64, layout=layout)
    e.set_tuning(nt, groups)
    e.set_resampler(scheme, steps, ess_frac)
    e.advance(pb.T)
    eager = (e.trace()[0], e.get_state(), e.ancestors())
    e.close()
    g = pfm.Filter(pb, precision=pfm.PF_FP64, layout=layout)
    g.set_tuning(nt, groups)
    g.set_resampler(scheme, steps, ess_frac)
    g.graph_run(pb.T)
    for got, want in zip((g.trace()[0], g.get_state(), g.ancestors()), eager):
        np.testing.assert_array_equal(got, want)
    g.close()
    return flips


@pytest.mark.parametrize("i", range(20))
def test_random_batched_configuration(pfm, i):
    _run_config(pfm, i, pfm.PF_LAYOUT_BATCHED)


@pytest.mark.parametrize("i", range(12))
def test_random_plain_configuration(pfm, i):
    _run_config(pfm, i, pfm.PF_LAYOUT_PLAIN)
