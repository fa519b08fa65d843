"""GPU parity of the resampling variants and of ESS-triggered resampling
with the oracle, through the C ABI, FP64, plain and batched layouts:
log-weights (carried ones included) bit for bit at every time, likelihood
increments within 1e-10 relative, ESS within 1e-9; ancestors bit for bit
(Metropolis and rejection resampling decide on bit-identical log-weights
with the same logarithm; stratified and multinomial resampling compare FP64 sums taken in
another order, so a flip within 1e-9 of an edge would be legitimate and is
checked); final particles bit for bit."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle_resync import resync
import workloads as W

pytestmark = pytest.mark.gpu

REL64 = 1e-10
BAND = 1e-9


@pytest.fixture(scope="module")
def pfm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_3277_amd as pfm
    pfm.load()
    return pfm


def _strat_flips_in_band(lw, a_gpu, a_ref, seed, t, b):
    mism = np.flatnonzero(a_gpu != a_ref)
    if mism.size:
        w = np.exp(lw - lw.max())
        cw = np.cumsum(w) / w.sum()
        N = lw.size
        for k in mism:
            uk = oracle.strat_u(seed, t, b, 0, int(k))
            assert np.min(np.abs(cw - (uk + k) / N)) < BAND
    return mism.size


def _multi_flips_in_band(lw, a_gpu, a_ref, seed, t, b):
    mism = np.flatnonzero(a_gpu != a_ref)
    if mism.size:
        w = np.exp(lw - lw.max())
        cw = np.cumsum(w) / w.sum()
        for k in mism:
            uk = oracle.multi_u(seed, t, b, 0, int(k))
            assert np.min(np.abs(cw - uk)) < BAND
    return mism.size


def _check(pfm, pb, layout, scheme, steps, ess_frac):
    n = pb.n_particles
    off = np.concatenate([[0], np.cumsum(n)])
    refs = [oracle.pf_run_ex(pb, theta=pb.theta[b], N=int(n[b]), b=b, resampler=scheme,
                             steps=steps, ess_frac=ess_frac, traces=True) for b in range(pb.B)]
    f = pfm.Filter(pb, precision=pfm.PF_FP64, layout=layout)
    f.set_resampler(scheme, steps, ess_frac)
    flips = 0
    for t in range(1, pb.T + 1):
        f.step()
        lw = f.logweights()
        for b in range(pb.B):
            np.testing.assert_array_equal(lw[off[b]:off[b + 1]], refs[b]["lw"][t - 1],
                                          err_msg=f"filter {b}, t = {t}")
        f.resample()
        a = f.ancestors()
        flipped = []
        for b in range(pb.B):
            ag, ar = a[off[b]:off[b + 1]], refs[b]["anc"][t - 1]
            if scheme == oracle.RESAMPLE_STRATIFIED:
                nf = _strat_flips_in_band(refs[b]["lw"][t - 1], ag, ar, pb.seed, t, b)
            elif scheme == oracle.RESAMPLE_MULTINOMIAL:
                nf = _multi_flips_in_band(refs[b]["lw"][t - 1], ag, ar, pb.seed, t, b)
            else:
                np.testing.assert_array_equal(ag, ar, err_msg=f"filter {b}, t = {t}")
                nf = 0
            if nf:
                flipped.append(b)
                flips += nf
        if flipped:  # in-band flips: carry on from the oracle's particles
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
    return refs


CASES = [(oracle.RESAMPLE_STRATIFIED, 0, float("inf")),
         (oracle.RESAMPLE_METROPOLIS, 9, float("inf")),
         (oracle.RESAMPLE_SYSTEMATIC, 0, 0.5),
         (oracle.RESAMPLE_STRATIFIED, 0, 0.5),
         (oracle.RESAMPLE_METROPOLIS, 4, 0.5),
         (oracle.RESAMPLE_MULTINOMIAL, 0, float("inf")),
         (oracle.RESAMPLE_MULTINOMIAL, 0, 0.5),
         (oracle.RESAMPLE_REJECTION, 0, float("inf")),
         (oracle.RESAMPLE_REJECTION, 0, 0.5)]


@pytest.mark.parametrize("scheme,steps,ess_frac", CASES)
def test_plain_variants_match_oracle(pfm, scheme, steps, ess_frac):
    base = W.windkessel(N=1, T=12)
    _, y = oracle.simulate(base)
    pb = dataclasses.replace(base.with_obs(y), n_particles=np.array([1500], dtype=np.int64))
    refs = _check(pfm, pb, pfm.PF_LAYOUT_PLAIN, scheme, steps, ess_frac)
    if ess_frac < 1:
        assert 0 < refs[0]["resampled"].sum() < pb.T


@pytest.mark.parametrize("scheme,steps,ess_frac", CASES)
def test_batched_variants_match_oracle(pfm, scheme, steps, ess_frac):
    base = W.lorenz96(d=8, N=1, T=6)
    _, y = oracle.simulate(base)
    th0, _ = W.batched_thetas(4, seed=61)
    pb = dataclasses.replace(base.with_obs(y), theta=th0,
                             n_particles=np.array([300, 64, 2048, 1000], dtype=np.int64))
    _check(pfm, pb, pfm.PF_LAYOUT_BATCHED, scheme, steps, ess_frac)


def test_lorenz96_plain_stratified(pfm):
    base = W.lorenz96(d=8, N=5000, T=5)
    _, y = oracle.simulate(base)
    _check(pfm, base.with_obs(y), pfm.PF_LAYOUT_PLAIN, oracle.RESAMPLE_STRATIFIED, 0,
           float("inf"))


def test_lorenz96_plain_rejection(pfm):
    """Rejection resampling on a larger filter whose weights are far from
    even (many attempts per output)."""
    base = W.lorenz96(d=8, N=5000, T=5)
    _, y = oracle.simulate(base)
    refs = _check(pfm, base.with_obs(y), pfm.PF_LAYOUT_PLAIN, oracle.RESAMPLE_REJECTION, 0,
                  float("inf"))
    assert min(refs[0]["ess"]) < 500


def test_variant_rules(pfm):
    base = W.lorenz96(d=8, N=64, T=3)
    _, y = oracle.simulate(base)
    pb = base.with_obs(y)
    f = pfm.Filter(pb, precision=pfm.PF_FP64)
    for bad in [(5, 0, 1.0), (0, -1, 1.0), (2, 509, 1.0), (0, 0, -0.5), (0, 0, float("nan"))]:
        with pytest.raises(pfm.PfError):
            f.set_resampler(*bad)
    f.set_resampler(pfm.PF_RESAMPLE_STRATIFIED)
    f.step()
    with pytest.raises(pfm.PfError):
        f.resample_u([0.5])
    f.close()
    # graph replay follows the setting like the eager calls
    outs = []
    for graph in (False, True):
        g = pfm.Filter(pb, precision=pfm.PF_FP64, layout=pfm.PF_LAYOUT_BATCHED)
        g.set_resampler(pfm.PF_RESAMPLE_METROPOLIS, 6, 0.7)
        if graph:
            g.graph_run(pb.T)
        else:
            g.advance(pb.T)
        outs.append((g.trace()[0], g.get_state()))
        g.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    outs = []
    for graph in (False, True):
        g = pfm.Filter(pb, precision=pfm.PF_FP64, layout=pfm.PF_LAYOUT_BATCHED)
        g.set_resampler(pfm.PF_RESAMPLE_REJECTION, 0, float("inf"))
        if graph:
            g.graph_run(pb.T)
        else:
            g.advance(pb.T)
        outs.append((g.trace()[0], g.get_state()))
        g.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
