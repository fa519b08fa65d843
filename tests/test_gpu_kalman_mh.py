"""GPU parity of marginal Metropolis-Hastings on the windkessel's (R, C, Z,
sigma^2) with the exact Kalman likelihood (Alg. 3 on Alg. 1), through the
C ABI, against the oracle's chains on the same inputs.  The device exp, log,
erfc and Phi^{-1} may differ from the host's in the last bits, so states and
likelihoods are compared within a relative tolerance; every accept decision
must be the oracle's."""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

REL_THETA = 1e-12
REL_LL = 1e-11


@pytest.fixture(scope="module")
def pfm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_3277_amd as pfm
    pfm.load()
    return pfm


def _paper_wk(B, T, K=10):
    pb = W.windkessel_paper(N=1, T=T, K=K, B=B)
    _, y = oracle.simulate(pb)
    return pb.with_obs(y)


def _run(pfm, pb, spec, inp, iters=None):
    f = pfm.Filter(pb, precision=pfm.PF_FP64, layout=pfm.PF_LAYOUT_PLAIN)
    out = f.kalman_pmmh(spec, inp.theta0, inp.prop, inp.alpha, iters=iters)
    res = {k: v.cpu().numpy() for k, v in out.items()}
    f.close()
    return res


def _subset(inp, sel):
    return W.WkMhInputs(inp.theta0[sel], inp.prop[:, sel], inp.alpha[:, sel])


def _compare(gpu, ref, spec, sel=None, iters=None):
    """Decisions equal; states within REL_THETA relative or 1e-12 of the step
    sd (a proposal near the truncation point is a difference of nearly equal
    numbers, where an ulp of Phi^{-1} is absolute, not relative)."""
    th, ll, acc = gpu["theta"], gpu["ll"], gpu["accepts"]
    if sel is not None:
        th, ll, acc = th[:, sel], ll[:, sel], acc[sel]
    if iters is not None:
        th, ll = th[:iters], ll[:iters]
    np.testing.assert_array_equal(acc, ref["accepts"])
    # same decisions: a state changes on the device exactly when it changes in the oracle
    moved_g = np.any(np.diff(th, axis=0) != 0, axis=2)
    moved_r = np.any(np.diff(ref["theta"], axis=0) != 0, axis=2)
    np.testing.assert_array_equal(moved_g, moved_r)
    atol = np.array(list(spec.step_sd) + [0.0]) * 1e-12
    bad = np.abs(th - ref["theta"]) > REL_THETA * np.abs(ref["theta"]) + atol
    assert not bad.any(), (np.argwhere(bad)[:5], th[bad][:5], ref["theta"][bad][:5])
    np.testing.assert_allclose(ll, ref["ll"], rtol=REL_LL, atol=1e-12)


@pytest.mark.parametrize("B", [1, 64, 100])
def test_paper_chains_match_oracle(pfm, B):
    pb = _paper_wk(B, T=60)
    spec = W.WkMh()
    # start near the data's parameters so the chains move (the paper's steps
    # are small against the prior)
    rng = np.random.default_rng(B)
    th0 = np.array([1.0, 1.5, 0.03, 25.0]) * rng.uniform(0.9, 1.1, size=(B, 4))
    inp = W.wk_mh_inputs(spec, chains=B, iters=150, seed=20 + B, theta0=th0)
    gpu = _run(pfm, pb, spec, inp)
    ref = oracle.kf_pmmh(pb, spec, inp)
    _compare(gpu, ref, spec)
    assert ref["accepts"].sum() > 0.05 * B * 150
    for c in range(B):
        ll0 = oracle.kf_wk(pb, oracle.wk_theta(pb, spec, th0[c]))[0]
        assert abs(gpu["ll0"][c] - ll0) <= REL_LL * abs(ll0)


def test_wide_steps_match_oracle(pfm):
    """Few observations, steps as wide as the priors: the truncation and the
    sigma^2 proposal's correction weigh on every move."""
    pb = _paper_wk(200, T=3)
    spec = W.WkMh(step_sd=(1.0, 1.5, 0.03))
    inp = W.wk_mh_inputs(spec, chains=200, iters=400, seed=31)
    gpu = _run(pfm, pb, spec, inp)
    ref = oracle.kf_pmmh(pb, spec, inp)
    _compare(gpu, ref, spec)
    assert ref["accepts"].sum() > 0.05 * 200 * 400


def test_extreme_uniforms_match_oracle(pfm):
    """Uniforms at the ends of (0, 1) (the inversion's far tails) and tiny or
    huge Gamma variates."""
    B, iters = 64, 60
    pb = _paper_wk(B, T=20)
    spec = W.WkMh(step_sd=(0.1, 0.2, 0.004))
    inp = W.wk_mh_inputs(spec, chains=B, iters=iters, seed=32,
                         theta0=np.array([1.0, 1.5, 0.03, 25.0]))
    rng = np.random.default_rng(5)
    ends = np.array([2.0 ** -33, 2.0 ** -20, 1e-6, 0.5, 0.5 + 2.0 ** -33, 1 - 1e-6,
                     1 - 2.0 ** -20, 1 - 2.0 ** -33])
    mask = rng.random((iters, B, 3)) < 0.3
    inp.prop[:, :, :3] = np.where(mask, rng.choice(ends, size=(iters, B, 3)), inp.prop[:, :, :3])
    g = inp.prop[:, :, 3]
    inp.prop[:, :, 3] = np.where(rng.random((iters, B)) < 0.2,
                                 rng.choice([1e-300, 1e-8, 1e8, 1e300], size=(iters, B)), g)
    gpu = _run(pfm, pb, spec, inp)
    ref = oracle.kf_pmmh(pb, spec, inp)
    _compare(gpu, ref, spec)


def test_fixed_parameters_accept_every_move(pfm):
    pb = _paper_wk(5, T=30)
    spec = W.WkMh(step_sd=(0.0, 0.0, 0.0), ig_prop_factor=0.0)
    inp = W.wk_mh_inputs(spec, chains=5, iters=25, seed=33)
    gpu = _run(pfm, pb, spec, inp)
    assert np.all(gpu["accepts"] == 25)
    np.testing.assert_array_equal(gpu["theta"], np.broadcast_to(inp.theta0, (25, 5, 4)))
    _compare(gpu, oracle.kf_pmmh(pb, spec, inp), spec)


def test_zero_iterations(pfm):
    pb = _paper_wk(3, T=30)
    spec = W.WkMh()
    inp = W.wk_mh_inputs(spec, chains=3, iters=1, seed=34)
    gpu = _run(pfm, pb, spec, inp, iters=0)
    assert gpu["theta"].shape == (0, 3, 4)
    assert np.all(gpu["accepts"] == 0)
    for c in range(3):
        ll0 = oracle.kf_wk(pb, oracle.wk_theta(pb, spec, inp.theta0[c]))[0]
        assert abs(gpu["ll0"][c] - ll0) <= REL_LL * abs(ll0)


def test_full_size_chains_sampled(pfm):
    """512 chains x 1,000 iterations on T = 100 (the benchmark's shape);
    chains 0, 1, 255, 256, 511 against the oracle, and every chain's final
    likelihood equal to a fresh Kalman run at its final state."""
    B, iters = 512, 1000
    pb = _paper_wk(B, T=100)
    spec = W.WkMh()
    rng = np.random.default_rng(7)
    th0 = np.array([1.0, 1.5, 0.03, 25.0]) * rng.uniform(0.8, 1.2, size=(B, 4))
    inp = W.wk_mh_inputs(spec, chains=B, iters=iters, seed=35, theta0=th0)
    gpu = _run(pfm, pb, spec, inp)
    sel = np.array([0, 1, 255, 256, 511])
    ref = oracle.kf_pmmh(pb, spec, _subset(inp, sel))
    _compare(gpu, ref, spec, sel=sel)
    for c in range(0, B, 37):
        ll = oracle.kf_wk(pb, oracle.wk_theta(pb, spec, gpu["theta"][-1, c]))[0]
        assert abs(gpu["ll"][-1, c] - ll) <= REL_LL * abs(ll)


def test_rejects_bad_arguments(pfm):
    pb = _paper_wk(2, T=10)
    spec = W.WkMh()
    inp = W.wk_mh_inputs(spec, chains=2, iters=3, seed=36)
    f = pfm.Filter(pb, precision=pfm.PF_FP64)
    for bad in [dict(prior_shape=(0.0, 2.0, 2.0)), dict(prior_scale=(0.9, -1.0, 0.03)),
                dict(step_sd=(0.03, float("nan"), 0.0)), dict(ig_scale=0.0),
                dict(ig_prop_factor=-1.0), dict(ig_prop_shape=0.0), dict(s0=-1.0)]:
        with pytest.raises(pfm.PfError):
            f.kalman_pmmh(dataclasses.replace(spec, **bad), inp.theta0, inp.prop, inp.alpha)
    f.close()
    l96 = pfm.Filter(W.lorenz96(d=8, N=64, T=3), precision=pfm.PF_FP64)
    with pytest.raises(pfm.PfError, match="windkessel"):
        l96.kalman_pmmh(spec, np.ones((1, 4)), np.full((3, 1, 4), 0.5), np.full((3, 1), 0.5))
    l96.close()
