"""Pins for the oracle's SMC over parameters with attached particle filters
(SMC^2, Sec. 3.2.2, Alg. 4), each against something other than the SMC^2
code itself:

* the whole-filter copy index against exact rational arithmetic (systematic
  selection on equal weights, brute force over small sizes);
* one theta-particle with every move rejected reduces the algorithm to the
  bootstrap filter of Alg. 2: likelihood increments, likelihood, evidence
  and final particles equal the oracle's filter run;
* with every move inside the prior accepted, each theta-particle's
  parameters are its ancestor's plus the random-walk step, its likelihood is
  a fresh filter run of the proposal over t_{0:i-1}, and its next increment
  is that proposal filter advanced one interval by the filter pieces;
* the theta-ancestors are the systematic resampling of the previous time's
  theta-log-weights;
* on the windkessel model, moving only the initial-pressure mean m0 under a
  uniform prior, the evidence estimate is unbiased for the integral of the
  Kalman likelihood over the prior (computed by quadrature).
"""
import dataclasses
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.special

import workloads as W


def _l96(B, n, T, d=8, seed=0):
    base = W.lorenz96(d=d, N=1, T=T, seed=seed)
    return base, np.asarray(n, dtype=np.int64)


def _with_data(orc, pb):
    _, y = orc.simulate(pb)
    return pb.with_obs(y)


@pytest.mark.parametrize("n_src,n_dst", [(1, 1), (1, 7), (7, 1), (5, 5), (3, 8), (8, 3),
                                         (64, 100), (100, 64), (8192, 256), (256, 8192)])
def test_copy_index_is_exact_systematic_selection(orc, n_src, n_dst):
    rng = np.random.default_rng(n_src * 131 + n_dst)
    for w in [0, 1, 2 ** 31, 2 ** 32 - 1] + list(rng.integers(0, 2 ** 32, size=4)):
        idx = np.array([orc.copy_index(k, n_src, n_dst, int(w)) for k in range(n_dst)])
        u = Fraction(int(w), 2 ** 32)
        ref = [math.floor((k + u) * n_src / n_dst) for k in range(n_dst)]
        np.testing.assert_array_equal(idx, ref)
        cnt = np.bincount(idx, minlength=n_src)
        assert cnt.sum() == n_dst and np.all(np.diff(idx) >= 0)
        assert set(np.unique(cnt)) <= {n_dst // n_src, -(-n_dst // n_src)}


@pytest.mark.parametrize("model", ["l96", "wk"])
def test_one_theta_particle_without_moves_is_the_particle_filter(orc, model):
    if model == "l96":
        pb = _with_data(orc, W.lorenz96(d=8, N=200, T=7))
    else:
        pb = _with_data(orc, W.windkessel(N=150, T=9))
    inp = W.smc2_inputs(pb.theta[:1], pb.T, np.full(pb.n_theta, 0.1),
                        np.full(pb.n_theta, -np.inf), np.full(pb.n_theta, np.inf), seed=11)
    inp = dataclasses.replace(inp, log_alpha=np.full_like(inp.log_alpha, np.inf))  # reject all
    r = orc.smc2(pb, inp)
    ref = orc.pf_run(pb, theta=pb.theta[0], N=int(pb.n_particles[0]), b=0, it=0)
    assert r["status"] == 0 and r["accepts"][0] == 0
    np.testing.assert_array_equal(r["logw_trace"][:, 0], ref["ell"])
    assert r["loglik"][0] == ref["loglik"]
    assert r["log_evidence"] == pytest.approx(ref["loglik"], rel=1e-14)
    np.testing.assert_array_equal(r["x"], ref["x"])
    np.testing.assert_array_equal(r["theta"][0], pb.theta[0])
    assert np.all(r["anc"] == 0) and np.all(r["ess"] == 1.0)


def test_accepted_moves_take_the_proposal_filter(orc):
    base, n = _l96(3, [40, 40, 40], T=5)
    pb = _with_data(orc, base)
    th0 = np.array([[8.0, 0.10], [7.5, 0.20], [8.6, 0.15]])
    pb = dataclasses.replace(pb, theta=th0, n_particles=n)
    inp = W.smc2_l96_inputs(th0, pb.T, seed=7, step_f=0.3, step_s=0.05)
    inp = dataclasses.replace(inp, log_alpha=np.full_like(inp.log_alpha, -np.inf))  # accept all
    r = orc.smc2(pb, inp)
    prev = th0
    for i in range(1, pb.T + 1):
        a = r["anc"][i - 1]
        cur = prev[a]
        prop = cur + inp.step_sd * inp.z[i - 1]
        inside = np.all((prop >= inp.lo) & (prop <= inp.hi), axis=1)
        np.testing.assert_array_equal(r["acc"][i - 1], inside.astype(np.int32))
        want = np.where(inside[:, None], prop, cur)
        np.testing.assert_array_equal(r["theta_trace"][i - 1], want)
        for j in np.flatnonzero(inside):
            # the proposal filter over t_{0:i-1}, then one interval with iteration 0
            p = orc.pf_run(pb, theta=want[j], N=int(n[j]), b=int(j), it=i, T=i - 1)
            xp = orc.propagate(pb, want[j], p["x"], i, b=int(j), it=0)
            lw = orc.weight(pb, want[j], xp, i)
            _, ell, _, _ = orc.reduce_resample(lw, orc.resample_u(pb.seed, i, int(j), 0))
            assert r["logw_trace"][i - 1, j] == ell
        prev = want


@pytest.mark.parametrize("moves", [True, False])
def test_theta_ancestors_are_systematic_on_the_theta_weights(orc, moves):
    base, n = _l96(6, [30, 64, 17, 50, 64, 9], T=6)
    pb = _with_data(orc, base)
    th0, _ = W.batched_thetas(6, seed=21)
    pb = dataclasses.replace(pb, theta=th0, n_particles=n)
    inp = W.smc2_l96_inputs(th0, pb.T, seed=8)
    if not moves:
        inp = dataclasses.replace(inp, log_alpha=np.full_like(inp.log_alpha, np.inf))
    r = orc.smc2(pb, inp)
    np.testing.assert_array_equal(r["anc"][0], np.arange(6))
    if not moves:
        # parameters and likelihoods travel down the theta-genealogy
        line = np.arange(6)
        ll = np.zeros(6)
        for i in range(pb.T):
            line = line[r["anc"][i]]
            ll = ll[r["anc"][i]] + r["logw_trace"][i]
            np.testing.assert_array_equal(r["theta_trace"][i], th0[line])
        np.testing.assert_array_equal(r["loglik"], ll)
    for i in range(2, pb.T + 1):
        v = r["logw_trace"][i - 2]
        st, ev, ess, a = orc.reduce_resample(v, inp.u[i - 1])
        np.testing.assert_array_equal(r["anc"][i - 1], a)
        assert r["ess"][i - 2] == ess
        wb = scipy.special.softmax(v)
        cnt = np.bincount(a, minlength=6)
        assert np.all((cnt == np.floor(6 * wb)) | (cnt == np.ceil(6 * wb)))
    ev = sum(scipy.special.logsumexp(r["logw_trace"][i]) - math.log(6) for i in range(pb.T))
    assert r["log_evidence"] == pytest.approx(ev, rel=1e-12)


def _kalman_evidence_over_m0(orc, pb, lo, hi, n=1601):
    grid = np.linspace(lo, hi, n)
    ll = np.empty(n)
    for g, m0 in enumerate(grid):
        th = pb.theta[0].copy()
        th[4] = m0
        ll[g], _ = orc.kf_wk(pb, th)
    wq = np.full(n, (hi - lo) / (n - 1))
    wq[0] *= 0.5
    wq[-1] *= 0.5
    return scipy.special.logsumexp(ll, b=wq / (hi - lo))


def test_windkessel_evidence_is_unbiased_for_the_kalman_integral(orc):
    """E[Z_hat] = integral of p(y | m0) over the prior: over R independent
    runs, mean(log Z_hat) + var/2 sits at log Z within sampling error."""
    B, N, T, R = 12, 64, 10, 40
    base = W.windkessel(N=N, T=T, B=B)
    # initial-pressure sd 3 (instead of 15) so that the likelihood varies by
    # about 25 nats over the prior of m0 and the moves matter
    th = base.theta.copy()
    th[:, 5] = 3.0
    base = dataclasses.replace(base, theta=th, data_theta=th[0].copy())
    _, y = orc.simulate(base)
    base = base.with_obs(y)
    log_z = _kalman_evidence_over_m0(orc, base, 70.0, 110.0)
    ev = []
    for rep in range(R):
        pb = dataclasses.replace(base, seed=100 + rep)
        inp = W.smc2_wk_m0_inputs(base.theta[0], B, T, seed=200 + rep)
        r = orc.smc2(pb, inp)
        assert r["status"] == 0
        ev.append(r["log_evidence"])
    ev = np.array(ev)
    sd = ev.std(ddof=1)
    centre = ev.mean() + 0.5 * sd ** 2
    assert abs(centre - log_z) <= 4.0 * sd / math.sqrt(R) + 0.02, (centre, log_z, sd)
    assert sd < 1.0


# ---------------------------------------------------------------- attached Kalman filters

def _wk_base(orc, B, N, T, s0=3.0):
    base = W.windkessel(N=N, T=T, B=B)
    th = base.theta.copy()
    th[:, 5] = s0
    base = dataclasses.replace(base, theta=th, data_theta=th[0].copy())
    _, y = orc.simulate(base)
    return base.with_obs(y)


def test_kalman_intervals_compose_to_the_kalman_filter(orc):
    pb = _wk_base(orc, 1, 1, 15)
    ll, ell = orc.kf_wk(pb)
    m, V, tot = pb.theta[0][4], pb.theta[0][5] ** 2, 0.0
    for t in range(1, pb.T + 1):
        e, m, V = orc.kf_wk_interval(pb, pb.theta[0], t, m, V)
        assert e == ell[t - 1]
        tot = tot + e
    assert tot == ll


def test_kalman_smc_single_theta_without_moves_is_the_kalman_filter(orc):
    pb = _wk_base(orc, 1, 1, 12)
    inp = W.smc2_wk_m0_inputs(pb.theta[0], 1, pb.T, seed=21)
    inp = dataclasses.replace(inp, log_alpha=np.full_like(inp.log_alpha, np.inf))
    r = orc.smc2_kalman(pb, inp)
    ll, ell = orc.kf_wk(pb, inp.theta0[0])
    np.testing.assert_array_equal(r["logw_trace"][:, 0], ell)
    assert r["loglik"][0] == ll
    assert r["log_evidence"] == pytest.approx(ll, rel=1e-14)
    assert r["accepts"][0] == 0


def test_kalman_smc_accepted_moves_carry_the_proposal_filter(orc):
    pb = _wk_base(orc, 4, 1, 6)
    inp = W.smc2_wk_m0_inputs(pb.theta[0], 4, pb.T, seed=22)
    inp = dataclasses.replace(inp, log_alpha=np.full_like(inp.log_alpha, -np.inf))
    r = orc.smc2_kalman(pb, inp)
    # every inside move accepted: the final likelihood of a theta-particle
    # whose last move was accepted is its proposal's Kalman likelihood over
    # t_{0:T-1} plus its last increment
    T = pb.T
    for j in np.flatnonzero(r["acc"][T - 1]):
        ll, ell = orc.kf_wk(pb, r["theta"][j])
        assert r["loglik"][j] == pytest.approx(ll, rel=1e-13)
        assert r["logw_trace"][T - 1, j] == pytest.approx(ell[T - 1], rel=1e-13)


def test_kalman_smc_evidence_is_unbiased_for_the_kalman_integral(orc):
    B, T, R = 16, 10, 40
    base = _wk_base(orc, B, 1, T)
    log_z = _kalman_evidence_over_m0(orc, base, 70.0, 110.0)
    ev = []
    for rep in range(R):
        inp = W.smc2_wk_m0_inputs(base.theta[0], B, T, seed=600 + rep)
        r = orc.smc2_kalman(base, inp)
        assert r["status"] == 0
        ev.append(r["log_evidence"])
    ev = np.array(ev)
    sd = ev.std(ddof=1)
    centre = ev.mean() + 0.5 * sd ** 2
    assert abs(centre - log_z) <= 4.0 * sd / math.sqrt(R) + 0.01, (centre, log_z, sd)


def test_kalman_smc_without_moves_follows_the_genealogy(orc):
    """No move accepted: every theta-particle's attached filter has seen
    t_1..t_i with one parameter value, so its increments and likelihood are
    the plain Kalman filter's for that value, whichever slots it passed."""
    pb = _wk_base(orc, 8, 1, 9)
    inp = W.smc2_wk_m0_inputs(pb.theta[0], 8, pb.T, seed=23)
    inp = dataclasses.replace(inp, log_alpha=np.full_like(inp.log_alpha, np.inf))
    r = orc.smc2_kalman(pb, inp)
    line = np.arange(8)
    moved = False
    for i in range(pb.T):
        line = line[r["anc"][i]]
        moved |= np.any(r["anc"][i] != np.arange(8))
        for j in range(8):
            _, ell = orc.kf_wk(pb, inp.theta0[line[j]])
            assert r["logw_trace"][i, j] == ell[i]
    for j in range(8):
        ll, _ = orc.kf_wk(pb, inp.theta0[line[j]])
        assert r["loglik"][j] == ll
    assert moved  # the theta-resampling did move filters between slots
