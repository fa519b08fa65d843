"""Pins for the oracle's filter: likelihood increment, ESS, systematic
resampling and the whole bootstrap filter (Alg. 2).

* ell_t against scipy's logsumexp minus ln N; ESS against 1/sum(wbar^2);
* systematic resampling: offspring counts sum to N and lie in
  {floor(N wbar_j), ceil(N wbar_j)}, ancestors are sorted, zero weights get no
  offspring; the outcome equals numpy's searchsorted on the normalised
  cumulative weights; brute force over every u-interval at N <= 8 gives the
  unbiased expectation E[o_j] = N wbar_j;
* the Kalman filter against the dense joint-Gaussian density of the
  observations (scipy multivariate normal);
* the particle filter against the Kalman filter: E[exp(ll - ll_KF)] = 1 (the
  estimate is unbiased, Sec. 3.1.2) and, with the state made deterministic,
  the likelihood collapses to a closed form;
* resume: the filter is defined over an interval (Sec. 3.1.2), and with a
  positional generator the run over t_{0:T} equals the run over t_{0:s}
  followed by a run over t_{s:T} started from its resampled set and running
  likelihood, bit for bit.
"""
import dataclasses
import math

import numpy as np
import pytest
import scipy.special
import scipy.stats

import workloads as W


def _offspring(a, N):
    return np.bincount(a, minlength=N)


def test_ell_and_ess(orc):
    rng = np.random.default_rng(0)
    for N in (1, 2, 7, 1000):
        lw = rng.normal(size=N) * 30 - 500
        st, ell, ess, a = orc.reduce_resample(lw, 0.3)
        assert st == orc.ORC_OK
        assert ell == pytest.approx(scipy.special.logsumexp(lw) - math.log(N), abs=1e-12)
        wb = scipy.special.softmax(lw)
        assert ess == pytest.approx(1.0 / np.sum(wb ** 2), rel=1e-12)


ADVERSARIAL = [
    np.array([0.0]),
    np.array([0.0, -np.inf, -np.inf, -np.inf]),          # one dominant
    np.log(np.array([2.0, 1.0, 1.0, 0.0, 4.0, 0.0, 0.0, 0.0])),  # exact multiples of 1/N, zeros
    np.zeros(8),                                           # ties
    np.array([-1e-3, 0.0, np.nan, -2.0, -np.inf, 5.0, 5.0, -40.0]),  # NaN counts as zero weight
    np.array([-800.0, -800.0 - 1e-12, -801.0]),            # far from 0: max shift
]


@pytest.mark.parametrize("lw", ADVERSARIAL + [np.random.default_rng(s).normal(size=n) * 4
                                              for s, n in [(1, 5), (2, 64), (3, 1000), (4, 4097)]])
def test_systematic_invariants(orc, lw):
    N = lw.size
    w = np.where(np.isnan(lw), 0.0, np.exp(lw - np.nanmax(lw)))
    wb = w / w.sum()
    for u in (orc.u01(0), 0.123456789, 0.5, orc.u01(2 ** 32 - 1)):
        st, ell, ess, a = orc.reduce_resample(lw, u)
        assert st == orc.ORC_OK
        assert np.all(np.diff(a) >= 0) and a.min() >= 0 and a.max() < N
        o = _offspring(a, N)
        assert o.sum() == N
        assert np.all(o >= np.floor(N * wb - 1e-9)) and np.all(o <= np.ceil(N * wb + 1e-9))
        assert np.all(o[wb == 0] == 0)
        # library routine: first j whose normalised cumulative weight exceeds (u+k)/N
        cw = np.cumsum(wb)
        ref = np.searchsorted(cw, (u + np.arange(N)) / N, side="right")
        ref = np.minimum(ref, np.flatnonzero(wb > 0).max())
        mism = np.flatnonzero(ref != a)
        # only strata within rounding of a cell boundary may differ
        for k in mism:
            assert np.min(np.abs(cw - (u + k) / N)) < 1e-12


def _breakpoints(wb):
    N = wb.size
    c = np.cumsum(wb) * N
    f = np.mod(c, 1.0)
    pts = np.unique(np.concatenate([[0.0, 1.0], f[(f > 0) & (f < 1)]]))
    return pts


@pytest.mark.parametrize("weights", [
    [1.0], [0.3, 0.7], [1, 2, 3], [5, 1, 1, 1, 1, 1, 1, 1], [1, 0, 0, 3, 0, 2, 2, 0],
    [0.25, 0.25, 0.25, 0.25], [1e-9, 1, 1e-9, 1, 1e-9], [0.9, 0.01, 0.01, 0.08],
])
def test_systematic_brute_force_unbiased(orc, weights):
    w = np.asarray(weights, dtype=np.float64)
    N = w.size
    wb = w / w.sum()
    with np.errstate(divide="ignore"):
        lw = np.log(w)
    pts = _breakpoints(wb)
    exp = np.zeros(N)
    for lo, hi in zip(pts[:-1], pts[1:]):
        if hi - lo < 1e-15:
            continue
        st, _, _, a = orc.reduce_resample(lw, 0.5 * (lo + hi))
        exp += (hi - lo) * _offspring(a, N)
    np.testing.assert_allclose(exp, N * wb, atol=1e-12)


def test_numeric_status(orc):
    for lw in (np.full(4, -np.inf), np.full(3, np.nan), np.array([np.inf, 0.0])):
        st, ell, ess, a = orc.reduce_resample(lw, 0.5)
        assert st == orc.ORC_NUMERIC and ell == -np.inf
        assert list(a) == list(range(lw.size))


def test_gather(orc):
    x = np.arange(12, dtype=np.float64).reshape(3, 4)
    a = np.array([0, 0, 2, 3], dtype=np.int32)
    np.testing.assert_array_equal(orc.gather(x, a), x[:, a])


def _wk_dense_loglik(pb, y):
    th = pb.theta[0]
    a, c, Z, sp, m0, s0 = th
    K, T = pb.K, pb.T
    n_tot = T * K
    # p_n = a^n p0 + sum_{m<n} a^(n-1-m) c q_m + sum_{m=1..n} a^(n-m) sp z_m
    A = np.zeros((n_tot + 1, n_tot + 1))
    mean = np.zeros(n_tot + 1)
    for n in range(n_tot + 1):
        A[n, 0] = a ** n * s0
        for m in range(1, n + 1):
            A[n, m] = a ** (n - m) * sp
        mean[n] = a ** n * m0 + sum(a ** (n - 1 - m) * c * pb.q[m] for m in range(n))
    obs_n = np.arange(1, T + 1) * K
    cov = (A @ A.T)[np.ix_(obs_n, obs_n)] + pb.obs_sd ** 2 * np.eye(T)
    mu = mean[obs_n] + Z * pb.q[obs_n]
    return scipy.stats.multivariate_normal.logpdf(y[:, 0], mean=mu, cov=cov)


def test_kalman_against_dense_gaussian(orc):
    for T, K in ((1, 10), (5, 10), (12, 3)):
        pb = W.windkessel(N=1, T=T, K=K)
        _, y = orc.simulate(pb)
        pb = pb.with_obs(y)
        ll, ell = orc.kf_wk(pb)
        assert ll == pytest.approx(_wk_dense_loglik(pb, y), abs=1e-9)
        assert ll == pytest.approx(ell.sum(), abs=1e-12)


def test_deterministic_collapse(orc):
    """s0 = sigma_p = 0: all particles coincide, ESS = N, ancestors are the
    identity and the estimate is exactly sum_t log N(y_t; p_t + Z q, 1)."""
    pb = W.windkessel(N=32, T=20)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    th = pb.theta[0].copy()
    th[3] = 0.0
    th[5] = 0.0
    r = orc.pf_run(pb, theta=th, traces=True)
    a, c, Z = th[0], th[1], th[2]
    ref = 0.0
    for t in range(1, pb.T + 1):
        n = t * pb.K
        p = a ** n * th[4] + sum(a ** (n - 1 - m) * c * pb.q[m] for m in range(n))
        ref += scipy.stats.norm.logpdf(y[t - 1, 0], loc=p + Z * pb.q[n], scale=pb.obs_sd)
    assert r["loglik"] == pytest.approx(ref, abs=1e-9)
    np.testing.assert_allclose(r["ess"], 32.0, rtol=1e-14)
    assert np.all(r["anc"] == np.arange(32)[None, :])


def test_pf_unbiased_against_kalman(orc):
    pb = W.windkessel(N=256, T=30)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    ll_kf, _ = orc.kf_wk(pb)
    R = 200
    lls = np.array([orc.pf_run(dataclasses.replace(pb, seed=s))["loglik"] for s in range(R)])
    ratio = np.exp(lls - ll_kf)
    assert abs(ratio.mean() - 1.0) < 4 * ratio.std(ddof=1) / math.sqrt(R) + 1e-3
    # lognormal correction form, as a second view of the same fact
    assert abs(lls.mean() + lls.var(ddof=1) / 2 - ll_kf) < 4 * lls.std(ddof=1) / math.sqrt(R) + 0.02


def test_pf_single_particle_is_plain_likelihood(orc):
    """N = 1: no resampling choice; ell_t = log p(y_t | x_t) along the path."""
    pb = W.lorenz96(d=8, N=1, T=10)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    r = orc.pf_run(pb)
    x = orc.init(pb, pb.theta[0], 1)
    for t in range(1, pb.T + 1):
        x = orc.propagate(pb, pb.theta[0], x, t)
        ref = scipy.stats.norm.logpdf(y[t - 1], loc=x[:, 0], scale=0.5).sum()
        assert r["ell"][t - 1] == pytest.approx(ref, abs=1e-11)
    np.testing.assert_array_equal(r["x"], x)


def _interval_run(orc, pb, th, x, t0, t1, ll):
    """Alg. 2 over t_{t0:t1} from the equally weighted set x and running
    log-likelihood ll, one step function at a time."""
    ells = []
    for t in range(t0 + 1, t1 + 1):
        xp = orc.propagate(pb, th, x, t)
        lw = orc.weight(pb, th, xp, t)
        _, e, _, a = orc.reduce_resample(lw, orc.resample_u(pb.seed, t))
        ll = ll + e
        ells.append(e)
        x = orc.gather(xp, a)
    return x, ll, ells


@pytest.mark.parametrize("model", ["windkessel", "lorenz96"])
def test_resume_from_a_checkpoint_is_the_whole_run(orc, model):
    pb = W.windkessel(N=300, T=16) if model == "windkessel" else W.lorenz96(d=8, N=300, T=16)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    th = pb.theta[0]
    full = orc.pf_run(pb)
    for s in (0, 1, 7, 15, 16):
        x, ll, e1 = _interval_run(orc, pb, th, orc.init(pb, th, 300), 0, s, 0.0)
        # the checkpoint crosses a serialisation, as a file would
        x_ck, ll_ck = np.frombuffer(x.tobytes()).reshape(x.shape), float(repr(ll))
        xe, lle, e2 = _interval_run(orc, pb, th, x_ck, s, pb.T, ll_ck)
        np.testing.assert_array_equal(np.array(e1 + e2), full["ell"])
        assert lle == full["loglik"]
        np.testing.assert_array_equal(xe, full["x"])


def test_pmmh_chain_has_the_posterior_as_its_law(orc):
    """Alg. 3 with an unbiased likelihood estimate leaves the exact posterior
    invariant (pseudo-marginal MH): the chain on log F with a uniform prior
    on F (Jacobian F) and a 16-particle filter must reproduce the mean and
    variance of p(log F | y) obtained by quadrature of the likelihood, itself
    the average of 512-particle estimates (unbiased) on a grid.  A dropped
    Jacobian shifts the mean by about the variance (0.013, six standard
    errors); a reversed acceptance test or a missed support check moves it
    further."""
    pb = W.lorenz96(d=4, N=1, T=1)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    th = np.linspace(math.log(6.0), math.log(10.0), 61)
    lik = np.array([np.mean(np.exp([orc.pf_run(pb, theta=np.array([math.exp(t), 0.1]), N=512,
                                               it=s)["loglik"] for s in range(8)]))
                    for t in th])
    dens = lik * np.exp(th)
    dens /= np.trapezoid(dens, th)
    mean_q = np.trapezoid(dens * th, th)
    var_q = np.trapezoid(dens * (th - mean_q) ** 2, th)
    inp = W.pmmh_inputs(chains=4, iters=30000, seed=11)
    r = orc.pmmh(pb, 16, inp)
    lf = r["log_f"][2000:]
    assert np.all(np.exp(lf) >= 6.0) and np.all(np.exp(lf) <= 10.0)
    # standard error from 50 batch means per chain (the chain is correlated)
    nb = 50
    bm = lf[:(lf.shape[0] // nb) * nb].reshape(nb, -1, lf.shape[1]).mean(axis=1)
    se = bm.std(ddof=1) / math.sqrt(bm.size)
    assert abs(lf.mean() - mean_q) < 4 * se + 1e-3, (lf.mean(), mean_q, se)
    assert abs(lf.var() - var_q) < 0.15 * var_q, (lf.var(), var_q)


def test_pmmh_limits(orc):
    pb = W.lorenz96(d=8, N=1, T=8)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    inp = W.pmmh_inputs(chains=2, iters=4)
    # proposals far outside the prior support are all rejected
    far = dataclasses.replace(inp, z=np.full_like(inp.z, 100.0))
    r = orc.pmmh(pb, 32, far)
    assert np.all(r["accepts"] == 0)
    np.testing.assert_array_equal(r["log_f"], np.tile(inp.log_f0, (4, 1)))
    # a zero acceptance uniform (log = -inf) accepts every in-support move; the
    # kept likelihood is the proposal's own filter estimate
    easy = dataclasses.replace(inp, z=np.full_like(inp.z, 0.1), alpha=np.zeros_like(inp.alpha))
    r = orc.pmmh(pb, 32, easy)
    lf = inp.log_f0[None, :] + 0.05 * 0.1 * np.arange(1, 5)[:, None]
    inside = np.all(np.exp(lf) <= 10.0, axis=0)
    for c in range(2):
        if inside[c]:
            assert r["accepts"][c] == 4
            np.testing.assert_allclose(r["log_f"][:, c], lf[:, c], rtol=1e-15)
            th = np.array([math.exp(r["log_f"][-1, c]), 0.1])
            ref = orc.pf_run(pb, theta=th, N=32, b=c, it=4)["loglik"]
            assert r["ll"][-1, c] == ref
