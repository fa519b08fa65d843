"""Pins for the oracle's marginal Metropolis-Hastings on the windkessel's
(R, C, Z, sigma^2) with the Kalman likelihood (Sec. 3.2.1, eq. mh, Alg. 3 on
Alg. 1; priors and proposals of Sec. 2.1.1), each against something other
than the chain code itself:

* Phi^{-1} against scipy's ndtri over both tails;
* the parameter map (a, c) against a numerical solution of the RC circuit's
  ODE over one substep with the flow held (eq. 2-windkessel);
* the Kalman log-likelihood at mapped parameters against the dense Gaussian
  density of all observations, built from the model's linear recursion;
* with no observations (T = 0) the chains' stationary law is the prior: the
  prior's CDF at the chain states is uniform.  Steps as wide as the priors
  make the truncated-Gaussian and Inverse-Gamma proposal corrections matter
  (leaving out or flipping any of them, or a prior exponent, moves one of
  these means by more than 0.03);
* with one parameter moving under data, the chains' mean matches the
  posterior mean by quadrature of prior x Kalman likelihood;
* with every step switched off every move is accepted (the ratio is 1).
"""
import numpy as np
import pytest
import scipy.integrate
import scipy.special
import scipy.stats

import workloads as W


def test_ndtri_matches_library(orc):
    # normal (not subnormal) p: the chains' arguments are at least 2^-34
    ps = np.concatenate([10.0 ** -np.arange(1.0, 307.0, 3.0), np.linspace(1e-3, 1 - 1e-3, 999),
                         1.0 - 10.0 ** -np.arange(1.0, 16.0), [0.5, 2.0 ** -34]])
    for p in ps:
        ref = scipy.special.ndtri(p)
        assert abs(orc.ndtri(p) - ref) <= 4e-15 * max(1.0, abs(ref)), p


@pytest.mark.parametrize("R,C", [(1.0, 1.5), (0.9, 3.0), (2.5, 0.4)])
def test_parameter_map_is_the_circuit_step(orc, R, C):
    pb = W.windkessel_paper(N=1, T=1)
    spec = W.WkMh()
    th = orc.wk_theta(pb, spec, [R, C, 0.05, 16.0])
    P0, F = 93.0, 310.0
    # C dP/dt = F - P / R over one substep with the flow held
    sol = scipy.integrate.solve_ivp(lambda t, P: (F - P / R) / C, (0.0, pb.h), [P0],
                                    rtol=1e-13, atol=1e-12, method="DOP853")
    assert abs(th[0] * P0 + th[1] * F - sol.y[0, -1]) < 1e-9
    # the same map with zero flow isolates a, with zero pressure c
    sol0 = scipy.integrate.solve_ivp(lambda t, P: (-P / R) / C, (0.0, pb.h), [1.0],
                                     rtol=1e-13, atol=1e-14, method="DOP853")
    assert abs(th[0] - sol0.y[0, -1]) < 1e-11
    assert th[2] == 0.05 and th[4] == spec.m0 and th[5] == spec.s0
    # noise on the flow: per-substep pressure sd = c sigma
    assert abs(th[3] - th[1] * 4.0) < 1e-14


def test_kalman_likelihood_is_the_dense_gaussian(orc):
    T, K = 6, 10
    pb = W.windkessel_paper(N=1, T=T, K=K)
    rng = np.random.default_rng(8)
    spec = W.WkMh()
    for R, C, Z, s2 in [(1.0, 1.5, 0.03, 25.0), (1.4, 0.8, 0.06, 4.0), (0.7, 2.2, 0.01, 60.0)]:
        y = 90.0 + 10.0 * rng.standard_normal((T, 1))
        pbo = pb.with_obs(y)
        th = orc.wk_theta(pbo, spec, [R, C, Z, s2])
        ll, _ = orc.kf_wk(pbo, th)
        # P_n = a P_{n-1} + c (F_{n-1} + xi_{n-1}): P_n is linear in
        # (P_0, xi_0..xi_{n-1}); build its mean and covariance directly
        a, c = np.exp(-pb.h / (R * C)), R * (1.0 - np.exp(-pb.h / (R * C)))
        n_sub = T * K
        mean = np.zeros(n_sub + 1)
        G = np.zeros((n_sub + 1, n_sub + 1))  # rows: P_n; cols: P_0, xi_0..
        mean[0], G[0, 0] = spec.m0, spec.s0
        for n in range(1, n_sub + 1):
            mean[n] = a * mean[n - 1] + c * pb.q[n - 1]
            G[n] = a * G[n - 1]
            G[n, n] = c * np.sqrt(s2)
        rows = np.arange(1, T + 1) * K
        mu = mean[rows] + Z * pb.q[rows]
        S = G[rows] @ G[rows].T + pb.obs_sd ** 2 * np.eye(T)
        ref = scipy.stats.multivariate_normal(mu, S).logpdf(y[:, 0])
        assert abs(ll - ref) < 1e-9 * max(1.0, abs(ref)), (R, C, Z, s2, ll, ref)


def _pit(th, spec):
    cols = [scipy.special.gammainc(spec.prior_shape[k], th[:, k] / spec.prior_scale[k])
            for k in range(3)]
    cols.append(scipy.special.gammaincc(spec.ig_shape, spec.ig_scale / th[:, 3]))
    return np.stack(cols, 1)


def test_prior_only_chains_sample_the_prior(orc):
    spec = W.WkMh(step_sd=(1.0, 1.5, 0.03))
    pb = W.windkessel_paper(N=1, T=0)
    inp = W.wk_mh_inputs(spec, chains=128, iters=4000, seed=11)
    out = orc.kf_pmmh(pb, spec, inp)
    assert np.all(out["ll"] == 0.0)
    acc = out["accepts"].mean() / 4000
    assert 0.1 < acc < 0.7
    pit = _pit(out["theta"].reshape(-1, 4), spec)
    np.testing.assert_allclose(pit.mean(0), 0.5, atol=0.02)
    np.testing.assert_allclose(pit.var(0), 1.0 / 12.0, atol=0.005)


def test_one_parameter_posterior_matches_quadrature(orc):
    R0, C0, Z0, s20 = 1.0, 1.5, 0.03, 25.0
    pb = W.windkessel_paper(N=1, T=40, R=R0, C=C0, Z=Z0, sigma2=s20)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    spec = W.WkMh(step_sd=(0.03, 0.0, 0.0), ig_prop_factor=0.0)

    def log_post(R):
        th = orc.wk_theta(pb, spec, [R, C0, Z0, s20])
        return orc.kf_wk(pb, th)[0] + orc.wk_log_prior(spec, [R, C0, Z0, s20])

    grid = np.linspace(0.5, 1.6, 2201)
    lp = np.array([log_post(R) for R in grid])
    w = np.exp(lp - lp.max())
    assert w[0] < 1e-12 and w[-1] < 1e-12  # the grid holds the posterior
    post_mean = np.trapezoid(grid * w, grid) / np.trapezoid(w, grid)
    post_sd = np.sqrt(np.trapezoid((grid - post_mean) ** 2 * w, grid) / np.trapezoid(w, grid))
    chains, iters, burn = 32, 3000, 300
    inp = W.wk_mh_inputs(spec, chains=chains, iters=iters, seed=12,
                         theta0=np.array([R0, C0, Z0, s20]))
    out = orc.kf_pmmh(pb, spec, inp)
    R = out["theta"][burn:, :, 0]
    assert np.all(out["theta"][:, :, 1:] == [C0, Z0, s20])
    # standard error from batch means over each chain's 10 batches
    bm = R.reshape(10, -1, chains).mean(1)
    se = bm.std(ddof=1) / np.sqrt(bm.size)
    assert abs(R.mean() - post_mean) < max(5.0 * se, 0.02 * post_sd), (R.mean(), post_mean, se)
    assert abs(R.std() - post_sd) < 0.15 * post_sd


def test_no_steps_accept_every_move(orc):
    pb = W.windkessel_paper(N=1, T=20)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    spec = W.WkMh(step_sd=(0.0, 0.0, 0.0), ig_prop_factor=0.0)
    inp = W.wk_mh_inputs(spec, chains=4, iters=30, seed=13)
    out = orc.kf_pmmh(pb, spec, inp)
    assert np.all(out["accepts"] == 30)
    np.testing.assert_array_equal(out["theta"], np.broadcast_to(inp.theta0, (30, 4, 4)))
    for c in range(4):
        ll = orc.kf_wk(pb, orc.wk_theta(pb, spec, inp.theta0[c]))[0]
        assert np.all(out["ll"][:, c] == ll)
