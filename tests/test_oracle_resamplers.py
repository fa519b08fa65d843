"""Pins for the oracle's resampling variants (Sec. 3.3: multinomial,
systematic and stratified resampling, and resamplers that avoid the
collective over the weights) and for resampling triggered by the ESS:

* the general run with systematic resampling at every time equals the plain
  filter run bit for bit;
* stratified ancestors equal numpy's searchsorted of the strata (u_k + k) S
  in N W (the same FP64 products), the offsets are the generator's uniforms,
  offspring counts sum to N and stay within one of floor(b) - floor(a), and
  their mean over many draws is N w_j (unbiased);
* multinomial resampling (as Alg. 2 writes it): the inverse CDF of the
  generator's uniforms (numpy searchsorted), offspring counts with the
  multinomial mean and variance, an unbiased filter;
* Metropolis resampling: no moves is the identity; equal weights give
  uniform ancestors; with many moves the offspring mean approaches N w_j
  (the chain's stationary law), which a reversed acceptance test fails;
* rejection resampling: equal weights keep every particle in place, one
  positive weight takes every output; the attempts are the generator's words
  at their stated counters (also past 512 attempts); each output's law is
  w_k/w_max on staying plus (1 - w_k/w_max) W_j on every j (a reversed or
  missing acceptance test fails), NaN weights are never taken, and the
  filter is unbiased for the Kalman likelihood;
* ESS-triggered resampling: never resampling is sequential importance
  sampling (likelihood = logsumexp of the accumulated log-weights - ln N,
  identity ancestors, particles never gathered); the resampling flags follow
  ESS < fraction N; stratified and ESS-triggered filters are unbiased for
  the Kalman likelihood on the windkessel model.
"""
import dataclasses
import math

import numpy as np
import pytest
import scipy.special
import scipy.stats

import workloads as W


def _data(orc, pb):
    _, y = orc.simulate(pb)
    return pb.with_obs(y)


def _seq_cumsum(w):
    out = np.empty_like(w)
    acc = 0.0
    for j in range(w.size):
        acc = acc + w[j]
        out[j] = acc
    return out


def test_general_run_reduces_to_the_plain_filter(orc):
    pb = _data(orc, W.lorenz96(d=8, N=150, T=6))
    r0 = orc.pf_run(pb, traces=True)
    r1 = orc.pf_run_ex(pb, traces=True)
    for k in ("ell", "ess", "anc", "lw", "x"):
        np.testing.assert_array_equal(r1[k], r0[k], err_msg=k)
    assert r1["loglik"] == r0["loglik"] and np.all(r1["resampled"] == 1)


def test_stratified_offsets_are_the_generator_uniforms(orc):
    for k in (0, 1, 2, 3, 4, 7, 1000):
        w = orc.philox([k >> 2, 5, (orc.TAG_RESAMPLE << 28) | (1 << 20) | 2, 9], [3, 0])
        assert orc.strat_u(3, 5, 9, 2, k) == orc.u01(int(w[k & 3]))


@pytest.mark.parametrize("N", [1, 5, 64, 1000])
def test_stratified_matches_searchsorted_and_counts(orc, N):
    rng = np.random.default_rng(N)
    lw = rng.normal(size=N) * 3.0
    t, b, it = 4, 2, 1
    a = orc.stratified_ancestors(lw, seed=11, t=t, b=b, it=it)
    w = np.exp(lw - lw.max())
    Wc = _seq_cumsum(w)
    S = Wc[-1]
    u = np.array([orc.strat_u(11, t, b, it, k) for k in range(N)])
    ref = np.searchsorted(N * Wc, (u + np.arange(N)) * S, side="right")
    np.testing.assert_array_equal(a, np.minimum(ref, N - 1))
    cnt = np.bincount(a, minlength=N)
    assert cnt.sum() == N and np.all(np.diff(a) >= 0)
    hi = N * Wc / S
    lo = np.concatenate([[0.0], hi[:-1]])
    base = np.floor(hi) - np.floor(lo)
    assert np.all(np.abs(cnt - base) <= 1)


@pytest.mark.parametrize("weights", [[0.3, 0.7], [5, 1, 1, 1, 1, 1, 1, 1], [0.9, 0.01, 0.01, 0.08],
                                     [1, 0, 0, 3, 0, 2, 2, 0]])
def test_stratified_unbiased(orc, weights):
    w = np.asarray(weights, dtype=np.float64)
    N = w.size
    with np.errstate(divide="ignore"):
        lw = np.log(w)
    R = 3000
    cnt = np.array([np.bincount(orc.stratified_ancestors(lw, seed=5, t=t), minlength=N)
                    for t in range(1, R + 1)])
    target = N * w / w.sum()
    sd = cnt.std(axis=0, ddof=1)
    assert np.all(np.abs(cnt.mean(axis=0) - target) <= 4 * sd / math.sqrt(R) + 1e-9)
    assert np.all(cnt[:, w == 0] == 0)


def test_metropolis_limits(orc):
    rng = np.random.default_rng(3)
    lw = rng.normal(size=50)
    np.testing.assert_array_equal(orc.metropolis_ancestors(lw, 0, seed=1, t=1), np.arange(50))
    # equal weights: every proposal is accepted, the last one is uniform
    N, R = 10, 400
    a = np.concatenate([orc.metropolis_ancestors(np.zeros(N), 3, seed=2, t=t) for t in range(R)])
    assert scipy.stats.chisquare(np.bincount(a, minlength=N)).pvalue > 1e-3


def test_metropolis_tends_to_the_weights(orc):
    w = np.array([0.05, 0.1, 0.15, 0.2, 0.5])
    lw = np.log(w)
    N, R, steps = w.size, 2000, 60
    cnt = np.array([np.bincount(orc.metropolis_ancestors(lw, steps, seed=4, t=t), minlength=N)
                    for t in range(1, R + 1)])
    sd = cnt.std(axis=0, ddof=1)
    assert np.all(np.abs(cnt.mean(axis=0) - N * w) <= 4 * sd / math.sqrt(R) + 0.01)
    # a reversed acceptance rule would favour the light particles
    rev = np.array([np.bincount(orc.metropolis_ancestors(-lw, steps, seed=4, t=t), minlength=N)
                    for t in range(1, R + 1)])
    assert rev.mean(axis=0)[-1] < N * w[-1] - 1.0


def test_never_resampling_is_importance_sampling(orc):
    pb = _data(orc, W.lorenz96(d=8, N=64, T=5))
    r = orc.pf_run_ex(pb, ess_frac=0.0, traces=True)
    assert np.all(r["resampled"] == 0)
    assert np.all(r["anc"] == np.arange(64)[None, :])
    ll = scipy.special.logsumexp(r["lw"][-1]) - math.log(64)
    assert r["loglik"] == pytest.approx(ll, rel=1e-12)
    x = orc.init(pb, pb.theta[0], 64)
    for t in range(1, pb.T + 1):
        x = orc.propagate(pb, pb.theta[0], x, t)
    np.testing.assert_array_equal(r["x"], x)
    # the carried log-weights are sums of the per-time log-densities
    x = orc.init(pb, pb.theta[0], 64)
    acc = np.zeros(64)
    for t in range(1, pb.T + 1):
        x = orc.propagate(pb, pb.theta[0], x, t)
        acc = acc + orc.weight(pb, pb.theta[0], x, t)
        np.testing.assert_array_equal(r["lw"][t - 1], acc)


def test_ess_trigger_follows_the_ess(orc):
    pb = _data(orc, W.windkessel(N=200, T=40))
    r = orc.pf_run_ex(pb, ess_frac=0.5, traces=True)
    np.testing.assert_array_equal(r["resampled"], (r["ess"] < 100.0).astype(np.int32))
    assert 0 < r["resampled"].sum() < pb.T


@pytest.mark.parametrize("resampler,ess_frac", [(1, float("inf")), (0, 0.5), (1, 0.5)])
def test_variants_unbiased_against_kalman(orc, resampler, ess_frac):
    pb = W.windkessel(N=128, T=30)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    ll_kf, _ = orc.kf_wk(pb)
    R = 200
    lls = np.array([orc.pf_run_ex(dataclasses.replace(pb, seed=s), resampler=resampler,
                                  ess_frac=ess_frac)["loglik"] for s in range(R)])
    ratio = np.exp(lls - ll_kf)
    assert abs(ratio.mean() - 1.0) < 4 * ratio.std(ddof=1) / math.sqrt(R) + 1e-3


def test_multinomial_is_the_inverse_cdf_of_the_generator_uniforms(orc):
    for k in (0, 1, 5, 999):
        w = orc.philox([k >> 2, 3, (orc.TAG_MULTI << 28) | 1, 6], [2, 0])
        assert orc.multi_u(2, 3, 6, 1, k) == orc.u01(int(w[k & 3]))
    rng = np.random.default_rng(8)
    N = 500
    lw = rng.normal(size=N) * 2
    a = orc.multinomial_ancestors(lw, seed=2, t=3, b=6, it=1)
    w = np.exp(lw - lw.max())
    Wc = _seq_cumsum(w)
    u = np.array([orc.multi_u(2, 3, 6, 1, k) for k in range(N)])
    np.testing.assert_array_equal(a, np.minimum(np.searchsorted(Wc, u * Wc[-1], side="right"),
                                                N - 1))


@pytest.mark.parametrize("weights", [[0.3, 0.7], [0.9, 0.01, 0.01, 0.08], [1, 0, 0, 3, 0, 2, 2, 0]])
def test_multinomial_counts_are_multinomial(orc, weights):
    """Offspring counts: mean N w_j and the multinomial variance N w_j (1 - w_j)."""
    w = np.asarray(weights, dtype=np.float64)
    N = w.size
    with np.errstate(divide="ignore"):
        lw = np.log(w)
    R = 4000
    cnt = np.array([np.bincount(orc.multinomial_ancestors(lw, seed=9, t=t), minlength=N)
                    for t in range(1, R + 1)])
    p = w / w.sum()
    sd = np.sqrt(N * p * (1 - p))
    assert np.all(np.abs(cnt.mean(axis=0) - N * p) <= 4 * sd / math.sqrt(R) + 1e-9)
    v = cnt.var(axis=0, ddof=1)
    ok = p > 0
    assert np.all(np.abs(v[ok] - (N * p * (1 - p))[ok]) <= 0.15 * (N * p * (1 - p))[ok] + 1e-9)
    assert np.all(cnt[:, ~ok] == 0)


def test_multinomial_filter_unbiased_against_kalman(orc):
    pb = W.windkessel(N=128, T=30)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    ll_kf, _ = orc.kf_wk(pb)
    R = 200
    lls = np.array([orc.pf_run_ex(dataclasses.replace(pb, seed=s), resampler=3)["loglik"]
                    for s in range(R)])
    ratio = np.exp(lls - ll_kf)
    assert abs(ratio.mean() - 1.0) < 4 * ratio.std(ddof=1) / math.sqrt(R) + 1e-3


def test_rejection_limits(orc):
    N = 300
    np.testing.assert_array_equal(orc.rejection_ancestors(np.full(N, -3.5), 4, 2), np.arange(N))
    lw = np.full(N, -np.inf)
    lw[217] = 1.0
    np.testing.assert_array_equal(orc.rejection_ancestors(lw, 4, 2), np.full(N, 217))
    lw = np.zeros(N)
    lw[::3] = np.nan
    a = orc.rejection_ancestors(lw, 4, 2)
    assert np.all(a % 3 != 0)
    keep = np.arange(N) % 3 != 0
    np.testing.assert_array_equal(a[keep], np.arange(N)[keep])


def test_rejection_attempts_are_the_generator_words(orc):
    seed, t, b, it, N = 7, 13, 5, 3, 1000
    for k, r in [(0, 0), (4, 1), (9, 2), (9, 3), (31, 511), (31, 512), (2, 600), (77, 70001)]:
        p = r >> 1
        w = orc.philox([k, t + ((p >> 8) << 20), (orc.TAG_REJECT << 28) | ((p & 255) << 20) | it, b],
                       [seed, 0])
        h = r & 1
        j, u = orc.reject_pair(seed, t, b, it, k, r, N)
        assert j == (k if r == 0 else (int(w[2 * h]) * N) >> 32)
        assert u == orc.u01(int(w[2 * h + 1]))


@pytest.mark.parametrize("weights", [[0.3, 0.7], [5, 1, 1, 1, 1, 1], [0.9, 0.01, 0.01, 0.08],
                                     [1, 0, 0, 3, 0, 2]])
def test_rejection_output_law(orc, weights):
    """P(a_k = j) = [j = k] w_k/w_max + (1 - w_k/w_max) W_j, checked per output
    over many times; the offspring mean is then N W_j."""
    w = np.asarray(weights, dtype=np.float64)
    N = w.size
    with np.errstate(divide="ignore"):
        lw = np.log(w)
    R = 6000
    a = np.array([orc.rejection_ancestors(lw, seed=12, t=t, b=1) for t in range(1, R + 1)])
    Wn = w / w.sum()
    for k in range(N):
        p = (1.0 - w[k] / w.max()) * Wn
        p[k] += w[k] / w.max()
        f = np.bincount(a[:, k], minlength=N) / R
        sd = np.sqrt(p * (1 - p) / R)
        assert np.all(np.abs(f - p) <= 5 * sd + 1e-12), (k, f, p)
    cnt = np.array([np.bincount(r, minlength=N) for r in a])
    assert np.all(np.abs(cnt.mean(0) - N * Wn) <= 5 * cnt.std(0, ddof=1) / math.sqrt(R) + 1e-12)


def test_rejection_filter_unbiased_against_kalman(orc):
    pb = W.windkessel(N=128, T=30)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    ll_kf, _ = orc.kf_wk(pb)
    R = 200
    lls = np.array([orc.pf_run_ex(dataclasses.replace(pb, seed=s), resampler=4)["loglik"]
                    for s in range(R)])
    ratio = np.exp(lls - ll_kf)
    assert abs(ratio.mean() - 1.0) < 4 * ratio.std(ddof=1) / math.sqrt(R) + 1e-3
