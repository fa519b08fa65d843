"""Pins for the oracle's single state sample of the bootstrap filter (the last
lines of Alg. 2: one particle drawn from the final weights and traced back
through its ancestry), against things other than that code:

* with one particle the sample is that particle's trajectory, rebuilt from
  the initialisation and propagation pieces;
* the sampled indices follow the ancestors the filter run records, and the
  sampled states are the propagated particles at those indices, rebuilt
  from the pieces;
* the final slot is uniform over the particles (chi-square);
* on the linear-Gaussian windkessel model the sample's mean at every time
  matches the Rauch-Tung-Striebel smoother mean (textbook Kalman smoother,
  written here in numpy), which differs from the filtering mean by far more
  than the tolerance.
"""
import dataclasses
import math

import numpy as np
import pytest
import scipy.stats

import workloads as W


def _with_data(orc, pb):
    _, y = orc.simulate(pb)
    return pb.with_obs(y)


@pytest.mark.parametrize("model", ["l96", "wk"])
def test_single_particle_path_is_its_trajectory(orc, model):
    pb = _with_data(orc, W.lorenz96(d=8, N=1, T=6) if model == "l96" else W.windkessel(N=1, T=6))
    st, ll, path, idx = orc.pf_path(pb, N=1)
    assert np.all(idx == 0)
    x = orc.init(pb, pb.theta[0], 1)
    np.testing.assert_array_equal(path[0], x[:, 0])
    for t in range(1, pb.T + 1):
        x = orc.propagate(pb, pb.theta[0], x, t)
        np.testing.assert_array_equal(path[t], x[:, 0])


@pytest.mark.parametrize("N,T", [(37, 5), (200, 8)])
def test_path_follows_the_recorded_ancestry(orc, N, T):
    pb = _with_data(orc, W.lorenz96(d=8, N=N, T=T))
    st, ll, path, idx = orc.pf_path(pb, b=0, it=3)
    ref = orc.pf_run(pb, N=N, b=0, it=3, traces=True)
    assert ll == ref["loglik"]
    anc = ref["anc"]
    k = orc.path_slot(pb.seed, T, 0, 3, N)
    assert idx[T] == anc[T - 1][k]
    for i in range(T, 1, -1):
        assert idx[i - 1] == anc[i - 2][idx[i]]
    assert idx[0] == idx[1]
    # propagated particles per time, rebuilt from the pieces
    x = orc.init(pb, pb.theta[0], N, b=0, it=3)
    np.testing.assert_array_equal(path[0], x[:, idx[0]])
    for t in range(1, T + 1):
        xp = orc.propagate(pb, pb.theta[0], x, t, b=0, it=3)
        np.testing.assert_array_equal(path[t], xp[:, idx[t]])
        x = orc.gather(xp, anc[t - 1])


def test_path_slot_is_uniform(orc):
    N = 10
    ks = np.array([orc.path_slot(7, s, b, 0, N) for s in range(1, 201) for b in range(25)])
    assert ks.min() >= 0 and ks.max() < N
    cnt = np.bincount(ks, minlength=N)
    assert scipy.stats.chisquare(cnt).pvalue > 1e-3


def _wk_rts(pb):
    """Kalman filter and Rauch-Tung-Striebel smoother of the windkessel
    pressure at the observation times t_0..t_T (the interval transition is
    linear: p_i = a^K p_{i-1} + u_i + noise of variance sigma_p^2 sum a^2s)."""
    a, c, Z, sp, m0, s0 = pb.theta[0]
    K, T, q, y = pb.K, pb.T, pb.q, pb.obs[:, 0]
    A = a ** K
    Q = sp ** 2 * sum(a ** (2 * s) for s in range(K))
    mf, Pf, mp, Pp = np.zeros(T + 1), np.zeros(T + 1), np.zeros(T + 1), np.zeros(T + 1)
    mf[0], Pf[0] = m0, s0 ** 2
    for i in range(1, T + 1):
        u = sum(a ** (K - s) * c * q[(i - 1) * K + s - 1] for s in range(1, K + 1))
        mp[i], Pp[i] = A * mf[i - 1] + u, A * A * Pf[i - 1] + Q
        S = Pp[i] + pb.obs_sd ** 2
        G = Pp[i] / S
        mf[i] = mp[i] + G * (y[i - 1] - Z * q[i * K] - mp[i])
        Pf[i] = (1 - G) * Pp[i]
    ms, Ps = mf.copy(), Pf.copy()
    for i in range(T - 1, -1, -1):
        J = Pf[i] * A / Pp[i + 1]
        ms[i] = mf[i] + J * (ms[i + 1] - mp[i + 1])
        Ps[i] = Pf[i] + J * J * (Ps[i + 1] - Pp[i + 1])
    return ms, Ps, mf


def test_windkessel_path_mean_is_the_smoother_mean(orc):
    base = W.windkessel(N=256, T=10)
    th = base.theta.copy()
    th[:, 5] = 5.0  # a tighter initial law: filtering and smoothing means differ clearly
    base = dataclasses.replace(base, theta=th, data_theta=th[0].copy())
    pb = _with_data(orc, base)
    ms, Ps, mf = _wk_rts(pb)
    R = 120
    paths = np.array([orc.pf_path(dataclasses.replace(pb, seed=500 + r))[2][:, 0]
                      for r in range(R)])
    tol = 4.0 * np.sqrt(Ps / R) + 0.05
    assert np.all(np.abs(paths.mean(axis=0) - ms) <= tol), (paths.mean(axis=0) - ms, tol)
    # the check discriminates: a filtering (not traced-back) sample would fail it
    assert np.any(np.abs(mf - ms) > 2 * tol)
    # and the spread matches the smoother's
    sd = paths.std(axis=0, ddof=1)
    assert np.all(sd < 1.5 * np.sqrt(Ps) + 0.1) and np.all(sd > 0.6 * np.sqrt(Ps) - 0.1)
