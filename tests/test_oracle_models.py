"""Pins for the oracle's model arithmetic (transition and observation).

Windkessel: the noise-free exact step composed n times equals the closed
form a^n p0 + sum_m a^(n-1-m) c q_m (eq. 2-windkessel); the noise enters as
sigma_p times the generator's normal at substep n.
Lorenz '96: the quadratic term conserves energy (sum_i x_i A_i(x) = 0), a
hand-computed value at d=4, the uniform fixed point x = F, rotation
equivariance, and fourth-order convergence of one RK4 step against an
adaptive high-order solver.
Observation density: scipy's normal log-pdf.
"""
import dataclasses
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.stats

import workloads as W


def test_wk_noise_free_closed_form(orc):
    pb = W.windkessel(N=4, T=6, K=10)
    th = pb.theta[0].copy()
    th[3] = 0.0  # sigma_p
    a, c = th[0], th[1]
    x0 = np.array([[80.0, 90.0, 100.0, 120.0]])
    x = x0.copy()
    for t in range(1, pb.T + 1):
        x = orc.propagate(pb, th, x, t)
        n = t * pb.K
        ref = a ** n * x0[0] + sum(a ** (n - 1 - m) * c * pb.q[m] for m in range(n))
        np.testing.assert_allclose(x[0], ref, rtol=1e-12)


def test_wk_noise_enters_at_substep_n(orc):
    pb = W.windkessel(N=3, T=2, K=10, seed=11)
    th = pb.theta[0]
    a, c, sp = th[0], th[1], th[3]
    x0 = np.array([[90.0, 91.0, 92.0]])
    th0 = th.copy(); th0[3] = 0.0
    x_free = orc.propagate(pb, th0, x0, 2)
    x = orc.propagate(pb, th, x0, 2)
    n0, n1 = pb.K + 1, 2 * pb.K
    for j in range(3):
        noise = sum(a ** (n1 - n) * sp * orc.normals4(pb.seed, orc.TAG_NOISE, 0, 0, j, n, 0)[0]
                    for n in range(n0, n1 + 1))
        assert x[0, j] - x_free[0, j] == pytest.approx(noise, abs=1e-11)


def test_l96_drift_hand_value_and_energy(orc):
    # d = 4: f_0 = (x1 - x2) x3 - x0 + F = (2-3)*4 - 1 + 8 = 3
    f = orc.l96_drift(np.array([1.0, 2.0, 3.0, 4.0]), 8.0)
    # f_1 = (x2 - x3) x0 - x1 + F = (3-4)*1 - 2 + 8 = 5
    # f_2 = (x3 - x0) x1 - x2 + F = (4-1)*2 - 3 + 8 = 11
    # f_3 = (x0 - x1) x2 - x3 + F = (1-2)*3 - 4 + 8 = 1
    assert list(f) == [3.0, 5.0, 11.0, 1.0]
    rng = np.random.default_rng(0)
    for d in (5, 8, 40):
        x = rng.normal(size=d) * 3
        F = 8.0
        adv = orc.l96_drift(x, F) + x - F   # the quadratic (advection) part
        assert abs(np.dot(x, adv)) < 1e-12 * np.dot(np.abs(x), np.abs(adv)) * d


def test_l96_fixed_point_and_rotation(orc):
    pb = W.lorenz96(d=8, N=5, T=3)
    th = np.array([8.0, 0.0])
    x = np.full((8, 5), 8.0)
    for t in range(1, 4):
        x = orc.propagate(pb, th, x, t)
    assert np.all(x == 8.0)
    rng = np.random.default_rng(1)
    x0 = rng.normal(size=(8, 5)) * 2
    out = orc.propagate(pb, th, x0, 1)
    out_rot = orc.propagate(pb, th, np.roll(x0, 3, axis=0), 1)
    assert np.array_equal(np.roll(out, 3, axis=0), out_rot)


def test_l96_noise_after_rk4(orc):
    """From the fixed point, one substep gives F + sigma*sqrt(h)*z exactly."""
    pb = dataclasses.replace(W.lorenz96(d=8, N=3, T=1, seed=5), K=1)
    th = np.array([8.0, 0.1])
    x = orc.propagate(pb, th, np.full((8, 3), 8.0), 1)
    sq = 0.1 * math.sqrt(pb.h)
    for j in range(3):
        z = np.concatenate([orc.normals4(5, orc.TAG_NOISE, blk, 0, j, 1, 0) for blk in range(2)])
        np.testing.assert_array_equal(x[:, j], 8.0 + sq * z)


def test_l96_rk4_fourth_order(orc):
    d = 8
    F = 8.0
    x0 = np.random.default_rng(3).normal(size=d) * 2 + 1

    def rhs(_, x):
        return (np.roll(x, -1) - np.roll(x, 2)) * np.roll(x, 1) - x + F

    errs = []
    for h in (0.05, 0.025, 0.0125):
        pb = dataclasses.replace(W.lorenz96(d=d, N=1, T=1), K=1, h=h)
        got = orc.propagate(pb, np.array([F, 0.0]), x0[:, None], 1)[:, 0]
        ref = scipy.integrate.solve_ivp(rhs, (0, h), x0, method="DOP853", rtol=1e-13,
                                        atol=1e-13).y[:, -1]
        errs.append(np.abs(got - ref).max())
    # local error of a fourth-order method scales as h^5
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 20 < r1 < 45 and 20 < r2 < 45, errs


def test_observation_logdensity(orc):
    rng = np.random.default_rng(4)
    pb = W.lorenz96(d=40, N=64, T=3, obs_every=2).with_obs(rng.normal(size=(3, 20)))
    x = rng.normal(size=(40, 64)) * 2
    lw = orc.weight(pb, pb.theta[0], x, 2)
    ref = scipy.stats.norm.logpdf(pb.obs[1][:, None], loc=x[pb.obs_idx], scale=0.5).sum(0)
    np.testing.assert_allclose(lw, ref, rtol=1e-13)
    wk = W.windkessel(N=16, T=3).with_obs(np.array([[95.0], [101.0], [99.0]]))
    p = rng.normal(90, 10, size=(1, 16))
    lw = orc.weight(wk, wk.theta[0], p, 3)
    mu = p[0] + wk.theta[0][2] * wk.q[3 * wk.K]
    np.testing.assert_allclose(lw, scipy.stats.norm.logpdf(99.0, loc=mu, scale=1.0), rtol=1e-13)


def test_simulated_observation_noise(orc):
    pb = W.lorenz96(d=40, N=1, T=500, obs_every=2)
    xt, y = orc.simulate(pb)
    r = (y - xt[1:, pb.obs_idx]) / pb.obs_sd
    n = r.size
    assert abs(r.mean()) < 4 / math.sqrt(n)
    assert abs(r.var() - 1) < 4 * math.sqrt(2 / n)
    assert np.abs(xt).max() < 20  # bounded chaotic attractor


# ---------------------------------------------------------------- the paper's model forms

def test_l96_stage_noise_reduces_without_noise(orc):
    """sigma = 0: the in-stage form is the plain RK4 step, bit for bit."""
    for stage in (False, True):
        pb = W.lorenz96(d=8, N=5, T=3, sigma=0.0, stage_noise=stage)
        x0 = orc.init(pb, pb.theta[0], 5)
        x = x0
        for t in range(1, 4):
            x = orc.propagate(pb, pb.theta[0], x, t)
        if not stage:
            ref = x
    np.testing.assert_array_equal(x, ref)


def test_l96_stage_noise_is_the_rk4_propagator_of_the_forcing(orc):
    """At the uniform fixed point x = F with a tiny sigma the step is linear
    in the noise: constant forcing c = sq z / h over the step gives, under
    RK4, h (I + hJ/2 + (hJ)^2/6 + (hJ)^3/24) c with J the drift's Jacobian
    at x = F (J_{i,i+1} = F, J_{i,i-2} = -F, J_ii = -1).  The noise added
    after the step instead gives sq z exactly."""
    d, F, sig = 8, 8.0, 1e-6
    for stage in (True, False):
        pb = W.lorenz96(d=d, N=1, T=1, K=1, F=F, sigma=sig, stage_noise=stage)
        x = orc.propagate(pb, pb.theta[0], np.full((d, 1), F), 1)[:, 0] - F
        z = np.concatenate([orc.normals4(pb.seed, orc.TAG_NOISE, blk, 0, 0, 1, 0)
                            for blk in range(d // 4)])
        sq = sig * math.sqrt(pb.h)
        if stage:
            J = -np.eye(d)
            for i in range(d):
                J[i, (i + 1) % d] += F
                J[i, (i - 2) % d] -= F
            A = pb.h * J
            P = np.eye(d) + A / 2 + A @ A / 6 + A @ A @ A / 24
            np.testing.assert_allclose(x, sq * (P @ z), rtol=1e-5, atol=1e-14)
        else:
            np.testing.assert_allclose(x, sq * z, rtol=1e-6, atol=1e-14)


def test_paper_windkessel_inputs(orc):
    pb = W.windkessel_paper(N=64, T=80)
    q = pb.q
    t = np.arange(q.size) * pb.h
    # systole: the sin^2 pulse (period 0.8 s, as printed) up to 0.3 s of every
    # period, zero after; it is cut at 500 sin^2(0.375 pi) before its peak
    np.testing.assert_allclose(q[30], 500.0 * math.sin(0.375 * math.pi) ** 2, rtol=1e-12)
    assert q.max() == q[30]
    assert np.all(q[(np.mod(t, 0.8) > 0.3 + 1e-9)] == 0.0)
    assert np.all(q[(np.mod(t, 0.8) > 1e-9) & (np.mod(t, 0.8) < 0.3 - 1e-9)] > 0.0)
    # flow noise of variance sigma^2 is pressure noise of sd c sigma
    a, c, Z, sp, m0, s0 = pb.theta[0]
    assert sp == pytest.approx(c * 5.0, rel=1e-15)
    assert pb.obs_sd == 2.0 and (m0, s0) == (90.0, 15.0)
    # the Kalman filter and the particle filter agree on it (unbiasedness)
    _, y = orc.simulate(pb)
    pb = pb.with_obs(y)
    ll_kf, _ = orc.kf_wk(pb)
    lls = np.array([orc.pf_run(dataclasses.replace(pb, seed=s))["loglik"] for s in range(60)])
    assert abs(lls.mean() + lls.var(ddof=1) / 2 - ll_kf) < 4 * lls.std(ddof=1) / math.sqrt(60) + 0.02
