"""GPU parity of SMC over the parameters with attached particle filters
(SMC^2, Sec. 3.2.2, Alg. 4) against the oracle, through the C ABI.

FP64, small sizes the oracle finishes in seconds: theta-ancestors, accept
decisions and theta-particles bit for bit (the theta-resampling compares
FP64 sums taken in a different order, so a flip within 1e-9 of a stratum
boundary would be legitimate; the cases below have none), likelihood
increments, likelihoods and the evidence within 1e-10 relative, the final
particles bit for bit.  At larger sizes, FP64 and FP32, the evidence on the
windkessel model centres on the Kalman integral over the prior.
"""
import dataclasses
import math

import numpy as np
import pytest
import scipy.special

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

REL64 = 1e-10


@pytest.fixture(scope="module")
def pfm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_3277_amd as pfm
    pfm.load()
    return pfm


def _run_gpu(pfm, pb, inp, precision):
    f = pfm.Filter(pb, precision=precision, layout=pfm.PF_LAYOUT_BATCHED)
    p = pfm.Filter(pb, precision=precision, layout=pfm.PF_LAYOUT_BATCHED)
    r = f.smc2(p, inp)
    r["x"] = f.get_state()
    t = f.loglik(allow_numeric=True)[2]
    f.close()
    p.close()
    return r, t


def _band_free(ref, B):
    """True if no theta-resampling threshold lies within 1e-9 of a scan point."""
    for i in range(2, ref["anc"].shape[0] + 1):
        v = ref["logw_trace"][i - 2]
        w = np.exp(v - v.max())
        cw = np.cumsum(w) / w.sum()
        for k in range(B):
            if np.min(np.abs(cw - (ref["u"][i - 1] + k) / B)) < 1e-9:
                return False
    return True


def _compare(pfm, pb, inp, ref, r):
    B = pb.B
    ref = dict(ref, u=inp.u)
    assert _band_free(ref, B)
    np.testing.assert_array_equal(r["anc"], ref["anc"])
    np.testing.assert_array_equal(r["acc"], ref["acc"])
    np.testing.assert_array_equal(r["accepts"], ref["accepts"])
    np.testing.assert_array_equal(r["theta_trace"], ref["theta_trace"])
    np.testing.assert_array_equal(r["theta"], ref["theta"])
    np.testing.assert_array_less(np.abs(r["logw_trace"] - ref["logw_trace"]),
                                 REL64 * np.maximum(1.0, np.abs(ref["logw_trace"])))
    np.testing.assert_array_less(np.abs(r["loglik"] - ref["loglik"]),
                                 REL64 * np.maximum(1.0, np.abs(ref["loglik"])))
    assert abs(r["log_evidence"] - ref["log_evidence"]) <= REL64 * max(1.0, abs(ref["log_evidence"]))
    np.testing.assert_allclose(r["ess"], ref["ess"], rtol=1e-9)
    np.testing.assert_array_equal(r["x"], ref["x"])


@pytest.mark.parametrize("accept", ["draw", "all", "none"])
def test_smc2_lorenz96_uneven_fp64_matches_oracle(pfm, accept):
    base = W.lorenz96(d=8, N=1, T=6)
    _, y = oracle.simulate(base)
    th0, _ = W.batched_thetas(6, seed=31)
    n = np.array([64, 100, 128, 50, 256, 33], dtype=np.int64)
    pb = dataclasses.replace(base.with_obs(y), theta=th0, n_particles=n)
    inp = W.smc2_l96_inputs(th0, pb.T, seed=9, step_f=0.3, step_s=0.03)
    if accept != "draw":
        fill = -np.inf if accept == "all" else np.inf
        inp = dataclasses.replace(inp, log_alpha=np.full_like(inp.log_alpha, fill))
    ref = oracle.smc2(pb, inp)
    r, t = _run_gpu(pfm, pb, inp, pfm.PF_FP64)
    assert t == pb.T and r["status"] == 0
    _compare(pfm, pb, inp, ref, r)
    if accept == "all":
        assert r["acc"].sum() > 0


def test_smc2_windkessel_fp64_matches_oracle(pfm):
    base = W.windkessel(N=100, T=8, B=8)
    th = base.theta.copy()
    th[:, 5] = 3.0
    base = dataclasses.replace(base, theta=th, data_theta=th[0].copy())
    _, y = oracle.simulate(base)
    pb = base.with_obs(y)
    inp = W.smc2_wk_m0_inputs(th[0], pb.B, pb.T, seed=12)
    pb = dataclasses.replace(pb, theta=inp.theta0)
    ref = oracle.smc2(pb, inp)
    r, _ = _run_gpu(pfm, pb, inp, pfm.PF_FP64)
    _compare(pfm, pb, inp, ref, r)


def test_smc2_shorter_run_than_the_handle(pfm):
    """T_run < T: the run stops after T_run times and matches the oracle's."""
    base = W.lorenz96(d=8, N=1, T=7)
    _, y = oracle.simulate(base)
    th0, _ = W.batched_thetas(4, seed=41)
    n = np.array([80, 80, 80, 80], dtype=np.int64)
    pb = dataclasses.replace(base.with_obs(y), theta=th0, n_particles=n)
    inp = W.smc2_l96_inputs(th0, 4, seed=13)
    ref = oracle.smc2(pb, inp)
    r, t = _run_gpu(pfm, pb, inp, pfm.PF_FP64)
    assert t == 4
    _compare(pfm, pb, inp, ref, r)


def _kalman_evidence_over_m0(pb, lo, hi, n=1601):
    grid = np.linspace(lo, hi, n)
    ll = np.empty(n)
    for g, m0 in enumerate(grid):
        th = pb.theta[0].copy()
        th[4] = m0
        ll[g], _ = oracle.kf_wk(pb, th)
    wq = np.full(n, (hi - lo) / (n - 1))
    wq[0] *= 0.5
    wq[-1] *= 0.5
    return scipy.special.logsumexp(ll, b=wq / (hi - lo))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_smc2_windkessel_evidence_centres_on_kalman_integral(pfm, precision):
    B, N, T, R = 64, 512, 20, 12
    base = W.windkessel(N=N, T=T, B=B)
    th = base.theta.copy()
    th[:, 5] = 3.0
    base = dataclasses.replace(base, theta=th, data_theta=th[0].copy())
    _, y = oracle.simulate(base)
    base = base.with_obs(y)
    log_z = _kalman_evidence_over_m0(base, 70.0, 110.0)
    prec = pfm.PF_FP64 if precision == "fp64" else pfm.PF_FP32_MIXED
    ev = []
    for rep in range(R):
        pb = dataclasses.replace(base, seed=300 + rep)
        inp = W.smc2_wk_m0_inputs(th[0], B, T, seed=400 + rep)
        pb = dataclasses.replace(pb, theta=inp.theta0)
        r, _ = _run_gpu(pfm, pb, inp, prec)
        assert r["status"] == 0
        ev.append(r["log_evidence"])
    ev = np.array(ev)
    sd = ev.std(ddof=1)
    centre = ev.mean() + 0.5 * sd ** 2
    assert abs(centre - log_z) <= 4.0 * sd / math.sqrt(R) + 0.02, (centre, log_z, sd)
    assert sd < 0.5


def test_smc2_rejects_mismatched_proposal_handle(pfm):
    base = W.lorenz96(d=8, N=1, T=3)
    pb = dataclasses.replace(base.with_obs(np.zeros((3, 8))), theta=np.array([[8.0, 0.1]] * 2),
                             n_particles=np.array([64, 64], dtype=np.int64))
    other = dataclasses.replace(pb, n_particles=np.array([64, 65], dtype=np.int64))
    f = pfm.Filter(pb, layout=pfm.PF_LAYOUT_BATCHED)
    p = pfm.Filter(other, layout=pfm.PF_LAYOUT_BATCHED)
    inp = W.smc2_l96_inputs(pb.theta, 3)
    with pytest.raises(pfm.PfError):
        f.smc2(p, inp)
    with pytest.raises(pfm.PfError):
        f.smc2(f, inp)
    f.close()
    p.close()
