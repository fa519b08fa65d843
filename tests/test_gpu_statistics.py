"""Statistical checks of the HIP path at sizes the oracle cannot follow step
by step, pinned to results independent of the oracle's filter code.

* On the linear-Gaussian windkessel model the Kalman filter gives the exact
  log-likelihood (Alg. 1, reduced to one dimension); the particle estimate of
  the likelihood is unbiased, so over independent seeds the GPU filter's
  log-likelihoods centre on it (minus half their variance), FP64 and FP32.
* On chaotic Lorenz '96 a free-running FP32 filter decorrelates from the
  FP64 one, so the two are compared over seeds: the paired differences of
  their log-likelihoods must have mean zero within sampling error.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pfm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_3277_amd as pfm
    pfm.load()
    return pfm


def _logliks(pfm, pb, precision, seeds):
    out = []
    for s in seeds:
        f = pfm.Filter(pb, precision=precision, seed=int(s))
        f.graph_run(pb.T)
        out.append(f.loglik()[0][0])
        f.close()
    return np.array(out)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_windkessel_large_filter_centres_on_kalman(pfm, precision):
    pb = W.windkessel(N=1 << 18, T=100)
    _, y = oracle.simulate(pb)
    pb = pb.with_obs(y)
    ll_kf, _ = oracle.kf_wk(pb)
    prec = pfm.PF_FP64 if precision == "fp64" else pfm.PF_FP32_MIXED
    ll = _logliks(pfm, pb, prec, range(100, 112))
    R = ll.size
    sd = ll.std(ddof=1)
    # E[exp(ll)] = exp(ll_kf): the mean of ll sits var/2 below ll_kf
    centre = ll.mean() + 0.5 * sd ** 2
    assert abs(centre - ll_kf) <= 4.0 * sd / np.sqrt(R) + 2e-3, (centre, ll_kf, sd)
    assert sd < 0.5  # 2^18 particles on a 1-D linear model: a tight estimate


def test_lorenz96_fp32_free_running_matches_fp64_over_seeds(pfm):
    pb = W.lorenz96(d=8, N=4096, T=30)
    _, y = oracle.simulate(pb)
    pb = pb.with_obs(y)
    seeds = range(200, 224)
    ll64 = _logliks(pfm, pb, pfm.PF_FP64, seeds)
    ll32 = _logliks(pfm, pb, pfm.PF_FP32_MIXED, seeds)
    d = ll32 - ll64
    R = d.size
    assert np.all(np.isfinite(d))
    assert abs(d.mean()) <= 3.0 * d.std(ddof=1) / np.sqrt(R) + 1e-3, (d.mean(), d.std(ddof=1))
