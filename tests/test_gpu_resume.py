"""Checkpoint and resume through the C ABI (pf_restore).  The filter is
defined over an interval so that it can restart from its own output
(Sec. 3.1.2), and the generator is positional, so T intervals in one run
and T/2 intervals, a checkpoint (pf_get_state, pf_loglik), pf_restore on a
fresh handle and T/2 more must give the same bits: likelihoods, trace rows
and final particles, in every layout and precision, eager and replayed from
graphs."""
import dataclasses

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


def _batched_problem(T=12):
    base = W.lorenz96(d=8, N=1, T=T)
    _, y = oracle.simulate(base)
    n = [300, 1000, 4100, 256, 8192]
    th = [[8.0, 0.1], [8.5, 0.2], [7.5, 0.15], [8.0, 0.3], [9.0, 0.1]]
    return dataclasses.replace(base.with_obs(y), theta=np.asarray(th, dtype=np.float64),
                               n_particles=np.asarray(n, dtype=np.int64))


def _plain_problem(T=12):
    pb = W.lorenz96(d=8, N=5000, T=T)
    _, y = oracle.simulate(pb)
    return pb.with_obs(y)


CASES = [("plain", "PF_FP64"), ("plain", "PF_FP32_MIXED"), ("batched", "PF_FP64"),
         ("batched", "PF_FP32_ACCURATE"), ("batched", "PF_FP32_MIXED")]


def _run(pfm, f, n, graph):
    if graph:
        f.graph_run(n)
    else:
        f.advance(n)


@pytest.mark.parametrize("layout,prec", CASES)
@pytest.mark.parametrize("graph", [False, True])
def test_resume_is_the_whole_run(pfm, layout, prec, graph):
    pb = _plain_problem() if layout == "plain" else _batched_problem()
    kw = dict(precision=getattr(pfm, prec),
              layout=pfm.PF_LAYOUT_PLAIN if layout == "plain" else pfm.PF_LAYOUT_BATCHED)
    T, s = pb.T, pb.T // 2
    a = pfm.Filter(pb, **kw)
    _run(pfm, a, T, graph)
    ll_a, _, _ = a.loglik()
    ell_a, ess_a = a.trace()
    x_a = a.get_state()
    a.close()
    b = pfm.Filter(pb, **kw)
    _run(pfm, b, s, graph)
    ll_s, _, t_s = b.loglik()
    assert t_s == s
    x_s = b.get_state()
    b.close()
    c = pfm.Filter(pb, **kw)
    c.restore(s, x_s, ll_s)
    assert c.loglik()[2] == s
    _run(pfm, c, T - s, graph)
    ll_c, _, t_c = c.loglik()
    ell_c, ess_c = c.trace()
    assert t_c == T
    np.testing.assert_array_equal(ll_c, ll_a)
    np.testing.assert_array_equal(ell_c[:, s:], ell_a[:, s:])
    np.testing.assert_array_equal(ess_c[:, s:], ess_a[:, s:])
    assert np.all(ell_c[:, :s] == 0.0)
    np.testing.assert_array_equal(c.get_state(), x_a)
    # the same handle, rewound to its own checkpoint, replays the second half
    c.restore(s, x_s, ll_s)
    _run(pfm, c, T - s, not graph)
    np.testing.assert_array_equal(c.loglik()[0], ll_a)
    np.testing.assert_array_equal(c.get_state(), x_a)
    c.close()


def test_resume_matches_the_oracle(pfm):
    """The restored FP64 plain filter against the oracle run over the whole
    horizon (every particle and increment equal, as for a fresh run)."""
    pb = _plain_problem(T=10)
    ref = oracle.pf_run(pb, traces=True)
    f = pfm.Filter(pb, precision=pfm.PF_FP64)
    f.advance(4)
    x, ll = f.get_state(), f.loglik()[0]
    f.close()
    g = pfm.Filter(pb, precision=pfm.PF_FP64)
    g.restore(4, x, ll)
    g.advance(6)
    ell, _ = g.trace()
    assert np.max(np.abs(ell[0, 4:] - ref["ell"][4:]) / np.abs(ref["ell"][4:])) <= 1e-10
    assert abs(g.loglik()[0][0] - ref["loglik"]) <= 1e-10 * abs(ref["loglik"])
    g.close()


def test_restore_edges_and_errors(pfm):
    pb = _batched_problem(T=6)
    f = pfm.Filter(pb, precision=pfm.PF_FP64, layout=pfm.PF_LAYOUT_BATCHED)
    x0 = f.get_state()
    ll0 = np.zeros(pb.B)
    # t = T: nothing left to run; t = 0: a given initial set
    f.restore(pb.T, x0, ll0)
    assert f.loglik()[2] == pb.T
    with pytest.raises(pfm.PfError):
        f.step()
    f.restore(0, x0, ll0)
    f.advance(pb.T)
    assert f.loglik()[2] == pb.T
    for bad_t in (-1, pb.T + 1):
        with pytest.raises(pfm.PfError):
            f.restore(bad_t, x0, ll0)
    for bad_ll in (np.nan, np.inf):
        with pytest.raises(pfm.PfError):
            f.restore(1, x0, np.full(pb.B, bad_ll))
    # -infinity: the filter carries the numeric flag
    ll = ll0.copy()
    ll[2] = -np.inf
    f.restore(1, x0, ll)
    with pytest.raises(pfm.PfError):
        f.loglik()
    out, _, _ = f.loglik(allow_numeric=True)
    assert out[2] == -np.inf and np.all(np.isfinite(np.delete(out, 2)))
    # only between intervals
    f.restore(1, x0, ll0)
    f.step()
    with pytest.raises(pfm.PfError):
        f.restore(1, x0, ll0)
    f.resample()
    f.close()
    # not with a history attached
    h = pfm.Filter(pb, precision=pfm.PF_FP64, layout=pfm.PF_LAYOUT_BATCHED)
    h.attach_history()
    with pytest.raises(pfm.PfError, match="history"):
        h.restore(1, x0, ll0)
    h.close()
