"""GPU parity of the bootstrap filter's single state sample (Alg. 2, last
lines: ancestry storage, final draw, backtrace) with the oracle, through the
C ABI: particle indices and FP64 paths bit for bit, plain and batched
layouts, eager and graph-replayed intervals; FP32 batched equals FP32 plain
(the same propagation arithmetic)."""
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


def _data(pb):
    _, y = oracle.simulate(pb)
    return pb.with_obs(y)


def _run(pfm, pb, precision, layout, graph, T=None):
    T = pb.T if T is None else T
    f = pfm.Filter(pb, precision=precision, layout=layout)
    f.attach_history()
    if graph:
        f.graph_run(T)
    else:
        f.advance(T)
    path, idx = f.backtrace()
    f.close()
    return path, idx


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("model", ["l96", "wk"])
def test_plain_fp64_path_matches_oracle(pfm, model, graph):
    pb = _data(W.lorenz96(d=8, N=300, T=6) if model == "l96" else W.windkessel(N=500, T=9))
    path, idx = _run(pfm, pb, pfm.PF_FP64, pfm.PF_LAYOUT_PLAIN, graph)
    st, ll, rpath, ridx = oracle.pf_path(pb)
    np.testing.assert_array_equal(idx[0], ridx)
    np.testing.assert_array_equal(path[0], rpath)


@pytest.mark.parametrize("graph", [False, True])
def test_batched_fp64_path_matches_oracle(pfm, graph):
    base = _data(W.lorenz96(d=8, N=1, T=7))
    th0, _ = W.batched_thetas(4, seed=51)
    n = np.array([257, 64, 1000, 33], dtype=np.int64)
    pb = dataclasses.replace(base, theta=th0, n_particles=n)
    path, idx = _run(pfm, pb, pfm.PF_FP64, pfm.PF_LAYOUT_BATCHED, graph)
    for b in range(pb.B):
        st, ll, rpath, ridx = oracle.pf_path(pb, theta=th0[b], N=int(n[b]), b=b)
        np.testing.assert_array_equal(idx[b], ridx, err_msg=f"filter {b}")
        np.testing.assert_array_equal(path[b], rpath, err_msg=f"filter {b}")


def test_path_before_the_end_and_at_t0(pfm):
    pb = _data(W.lorenz96(d=8, N=128, T=8))
    for T in (0, 3):
        f = pfm.Filter(pb, precision=pfm.PF_FP64)
        f.attach_history()
        f.advance(T)
        path, idx = f.backtrace()
        f.close()
        st, ll, rpath, ridx = oracle.pf_path(pb, T=T)
        assert path.shape == (1, T + 1, 8)
        np.testing.assert_array_equal(idx[0], ridx)
        np.testing.assert_array_equal(path[0], rpath)


def test_reset_records_the_new_run(pfm):
    pb = _data(W.lorenz96(d=8, N=200, T=5))
    f = pfm.Filter(pb, precision=pfm.PF_FP64, layout=pfm.PF_LAYOUT_BATCHED)
    f.attach_history()
    f.graph_run(5)
    f.reset(7)
    f.graph_run(4)
    path, idx = f.backtrace()
    f.close()
    st, ll, rpath, ridx = oracle.pf_path(pb, it=7, T=4)
    np.testing.assert_array_equal(idx[0], ridx)
    np.testing.assert_array_equal(path[0], rpath)


def test_fp32_batched_path_equals_fp32_plain(pfm):
    base = _data(W.lorenz96(d=8, N=1, T=6, precision=W.FP32_MIXED))
    th0, _ = W.batched_thetas(3, seed=52)
    n = np.array([300, 1024, 77], dtype=np.int64)
    pb = dataclasses.replace(base, theta=th0, n_particles=n)
    p1, i1 = _run(pfm, pb, pfm.PF_FP32_MIXED, pfm.PF_LAYOUT_PLAIN, True)
    p2, i2 = _run(pfm, pb, pfm.PF_FP32_MIXED, pfm.PF_LAYOUT_BATCHED, True)
    np.testing.assert_array_equal(i2, i1)
    np.testing.assert_array_equal(p2, p1)


def test_history_rules(pfm):
    pb = _data(W.lorenz96(d=8, N=64, T=3))
    pb2 = dataclasses.replace(pb, theta=np.array([[8.0, 0.1], [7.0, 0.2]]),
                              n_particles=np.array([64, 64], dtype=np.int64))
    f = pfm.Filter(pb2, layout=pfm.PF_LAYOUT_BATCHED)
    with pytest.raises(pfm.PfError):
        f.backtrace()  # nothing attached
    f.attach_history()
    p = pfm.Filter(pb2, layout=pfm.PF_LAYOUT_BATCHED)
    with pytest.raises(pfm.PfError):
        f.smc2(p, W.smc2_l96_inputs(pb2.theta, 3))
    f.step()
    with pytest.raises(pfm.PfError):
        f.attach_history()  # only at t = 0
    f.close()
    p.close()


def _history_arrays(f, pb, fp64):
    """The attached history as (particles [T+1][d][N_total], ancestors
    [T][N_total]), laid out as pf.h states (each part 256-byte aligned)."""
    import torch
    torch.cuda.synchronize()
    raw = f.history.cpu().numpy()
    start = ((f.history.data_ptr() + 255) & ~255) - f.history.data_ptr()
    n = int(pb.n_particles.sum())
    sx = 8 if fp64 else 4
    nx = sx * (pb.T + 1) * pb.d * n
    xh = raw[start:start + nx].view(np.float64 if fp64 else np.float32)
    a0 = start + (nx + 255) // 256 * 256
    ah = raw[a0:a0 + 4 * pb.T * n].view(np.int32)
    return xh.reshape(pb.T + 1, pb.d, n), ah.reshape(pb.T, n)


@pytest.mark.parametrize("fp64,scheme,steps,ess_frac",
                         [(True, 0, 0, float("inf")), (False, 0, 0, float("inf")),
                          (True, 1, 0, 0.7), (True, 2, 5, float("inf")), (True, 3, 0, 0.7)])
def test_batched_history_holds_every_slot(pfm, fp64, scheme, steps, ess_frac):
    """Every slot of a batched history equals the state and ancestors the
    inspection calls read after each step and resampling (one group, eager),
    and a graph-replayed run in three filter groups records the same bytes;
    for every resampler (the collective stores the ancestor slots in each of
    its variants) and with the ESS trigger."""
    precision = pfm.PF_FP64 if fp64 else pfm.PF_FP32_MIXED
    base = _data(W.lorenz96(d=8, N=1, T=6, precision=precision))
    th0, _ = W.batched_thetas(5, seed=53)
    n = np.array([300, 64, 1000, 33, 257], dtype=np.int64)
    pb = dataclasses.replace(base, theta=th0, n_particles=n)
    f = pfm.Filter(pb, precision=precision, layout=pfm.PF_LAYOUT_BATCHED)
    f.set_resampler(scheme, steps, ess_frac)
    f.attach_history()
    xs = [f.get_state()]
    anc = []
    for _ in range(pb.T):
        f.step()
        xs.append(f.get_state())
        f.resample()
        anc.append(f.ancestors())
    xh, ah = _history_arrays(f, pb, fp64)
    for t in range(pb.T + 1):
        np.testing.assert_array_equal(xh[t].astype(np.float64), xs[t], err_msg=f"slot {t}")
    for t in range(pb.T):
        np.testing.assert_array_equal(ah[t], anc[t], err_msg=f"ancestors {t + 1}")
    f.close()
    g = pfm.Filter(pb, precision=precision, layout=pfm.PF_LAYOUT_BATCHED)
    g.set_tuning(512, 3)
    g.set_resampler(scheme, steps, ess_frac)
    g.attach_history()
    g.graph_run(pb.T)
    xh2, ah2 = _history_arrays(g, pb, fp64)
    np.testing.assert_array_equal(xh2, xh)
    np.testing.assert_array_equal(ah2, ah)
    g.close()
