"""The stateless systematic resampler (pf_systematic) on device log-weights,
through the C ABI, against the oracle's collective (orc_reduce_resample: max,
sums, sequential cumulative weights, a_k = min{j : N W_j > (u + k) S}) on the
same weights and uniform: ancestors equal except at strata within 1e-9
(normalised) of a cumulative weight, the likelihood increment within 1e-10
relative, the ESS within 1e-9.  Sizes span one partial block, ragged tails,
the combine inside the scan kernel (up to 1024 blocks of 256) and the
separate combine kernel beyond; weights spread, concentrated, with zero
(-inf) and NaN entries, and with none positive."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

BAND = 1e-9
REL64 = 1e-10


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_3277_amd as pfm
    pfm.load()
    return torch, pfm


def band_ok(lw, u, a_gpu, a_ref):
    mism = np.flatnonzero(a_gpu != a_ref)
    if mism.size == 0:
        return 0
    w = np.where(np.isnan(lw), 0.0, np.exp(lw - np.nanmax(lw)))
    cw = np.cumsum(w) / w.sum()
    N = lw.size
    for k in mism:
        gap = np.min(np.abs(cw - (u + k) / N))
        assert gap < BAND, f"ancestor {k}: gpu {a_gpu[k]} oracle {a_ref[k]} gap {gap}"
    return mism.size


def weights(kind, n, rng):
    if kind == "spread":
        return rng.normal(0.0, 1.0, n)
    if kind == "wide":
        return rng.normal(0.0, 30.0, n)
    if kind == "concentrated":
        lw = np.full(n, -800.0) + rng.normal(0.0, 1.0, n)
        lw[rng.integers(0, n, 3)] = rng.normal(0.0, 0.5, 3)
        return lw
    if kind == "holes":
        lw = rng.normal(0.0, 2.0, n)
        lw[rng.random(n) < 0.3] = -np.inf
        lw[rng.random(n) < 0.1] = np.nan
        return lw
    if kind == "last_only":
        lw = np.full(n, -np.inf)
        lw[-1] = 3.0
        return lw
    raise KeyError(kind)


def run(env, lw, u):
    torch, pfm = env
    d = torch.from_numpy(lw).to("cuda")
    anc, stats = pfm.systematic(d, u)
    torch.cuda.synchronize()
    return anc.cpu().numpy(), stats.cpu().numpy()


def check(lw, u, a, stats):
    st, ell, ess, a_ref = oracle.reduce_resample(lw, u)
    assert st == oracle.ORC_OK
    assert abs(stats[0] - ell) <= REL64 * max(1.0, abs(ell)), (stats[0], ell)
    assert stats[1] == pytest.approx(ess, rel=1e-9)
    assert np.all(np.diff(a) >= 0) and a[0] >= 0 and a[-1] < lw.size
    band_ok(lw, u, a, a_ref)
    # offspring counts in {floor(N w), ceil(N w)} up to the band
    N = lw.size
    w = np.where(np.isnan(lw), 0.0, np.exp(lw - np.nanmax(lw)))
    nw = N * w / w.sum()
    o = np.bincount(a, minlength=N)
    assert o.sum() == N
    assert np.all(o >= np.floor(nw - N * BAND)) and np.all(o <= np.ceil(nw + N * BAND))


@pytest.mark.parametrize("n", [1, 7, 255, 256, 1000, 4096 + 13, 65536, 262144 + 5])
@pytest.mark.parametrize("kind", ["spread", "wide", "concentrated", "holes", "last_only"])
def test_systematic_matches_oracle(env, n, kind):
    rng = np.random.default_rng(n * 7 + len(kind))
    lw = weights(kind, n, rng)
    for u in (0.0, float(rng.random()), 1.0 - 2.0 ** -40):
        a, stats = run(env, lw, u)
        check(lw, u, a, stats)


def test_systematic_full_size(env):
    """2^20 weights (4,096 block partials: the separate combine kernel)."""
    rng = np.random.default_rng(11)
    for kind in ("spread", "concentrated"):
        lw = weights(kind, 1 << 20, rng)
        u = float(rng.random())
        a, stats = run(env, lw, u)
        check(lw, u, a, stats)


def test_systematic_no_positive_weight(env):
    for lw in (np.full(300, -np.inf), np.full(5000, np.nan)):
        a, stats = run(env, lw, 0.5)
        st, ell, _, a_ref = oracle.reduce_resample(lw, 0.5)
        assert st == oracle.ORC_NUMERIC and ell == -np.inf
        assert stats[0] == -np.inf and stats[1] == 0.0
        np.testing.assert_array_equal(a, a_ref)


def test_systematic_workspace_reuse_and_graph(env):
    """One workspace over calls of different sizes, and the same call captured
    in a HIP graph and replayed several times with eager work between the
    replays: every result equals the eager call's."""
    torch, pfm = env
    rng = np.random.default_rng(5)
    big = torch.from_numpy(weights("holes", 70000, rng)).to("cuda")
    small = torch.from_numpy(weights("concentrated", 3000, rng)).to("cuda")
    from paper_1306_3277_amd import binding
    ws = torch.empty(int(binding.load().pf_systematic_workspace_bytes(70000)) + 256,
                     dtype=torch.uint8, device="cuda")
    a1, s1 = pfm.systematic(big, 0.25, workspace=ws)
    a2, s2 = pfm.systematic(small, 0.75, workspace=ws)
    a3, s3 = pfm.systematic(big, 0.25, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(a1, a3) and torch.equal(s1, s3)
    check(small.cpu().numpy(), 0.75, a2.cpu().numpy(), s2.cpu().numpy())
    s = torch.cuda.Stream()
    anc = torch.empty(70000, dtype=torch.int32, device="cuda")
    st = torch.empty(2, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        pfm.systematic(big, 0.25, anc=anc, stats=st, workspace=ws, stream=s)  # warm-up
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            pfm.systematic(big, 0.25, anc=anc, stats=st, workspace=ws, stream=s)
    for _ in range(3):
        anc.fill_(-7)
        st.fill_(0.0)
        pfm.systematic(small, 0.75, workspace=ws)  # eager work on the same scratch
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(anc, a1) and torch.equal(st, s1)


def test_systematic_rejects_bad_arguments(env):
    torch, pfm = env
    lw = torch.zeros(10, dtype=torch.float64, device="cuda")
    for u in (-0.1, 1.0, float("nan")):
        with pytest.raises(pfm.PfError) as ei:
            pfm.systematic(lw, u)
        assert ei.value.status == 1
