"""pf_systematic_noalloc, whose scratch is the library's static device array,
against pf_systematic with a caller workspace, through the C ABI: on the same
device log-weights and uniform both give the same ancestors and (ell, ESS)
bit for bit (the same kernels), over consecutive calls on the shared array
whose sizes shrink (so nothing of a larger earlier call leaks into a smaller
later one), at the maximum size, and under graph capture; a size above the
maximum is rejected."""
import ctypes as C

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1306_3277_amd import binding
    binding.load()
    return torch, binding


def _lw(rng, n, kind):
    if kind == "spread":
        return rng.normal(0.0, 2.0, n)
    lw = np.full(n, -700.0) + rng.normal(0.0, 1.0, n)
    lw[rng.integers(0, n, 2)] = 0.0
    lw[rng.random(n) < 0.05] = np.nan
    return lw


def _both(env, lw, u):
    torch, binding = env
    d = torch.from_numpy(lw).to("cuda")
    a_ws, s_ws = binding.systematic(d, u)
    a_na = torch.full((lw.size,), -5, dtype=torch.int32, device="cuda")
    s_na = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
    L = binding.load()
    st = L.pf_systematic_noalloc(C.c_void_p(d.data_ptr()), lw.size, float(u),
                                 C.c_void_p(a_na.data_ptr()), C.c_void_p(s_na.data_ptr()),
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, L.pf_last_error()
    torch.cuda.synchronize()
    return a_ws.cpu().numpy(), s_ws.cpu().numpy(), a_na.cpu().numpy(), s_na.cpu().numpy()


def test_noalloc_equals_workspace_variant(env):
    rng = np.random.default_rng(3)
    # two calls in a row, the second smaller, then more shrinking sizes
    for n, kind, u in [(300007, "spread", 0.3), (4099, "concentrated", 0.9),
                       (1 << 20, "concentrated", 0.5), (1000, "spread", 0.0), (1, "spread", 0.7)]:
        lw = _lw(rng, n, kind)
        a_ws, s_ws, a_na, s_na = _both(env, lw, u)
        np.testing.assert_array_equal(a_na, a_ws)
        np.testing.assert_array_equal(s_na, s_ws)
        st, ell, _, a_ref = oracle.reduce_resample(lw, u)
        assert st == oracle.ORC_OK
        assert abs(s_na[0] - ell) <= 1e-10 * max(1.0, abs(ell))


def test_noalloc_under_graph_capture(env):
    torch, binding = env
    rng = np.random.default_rng(4)
    lw = torch.from_numpy(_lw(rng, 50000, "spread")).to("cuda")
    small = torch.from_numpy(_lw(rng, 999, "concentrated")).to("cuda")
    ref_a, ref_s = binding.systematic(lw, 0.4)
    anc = torch.empty(50000, dtype=torch.int32, device="cuda")
    st = torch.empty(2, dtype=torch.float64, device="cuda")
    a2 = torch.empty(999, dtype=torch.int32, device="cuda")
    s2 = torch.empty(2, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        binding.systematic_noalloc(lw, 0.4, anc, st, stream=s)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            binding.systematic_noalloc(lw, 0.4, anc, st, stream=s)
    for _ in range(3):
        anc.fill_(-1)
        st.fill_(0.0)
        binding.systematic_noalloc(small, 0.6, a2, s2)  # eager use of the same array
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(anc, ref_a) and torch.equal(st, ref_s)


def test_noalloc_rejects_sizes_above_the_maximum(env):
    torch, binding = env
    n = binding.PF_SYSTEMATIC_NOALLOC_MAX_N + 1
    lw = torch.zeros(n, dtype=torch.float64, device="cuda")
    anc = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.PfError) as ei:
        binding.systematic_noalloc(lw, 0.5, anc, st)
    assert ei.value.status == binding.PF_E_INVAL
    assert "maximum" in str(ei.value)
