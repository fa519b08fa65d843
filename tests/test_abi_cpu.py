"""C-ABI checks that need no GPU: the built library exports every function
include/pf.h declares, and configurations are validated on the host (the
size query returns 0 with a message) before any HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_1306_3277_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pf_[a-z_0-9]+)\s*\(",
                                 src, flags=re.M)))


def test_header_declarations_are_bound_and_exported():
    names = declared_functions()
    assert "pf_init" in names and "pf_step" in names and "pf_resample" in names
    assert "pf_loglik" in names
    assert set(names) == set(binding.SIGNATURES), set(names) ^ set(binding.SIGNATURES)
    lib = binding.load()
    for n in names:
        assert hasattr(lib, n), n


def _size(pb, **kw):
    hc = binding._HostCfg(pb, **kw)
    return hc, binding.load().pf_workspace_bytes(C.byref(hc.cfg))


def test_valid_configs_have_a_size():
    for pb in (W.config("windkessel"), W.config("lorenz96_d8"), W.config("lorenz96_d40_large"), W.config("lorenz96_d8_batched")):
        _, n = _size(pb.with_obs(np.zeros((pb.T, pb.n_obs))),
                     layout=binding.PF_LAYOUT_BATCHED if pb.B > 1 else 0)
        assert n > 0
    # state, log-weights, counts, ancestors at least
    pb = W.config("lorenz96_d40_large").with_obs(np.zeros((500, 20)))
    _, n = _size(pb)
    N = 1 << 20
    assert n >= 2 * 40 * N * 4 + 3 * 4 * N


def _msg():
    return binding.load().pf_last_error().decode()


def test_smc2_workspace_size_and_run_length():
    pb = W.config("lorenz96_d8_batched")
    hc = binding._HostCfg(pb.with_obs(np.zeros((pb.T, pb.n_obs))),
                          layout=binding.PF_LAYOUT_BATCHED)
    L = binding.load()
    n = L.pf_smc2_workspace_bytes(C.byref(hc.cfg), pb.T)
    # the random inputs alone: normals, log-uniforms and copy words per (time, particle)
    assert n >= pb.T * pb.B * (8 * pb.n_theta + 8 + 4)
    assert L.pf_smc2_workspace_bytes(C.byref(hc.cfg), 10) < n
    assert L.pf_smc2_workspace_bytes(C.byref(hc.cfg), 0) == 0 and "T_run" in _msg()
    assert L.pf_smc2_workspace_bytes(C.byref(hc.cfg), pb.T + 1) == 0


@pytest.mark.parametrize("mutate,needle", [
    (lambda c: setattr(c, "model", 4), "model"),
    (lambda c: setattr(c, "precision", 7), "precision"),
    (lambda c: setattr(c, "d", 7), "d must be"),
    (lambda c: setattr(c, "K", 0), "K must"),
    (lambda c: setattr(c, "T", 0), "T must"),
    (lambda c: setattr(c, "h", -1.0), "h must"),
    (lambda c: setattr(c, "obs_sd", 0.0), "obs_sd"),
    (lambda c: setattr(c, "B", 0), "B must"),
    (lambda c: setattr(c, "n_theta", 3), "n_theta"),
])
def test_invalid_configs_rejected_on_host(mutate, needle):
    pb = W.config("lorenz96_d8", N=64, T=5).with_obs(np.zeros((5, 8)))
    hc = binding._HostCfg(pb)
    mutate(hc.cfg)
    assert binding.load().pf_workspace_bytes(C.byref(hc.cfg)) == 0
    assert needle in _msg()


def test_invalid_arrays_rejected_on_host():
    pb = W.config("lorenz96_d8", N=64, T=5)
    obs = np.zeros((5, 8))
    obs[2, 3] = np.nan
    _, n = _size(pb.with_obs(obs))
    assert n == 0 and "not finite" in _msg()
    pb2 = W.config("lorenz96_d8", N=64, T=5).with_obs(np.zeros((5, 8)))
    pb2.obs_idx = np.array([0, 2, 1, 3, 4, 5, 6, 7], dtype=np.int32)
    _, n = _size(pb2)
    assert n == 0 and "increasing" in _msg()
    _, n = _size(pb.with_obs(np.zeros((5, 8))), n_particles=[0])
    assert n == 0 and "n_particles" in _msg()
    big = W.config("lorenz96_d8_batched", B=3)
    _, n = _size(big.with_obs(np.zeros((big.T, 8))), layout=binding.PF_LAYOUT_BATCHED,
                 n_particles=[256, 9000, 512])
    assert n == 0 and "8192" in _msg()
    wk = W.config("windkessel", N=16, T=4)
    wk.q = None
    _, n = _size(wk.with_obs(np.zeros((4, 1))))
    assert n == 0 and "flow" in _msg()


def test_init_rejects_before_touching_the_device():
    pb = W.config("lorenz96_d8", N=64, T=5).with_obs(np.zeros((5, 8)))
    hc = binding._HostCfg(pb)
    hc.cfg.K = -3
    h = C.c_void_p()
    st = binding.load().pf_init(C.byref(hc.cfg), C.c_void_p(256), C.c_size_t(1 << 20), None,
                                C.byref(h))
    assert st == binding.PF_E_INVAL and not h.value
    hc = binding._HostCfg(pb)
    st = binding.load().pf_init(C.byref(hc.cfg), C.c_void_p(256), C.c_size_t(16), None,
                                C.byref(h))
    assert st == binding.PF_E_INVAL and "workspace" in _msg()


def test_version():
    assert binding.load().pf_version().decode().startswith("pfmi")


def test_systematic_arguments_checked_on_the_host():
    L = binding.load()
    assert L.pf_systematic_workspace_bytes(0) == 0 and "n = 0" in _msg()
    n = L.pf_systematic_workspace_bytes(1 << 20)
    # partials, offsets, one mark per weight, per-tile slots: about 4.2 bytes per weight
    assert 4 * (1 << 20) < n < 5 * (1 << 20)
    fake = C.c_void_p(0x10000)  # never dereferenced: every case fails before any HIP call
    cases = [
        ((None, 10, 0.5, fake, fake, fake, n), "NULL"),
        ((fake, 0, 0.5, fake, fake, fake, n), "n = 0"),
        ((fake, 10, 1.0, fake, fake, fake, n), "u = 1"),
        ((fake, 10, -0.5, fake, fake, fake, n), "u = -0.5"),
        ((fake, 10, 0.5, fake, fake, None, n), "workspace is NULL"),
        ((fake, 10, 0.5, fake, fake, C.c_void_p(0x10010), n), "aligned"),
        ((fake, 1 << 20, 0.5, fake, fake, fake, 1000), "needs"),
    ]
    for args, msg in cases:
        st = L.pf_systematic(*args, None)
        assert st == binding.PF_E_INVAL, (args, st)
        assert msg in _msg(), (msg, _msg())


def test_kalman_pmmh_needs_a_handle():
    L = binding.load()
    spec = binding.wk_mh_struct(W.WkMh())
    fake = C.c_void_p(0x10000)  # never dereferenced: the handle check fails first
    st = L.pf_kalman_pmmh(None, C.byref(spec), 1, fake, fake, fake, fake, fake, fake, None)
    assert st == binding.PF_E_INVAL, st


def test_restore_needs_a_handle():
    L = binding.load()
    x = np.zeros(8)
    ll = np.zeros(1)
    st = L.pf_restore(None, 0, x.ctypes.data_as(C.POINTER(C.c_double)),
                      ll.ctypes.data_as(C.POINTER(C.c_double)))
    assert st == binding.PF_E_INVAL, st


def test_tuning_calls_need_a_handle():
    L = binding.load()
    assert L.pf_set_replay(None, 1) == binding.PF_E_INVAL
    t = C.c_int32()
    assert L.pf_get_tuning(None, C.byref(t), None, None) == binding.PF_E_INVAL
