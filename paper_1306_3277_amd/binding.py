"""ctypes binding of the C ABI in include/pf.h — argument marshalling only.

Every step of the filter runs in the HIP library; PyTorch provides the device
workspace and the stream.  If the library is missing or no gfx950 device is
present, the calls raise: there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpf_mi355x.so")

PF_OK, PF_E_INVAL, PF_E_DEVICE, PF_E_STATE, PF_E_NUMERIC = 0, 1, 2, 3, 4
PF_MODEL_WK, PF_MODEL_L96, PF_MODEL_L96_STAGE = 1, 2, 3
PF_FP64, PF_FP32_MIXED, PF_FP32_ACCURATE = 0, 1, 2
PF_LAYOUT_PLAIN, PF_LAYOUT_BATCHED = 0, 1
PF_BATCHED_MAX_PARTICLES = 8192
PF_RESAMPLE_SYSTEMATIC, PF_RESAMPLE_STRATIFIED, PF_RESAMPLE_METROPOLIS = 0, 1, 2
PF_RESAMPLE_MULTINOMIAL = 3
PF_RESAMPLE_REJECTION = 4

_STATUS = {1: "PF_E_INVAL", 2: "PF_E_DEVICE", 3: "PF_E_STATE", 4: "PF_E_NUMERIC"}


class PfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class PfConfig(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("precision", C.c_int32), ("layout", C.c_int32),
        ("d", C.c_int32), ("K", C.c_int32), ("T", C.c_int32), ("h", C.c_double),
        ("n_obs", C.c_int32), ("obs_idx", C.POINTER(C.c_int32)), ("obs_sd", C.c_double),
        ("obs", C.POINTER(C.c_double)), ("q", C.POINTER(C.c_double)),
        ("B", C.c_int32), ("n_theta", C.c_int32), ("n_particles", C.POINTER(C.c_int64)),
        ("theta", C.POINTER(C.c_double)), ("seed", C.c_uint64),
    ]


class PfTiming(C.Structure):
    _fields_ = [
        ("propagate_ms", C.c_double), ("combine_ms", C.c_double), ("scan_ms", C.c_double),
        ("gather_ms", C.c_double), ("batched_ms", C.c_double),
        ("propagate_launches", C.c_int64), ("combine_launches", C.c_int64),
        ("scan_launches", C.c_int64), ("gather_launches", C.c_int64),
        ("batched_launches", C.c_int64),
    ]


class PfWkMh(C.Structure):
    _fields_ = [
        ("prior_shape", C.c_double * 3), ("prior_scale", C.c_double * 3),
        ("ig_shape", C.c_double), ("ig_scale", C.c_double), ("step_sd", C.c_double * 3),
        ("ig_prop_shape", C.c_double), ("ig_prop_factor", C.c_double),
        ("m0", C.c_double), ("s0", C.c_double),
    ]


def wk_mh_struct(spec) -> PfWkMh:
    """pf_wk_mh from an object with the same field names."""
    return PfWkMh((C.c_double * 3)(*spec.prior_shape), (C.c_double * 3)(*spec.prior_scale),
                  float(spec.ig_shape), float(spec.ig_scale), (C.c_double * 3)(*spec.step_sd),
                  float(spec.ig_prop_shape), float(spec.ig_prop_factor), float(spec.m0),
                  float(spec.s0))


class PfSmc2In(C.Structure):
    _fields_ = [
        ("T_run", C.c_int32), ("theta0", C.POINTER(C.c_double)), ("z", C.POINTER(C.c_double)),
        ("log_alpha", C.POINTER(C.c_double)), ("u", C.POINTER(C.c_double)),
        ("w_copy", C.POINTER(C.c_uint32)), ("step_sd", C.c_double * 8), ("lo", C.c_double * 8),
        ("hi", C.c_double * 8), ("filter", C.c_int32),
    ]


class PfSmc2Out(C.Structure):
    _fields_ = [
        ("theta", C.POINTER(C.c_double)), ("logw", C.POINTER(C.c_double)),
        ("loglik", C.POINTER(C.c_double)), ("accepts", C.POINTER(C.c_int32)),
        ("ess", C.POINTER(C.c_double)), ("log_evidence", C.POINTER(C.c_double)),
        ("anc_trace", C.POINTER(C.c_int32)), ("acc_trace", C.POINTER(C.c_int32)),
        ("logw_trace", C.POINTER(C.c_double)), ("theta_trace", C.POINTER(C.c_double)),
    ]


_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_H = C.c_void_p

# exported symbols and their signatures (also checked by the CPU tests)
SIGNATURES = {
    "pf_workspace_bytes": (C.c_size_t, [C.POINTER(PfConfig)]),
    "pf_init": (C.c_int, [C.POINTER(PfConfig), C.c_void_p, C.c_size_t, C.c_void_p,
                          C.POINTER(_H)]),
    "pf_step": (C.c_int, [_H]),
    "pf_resample": (C.c_int, [_H]),
    "pf_loglik": (C.c_int, [_H, _D, _D, _I]),
    "pf_get_trace": (C.c_int, [_H, _D, _D]),
    "pf_destroy": (C.c_int, [_H]),
    "pf_graph_run": (C.c_int, [_H, C.c_int32]),
    "pf_set_theta": (C.c_int, [_H, _D, C.c_uint32]),
    "pf_reset": (C.c_int, [_H, C.c_uint32]),
    "pf_get_state": (C.c_int, [_H, _D]),
    "pf_set_state": (C.c_int, [_H, _D]),
    "pf_restore": (C.c_int, [_H, C.c_int32, _D, _D]),
    "pf_get_logweights": (C.c_int, [_H, _D]),
    "pf_get_ancestors": (C.c_int, [_H, _I]),
    "pf_resample_u": (C.c_int, [_H, _D]),
    "pf_simulate_doubles": (C.c_size_t, [C.POINTER(PfConfig)]),
    "pf_simulate": (C.c_int, [C.POINTER(PfConfig), _D, C.c_uint64, C.c_void_p, C.c_size_t,
                              C.c_void_p]),
    "pf_pmmh": (C.c_int, [_H, C.c_int32, _D, _D, _D, C.c_double, C.c_double, C.c_double,
                          C.c_double, _D, _D, _I]),
    "pf_set_resampler": (C.c_int, [_H, C.c_int32, C.c_int32, C.c_double]),
    "pf_kalman": (C.c_int, [_H, _D, _D]),
    "pf_kalman_pmmh": (C.c_int, [_H, C.POINTER(PfWkMh), C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pf_history_bytes": (C.c_size_t, [C.POINTER(PfConfig)]),
    "pf_history_attach": (C.c_int, [_H, C.c_void_p, C.c_size_t]),
    "pf_backtrace": (C.c_int, [_H, _D, _I]),
    "pf_smc2_workspace_bytes": (C.c_size_t, [C.POINTER(PfConfig), C.c_int32]),
    "pf_smc2": (C.c_int, [_H, _H, C.c_void_p, C.c_size_t, C.POINTER(PfSmc2In),
                          C.POINTER(PfSmc2Out)]),
    "pf_autotune": (C.c_int, [_H, C.c_int32, _I, _I, _D]),
    "pf_set_tuning": (C.c_int, [_H, C.c_int32, C.c_int32]),
    "pf_set_replay": (C.c_int, [_H, C.c_int32]),
    "pf_get_tuning": (C.c_int, [_H, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32)]),
    "pf_timing_enable": (C.c_int, [_H, C.c_int32]),
    "pf_timing_get": (C.c_int, [_H, C.POINTER(PfTiming)]),
    "pf_systematic_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "pf_systematic": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_size_t, C.c_void_p]),
    "pf_systematic_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "pf_last_error": (C.c_char_p, []),
    "pf_version": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (built by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"HIP library {path} is not built; run __graft_entry__.build()")
        # PyTorch's HIP runtime must be the process's runtime: load it first so
        # the library binds to it rather than bringing in a second copy
        import torch  # noqa: F401
        L = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != PF_OK:
        raise PfError(st, load().pf_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(_D)


def _ip(a):
    return a.ctypes.data_as(_I)


class _HostCfg:
    """A pf_config plus the numpy arrays it points into."""

    def __init__(self, pb, precision: Optional[int] = None, layout: int = PF_LAYOUT_PLAIN,
                 theta=None, n_particles=None, seed: Optional[int] = None):
        self.obs_idx = np.ascontiguousarray(pb.obs_idx, dtype=np.int32)
        obs = pb.obs if pb.obs is not None else np.zeros((pb.T, len(self.obs_idx)))
        self.obs = np.ascontiguousarray(obs, dtype=np.float64)
        self.q = None if pb.q is None else np.ascontiguousarray(pb.q, dtype=np.float64)
        th = pb.theta if theta is None else theta
        self.theta = np.ascontiguousarray(np.atleast_2d(th), dtype=np.float64)
        npart = pb.n_particles if n_particles is None else n_particles
        self.n_particles = np.ascontiguousarray(np.atleast_1d(npart), dtype=np.int64)
        prec = pb.precision if precision is None else precision
        self.cfg = PfConfig(
            pb.model, prec, layout, pb.d, pb.K, pb.T, pb.h, len(self.obs_idx),
            _ip(self.obs_idx), pb.obs_sd, _dp(self.obs),
            _dp(self.q) if self.q is not None else None,
            self.theta.shape[0], self.theta.shape[1], self.n_particles.ctypes.data_as(
                C.POINTER(C.c_int64)), _dp(self.theta), int(pb.seed if seed is None else seed))


def _stream_handle(stream) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class Filter:
    """One handle over B filters (Alg. 2) on the current HIP device."""

    def __init__(self, pb, precision: Optional[int] = None, layout: int = PF_LAYOUT_PLAIN,
                 stream=None, seed: Optional[int] = None, device: str = "cuda"):
        import torch
        L = load()
        self.pb = pb
        self.hc = _HostCfg(pb, precision, layout, seed=seed)
        self.precision = self.hc.cfg.precision
        self.layout = layout
        self.B = self.hc.cfg.B
        self.d = pb.d
        self.T = pb.T
        self.n_total = int(self.hc.n_particles.sum())
        self.offsets = np.concatenate([[0], np.cumsum(self.hc.n_particles)])
        nbytes = L.pf_workspace_bytes(C.byref(self.hc.cfg))
        if nbytes == 0:
            _check(PF_E_INVAL)
        self.workspace = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream
        self._sh = _stream_handle(stream)
        h = _H()
        _check(L.pf_init(C.byref(self.hc.cfg), C.c_void_p(aligned), C.c_size_t(nbytes),
                         C.c_void_p(self._sh), C.byref(h)))
        self.h = h

    # -- the filter
    def step(self):
        _check(load().pf_step(self.h))

    def resample(self):
        _check(load().pf_resample(self.h))

    def resample_u(self, u):
        u = np.ascontiguousarray(np.atleast_1d(u), dtype=np.float64)
        _check(load().pf_resample_u(self.h, _dp(u)))

    def advance(self, n: int = 1):
        for _ in range(n):
            self.step()
            self.resample()

    def graph_run(self, n: int):
        _check(load().pf_graph_run(self.h, int(n)))

    def loglik(self, allow_numeric: bool = False):
        ll = np.zeros(self.B)
        ess = np.zeros(self.B)
        t = C.c_int32()
        st = load().pf_loglik(self.h, _dp(ll), _dp(ess), C.byref(t))
        if not (allow_numeric and st == PF_E_NUMERIC):
            _check(st)
        return ll, ess, t.value

    def trace(self):
        ell = np.zeros((self.B, self.T))
        ess = np.zeros((self.B, self.T))
        _check(load().pf_get_trace(self.h, _dp(ell), _dp(ess)))
        return ell, ess

    def set_theta(self, theta, iteration: int = 0):
        th = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
        _check(load().pf_set_theta(self.h, _dp(th), int(iteration)))

    def reset(self, iteration: int = 0):
        _check(load().pf_reset(self.h, int(iteration)))

    # -- parameter inference / tuning
    def pmmh(self, inputs, iters: Optional[int] = None):
        """Alg. 3 chains, one per filter; ``inputs`` is a workloads.PmmhInputs."""
        iters = inputs.z.shape[0] if iters is None else iters
        lf0 = np.ascontiguousarray(inputs.log_f0[:self.B], dtype=np.float64)
        z = np.ascontiguousarray(inputs.z[:iters, :self.B], dtype=np.float64)
        al = np.ascontiguousarray(inputs.alpha[:iters, :self.B], dtype=np.float64)
        lft = np.zeros((iters, self.B))
        llt = np.zeros((iters, self.B))
        acc = np.zeros(self.B, dtype=np.int32)
        _check(load().pf_pmmh(self.h, int(iters), _dp(lf0), _dp(z), _dp(al), inputs.step_sd,
                              inputs.f_lo, inputs.f_hi, inputs.sigma, _dp(lft), _dp(llt),
                              _ip(acc)))
        return dict(log_f=lft, ll=llt, accepts=acc)

    # -- resampling variants
    def set_resampler(self, scheme: int = PF_RESAMPLE_SYSTEMATIC, steps: int = 0,
                      ess_frac: float = float("inf")):
        _check(load().pf_set_resampler(self.h, int(scheme), int(steps), float(ess_frac)))

    # -- ancestry storage and the state sample (Alg. 2, last lines)
    def attach_history(self, device: str = "cuda"):
        """Allocate and attach a history (at t = 0); later intervals record."""
        import torch
        L = load()
        n = L.pf_history_bytes(C.byref(self.hc.cfg))
        if n == 0:
            _check(PF_E_INVAL)
        self.history = torch.empty(int(n) + 256, dtype=torch.uint8, device=device)
        aligned = (self.history.data_ptr() + 255) & ~255
        _check(L.pf_history_attach(self.h, C.c_void_p(aligned), C.c_size_t(int(n))))

    def detach_history(self):
        _check(load().pf_history_attach(self.h, None, 0))
        self.history = None

    def backtrace(self):
        """State sample per filter: (path [B, s+1, d], particle indices [B, s+1])."""
        t = self.loglik(allow_numeric=True)[2]
        path = np.zeros((self.B, t + 1, self.d))
        idx = np.zeros((self.B, t + 1), dtype=np.int32)
        _check(load().pf_backtrace(self.h, _dp(path), _ip(idx)))
        return path, idx

    def kalman(self):
        """Exact windkessel log-likelihood per filter (Kalman filter):
        (loglik [B], ell [B, T])."""
        ll = np.zeros(self.B)
        ell = np.zeros((self.B, self.T))
        _check(load().pf_kalman(self.h, _dp(ll), _dp(ell)))
        return ll, ell

    def kalman_pmmh(self, spec, theta0, prop, alpha, iters: Optional[int] = None,
                    device: str = "cuda", out=None, sync: bool = True):
        """Marginal Metropolis-Hastings chains on the windkessel's (R, C, Z,
        sigma^2) with the exact Kalman likelihood, one per filter slot.
        ``spec`` has pf_wk_mh's fields; theta0 [B, 4], prop [iters, B, 4],
        alpha [iters, B] are arrays or device tensors (FP64).  Returns device
        tensors theta [iters, B, 4], ll [iters, B], accepts [B], ll0 [B]
        (``out``, a dict of those, is reused when given)."""
        import torch
        dev = torch.device(device)

        def on_dev(a):
            if isinstance(a, torch.Tensor):
                return a.to(device=dev, dtype=torch.float64).contiguous()
            # a row-major copy (a broadcast view would otherwise keep its strides)
            return torch.from_numpy(np.array(a, dtype=np.float64, order="C")).to(dev)

        th0, pr, al = on_dev(theta0), on_dev(prop), on_dev(alpha)
        if not (th0.is_contiguous() and pr.is_contiguous() and al.is_contiguous()):
            raise ValueError("inputs must be row-major")
        iters = int(pr.shape[0]) if iters is None else int(iters)
        B = self.B
        if tuple(th0.shape) != (B, 4) or pr.shape[0] < iters or tuple(pr.shape[1:]) != (B, 4) \
                or al.shape[0] < iters or tuple(al.shape[1:]) != (B,):
            raise ValueError("theta0 [B, 4], prop [iters, B, 4], alpha [iters, B] expected")
        if out is None:
            out = dict(theta=torch.empty((iters, B, 4), dtype=torch.float64, device=dev),
                       ll=torch.empty((iters, B), dtype=torch.float64, device=dev),
                       accepts=torch.empty(B, dtype=torch.int32, device=dev),
                       ll0=torch.empty(B, dtype=torch.float64, device=dev))
        hs = wk_mh_struct(spec)
        torch.cuda.synchronize(dev)  # inputs made on torch's stream, the chains run on the handle's
        _check(load().pf_kalman_pmmh(self.h, C.byref(hs), iters, C.c_void_p(th0.data_ptr()),
                                     C.c_void_p(pr.data_ptr()), C.c_void_p(al.data_ptr()),
                                     C.c_void_p(out["theta"].data_ptr()),
                                     C.c_void_p(out["ll"].data_ptr()),
                                     C.c_void_p(out["accepts"].data_ptr()),
                                     C.c_void_p(out["ll0"].data_ptr())))
        if sync:
            torch.cuda.synchronize(dev)
        return out

    def smc2(self, proposal: Optional["Filter"], inputs, T: Optional[int] = None,
             traces: bool = True, device: str = "cuda", kalman: bool = False):
        """SMC over the parameters (Alg. 4) with this handle's filters attached
        to the theta-particles and ``proposal`` (a second batched handle of the
        same problem, on the same stream) running the rejuvenation proposals.
        ``inputs`` is a workloads.Smc2Inputs."""
        import torch
        L = load()
        T = inputs.T if T is None else int(T)
        B, nth = self.B, self.hc.cfg.n_theta
        th0 = np.ascontiguousarray(inputs.theta0, dtype=np.float64).reshape(B, nth)
        z = np.ascontiguousarray(inputs.z[:T], dtype=np.float64).reshape(T, B, nth)
        la = np.ascontiguousarray(inputs.log_alpha[:T], dtype=np.float64).reshape(T, B)
        u = np.ascontiguousarray(inputs.u[:T], dtype=np.float64).reshape(T)
        w = np.ascontiguousarray(inputs.w_copy[:T], dtype=np.uint32).reshape(T, B)
        ci = PfSmc2In(T, _dp(th0), _dp(z), _dp(la), _dp(u), w.ctypes.data_as(C.POINTER(C.c_uint32)))
        ci.filter = 1 if kalman else 0
        for p in range(nth):
            ci.step_sd[p] = float(inputs.step_sd[p])
            ci.lo[p] = float(inputs.lo[p])
            ci.hi[p] = float(inputs.hi[p])
        res = dict(theta=np.zeros((B, nth)), logw=np.zeros(B), loglik=np.zeros(B),
                   accepts=np.zeros(B, dtype=np.int32), ess=np.zeros(T),
                   log_evidence=np.zeros(1))
        if traces:
            res.update(anc=np.zeros((T, B), dtype=np.int32), acc=np.zeros((T, B), dtype=np.int32),
                       logw_trace=np.zeros((T, B)), theta_trace=np.zeros((T, B, nth)))
        co = PfSmc2Out(_dp(res["theta"]), _dp(res["logw"]), _dp(res["loglik"]),
                       _ip(res["accepts"]), _dp(res["ess"]), _dp(res["log_evidence"]),
                       _ip(res["anc"]) if traces else None, _ip(res["acc"]) if traces else None,
                       _dp(res["logw_trace"]) if traces else None,
                       _dp(res["theta_trace"]) if traces else None)
        nbytes = L.pf_smc2_workspace_bytes(C.byref(self.hc.cfg), T)
        if nbytes == 0:
            _check(PF_E_INVAL)
        ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
        aligned = (ws.data_ptr() + 255) & ~255
        st = L.pf_smc2(self.h, proposal.h if proposal is not None else None, C.c_void_p(aligned),
                       C.c_size_t(nbytes), C.byref(ci), C.byref(co))
        res["status"] = st
        if st not in (PF_OK, PF_E_NUMERIC):
            _check(st)
        res["log_evidence"] = float(res["log_evidence"][0])
        return res

    def autotune(self, steps: int = 8):
        """Returns (collective threads, groups, ms per interval [groups x sizes])."""
        th = C.c_int32()
        gr = C.c_int32()
        ms = np.zeros(9)
        _check(load().pf_autotune(self.h, int(steps), C.byref(th), C.byref(gr), _dp(ms)))
        return th.value, gr.value, ms.reshape(3, 3)

    def set_tuning(self, threads: int, groups: int):
        _check(load().pf_set_tuning(self.h, int(threads), int(groups)))

    def set_replay(self, eager: bool):
        """graph_run by eager launches (True) or graph replay (False)."""
        _check(load().pf_set_replay(self.h, 1 if eager else 0))

    def get_tuning(self):
        """(collective threads, groups, eager replay) of a batched handle."""
        th, gr, eg = C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().pf_get_tuning(self.h, C.byref(th), C.byref(gr), C.byref(eg)))
        return th.value, gr.value, bool(eg.value)

    # -- inspection / teacher forcing
    def get_state(self) -> np.ndarray:
        x = np.zeros((self.d, self.n_total))
        _check(load().pf_get_state(self.h, _dp(x)))
        return x

    def set_state(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.d, self.n_total)
        _check(load().pf_set_state(self.h, _dp(x)))

    def restore(self, t: int, x, loglik):
        """Resume from a checkpoint: every filter at t intervals with the
        equally weighted set x ([d][N_total]) and running log-likelihoods
        loglik[B] (what get_state and loglik return after a resampling)."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.d, self.n_total)
        ll = np.ascontiguousarray(loglik, dtype=np.float64).reshape(-1)
        if ll.size != self.B:
            raise ValueError(f"loglik has {ll.size} entries for {self.B} filters")
        _check(load().pf_restore(self.h, int(t), _dp(x), _dp(ll)))

    def logweights(self) -> np.ndarray:
        lw = np.zeros(self.n_total)
        _check(load().pf_get_logweights(self.h, _dp(lw)))
        return lw

    def ancestors(self) -> np.ndarray:
        a = np.zeros(self.n_total, dtype=np.int32)
        _check(load().pf_get_ancestors(self.h, _ip(a)))
        return a

    # -- measurement
    def timing(self, on: bool = True):
        _check(load().pf_timing_enable(self.h, 1 if on else 0))

    def timing_get(self) -> dict:
        t = PfTiming()
        _check(load().pf_timing_get(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in PfTiming._fields_}

    def close(self):
        if getattr(self, "h", None):
            load().pf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(pb, theta=None, data_seed: Optional[int] = None, stream=None, device: str = "cuda"):
    """Synthetic truth [T+1, d] and observations [T, n_obs], simulated on the GPU."""
    import torch
    L = load()
    th = np.ascontiguousarray(pb.data_theta if theta is None else theta, dtype=np.float64)
    hc = _HostCfg(pb, theta=th[None, :], n_particles=[1])
    n = L.pf_simulate_doubles(C.byref(hc.cfg))
    buf = torch.zeros(int(n), dtype=torch.float64, device=device)
    sh = _stream_handle(stream)
    _check(L.pf_simulate(C.byref(hc.cfg), _dp(th), int(pb.data_seed if data_seed is None
                                                         else data_seed),
                         C.c_void_p(buf.data_ptr()), C.c_size_t(int(n)), C.c_void_p(sh)))
    out = buf.cpu().numpy()
    nx = (pb.T + 1) * pb.d
    xt = out[:nx].reshape(pb.T + 1, pb.d)
    y = out[nx:nx + pb.T * len(pb.obs_idx)].reshape(pb.T, len(pb.obs_idx))
    return xt.copy(), y.copy()


def systematic(lw, u: float, anc=None, stats=None, workspace=None, stream=None):
    """pf_systematic on device tensors: lw (float64, n) and the uniform u;
    returns (ancestors int32 [n], stats float64 [2] = (ell, ESS)) as device
    tensors, written asynchronously on the stream.  Outputs and workspace are
    allocated here when not given."""
    import torch
    L = load()
    n = int(lw.numel())
    assert lw.dtype == torch.float64 and lw.is_contiguous()
    if anc is None:
        anc = torch.empty(n, dtype=torch.int32, device=lw.device)
    if stats is None:
        stats = torch.empty(2, dtype=torch.float64, device=lw.device)
    nb = int(L.pf_systematic_workspace_bytes(n))
    if nb == 0:
        _check(PF_E_INVAL)
    if workspace is None:
        workspace = torch.empty(nb + 256, dtype=torch.uint8, device=lw.device)
    base = workspace.data_ptr()
    pad = (-base) % 256
    _check(L.pf_systematic(C.c_void_p(lw.data_ptr()), n, float(u), C.c_void_p(anc.data_ptr()),
                           C.c_void_p(stats.data_ptr()), C.c_void_p(base + pad),
                           C.c_size_t(workspace.numel() - pad), C.c_void_p(_stream_handle(stream))))
    return anc, stats


PF_SYSTEMATIC_NOALLOC_MAX_N = 1 << 20


def systematic_noalloc(lw, u: float, anc, stats, stream=None):
    """pf_systematic_noalloc on device tensors: lw (float64, n), u, and the
    caller's outputs anc (int32, n) and stats (float64, 2), written
    asynchronously on the stream; the library's static scratch is used."""
    L = load()
    n = int(lw.numel())
    _check(L.pf_systematic_noalloc(C.c_void_p(lw.data_ptr()), n, float(u),
                                   C.c_void_p(anc.data_ptr()), C.c_void_p(stats.data_ptr()),
                                   C.c_void_p(_stream_handle(stream))))
    return anc, stats
