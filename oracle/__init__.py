"""Python access to the plain C oracle — TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It never imports the HIP library or
its binding, and the product never imports it.

``build()`` compiles ``pf_oracle.c`` with gcc (FP64, contraction off) into
``liborc.so`` beside it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

ORC_OK = 0
ORC_NUMERIC = 4
TAG_INIT, TAG_NOISE, TAG_RESAMPLE, TAG_DATA, TAG_OBS, TAG_PATH, TAG_MULTI = 1, 2, 3, 4, 8, 9, 10
TAG_REJECT = 11


def build(force: bool = True) -> str:
    """Compile the oracle (always, when force) and return the library path."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Problem(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("d", C.c_int32), ("K", C.c_int32), ("T", C.c_int32),
        ("h", C.c_double), ("n_obs", C.c_int32), ("obs_idx", C.POINTER(C.c_int32)),
        ("obs_sd", C.c_double), ("obs", C.POINTER(C.c_double)),
        ("q", C.POINTER(C.c_double)), ("seed", C.c_uint64),
    ]


class WkMh(C.Structure):
    _fields_ = [
        ("prior_shape", C.c_double * 3), ("prior_scale", C.c_double * 3),
        ("ig_shape", C.c_double), ("ig_scale", C.c_double), ("step_sd", C.c_double * 3),
        ("ig_prop_shape", C.c_double), ("ig_prop_factor", C.c_double),
        ("m0", C.c_double), ("s0", C.c_double),
    ]


def _wk_mh(spec) -> WkMh:
    return WkMh((C.c_double * 3)(*spec.prior_shape), (C.c_double * 3)(*spec.prior_scale),
                spec.ig_shape, spec.ig_scale, (C.c_double * 3)(*spec.step_sd),
                spec.ig_prop_shape, spec.ig_prop_factor, spec.m0, spec.s0)


_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_U = C.POINTER(C.c_uint32)


def lib():
    global _lib
    if _lib is None:
        stale = (not os.path.exists(_LIB)
                 or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                 os.path.getmtime(_SRC[:-1] + "h")))
        if stale:
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER(Problem)
        sig = {
            "orc_philox4x32_10": (None, [_U, _U, _U]),
            "orc_u01": (C.c_double, [C.c_uint32]),
            "orc_ln": (C.c_double, [C.c_double]),
            "orc_sincos2pi": (None, [C.c_double, _D, _D]),
            "orc_normals4": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                    C.c_uint32, C.c_uint32, _D]),
            "orc_normals_bulk": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint32, C.c_int64, _D]),
            "orc_l96_drift": (None, [C.c_int32, _D, C.c_double, _D]),
            "orc_init": (None, [P, _D, C.c_int64, C.c_uint32, C.c_uint32, _D]),
            "orc_propagate": (None, [P, _D, C.c_int64, C.c_uint32, C.c_uint32, C.c_int32, _D,
                                     _D]),
            "orc_init_idx": (None, [P, _D, C.c_int64, C.POINTER(C.c_int64), C.c_uint32,
                                    C.c_uint32, _D]),
            "orc_propagate_idx": (None, [P, _D, C.c_int64, C.POINTER(C.c_int64), C.c_uint32,
                                         C.c_uint32, C.c_int32, _D, _D]),
            "orc_weight": (None, [P, _D, C.c_int64, C.c_int32, _D, _D]),
            "orc_resample_u": (C.c_double, [C.c_uint64, C.c_int32, C.c_uint32, C.c_uint32]),
            "orc_reduce_resample": (C.c_int32, [C.c_int64, _D, C.c_double, _D, _D, _I]),
            "orc_gather": (None, [C.c_int32, C.c_int64, _D, _I, _D]),
            "orc_pf_run": (C.c_int32, [P, _D, C.c_int64, C.c_uint32, C.c_uint32, C.c_int32, _D,
                                       _D, _D, _I, _D, _D, _D]),
            "orc_kf_wk": (C.c_double, [P, _D, _D]),
            "orc_simulate": (None, [P, _D, C.c_uint64, _D, _D]),
            "orc_pmmh": (C.c_int32, [P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     _D, _D, _D, C.c_double, C.c_double, C.c_double, C.c_double,
                                     _D, _D, _I]),
            "orc_copy_index": (C.c_int64, [C.c_int64, C.c_int64, C.c_int64, C.c_uint32]),
            "orc_kf_wk_interval": (C.c_double, [P, _D, C.c_int32, _D, _D]),
            "orc_smc2_kalman": (C.c_int32, [P, C.c_int32, C.c_int32, _D, C.c_int32, _D, _D, _D,
                                            _D, _D, _D, _D, _D, _D, _I, _D, _D, _I, _I, _D,
                                            _D]),
            "orc_strat_u": (C.c_double, [C.c_uint64, C.c_int32, C.c_uint32, C.c_uint32,
                                         C.c_int64]),
            "orc_stratified_ancestors": (None, [C.c_int64, _D, C.c_double, C.c_int64,
                                                C.c_uint64, C.c_int32, C.c_uint32, C.c_uint32,
                                                _I]),
            "orc_multi_u": (C.c_double, [C.c_uint64, C.c_int32, C.c_uint32, C.c_uint32,
                                         C.c_int64]),
            "orc_multinomial_ancestors": (None, [C.c_int64, _D, C.c_double, C.c_int64,
                                                 C.c_uint64, C.c_int32, C.c_uint32, C.c_uint32,
                                                 _I]),
            "orc_metropolis_ancestors": (None, [C.c_int64, _D, C.c_int32, C.c_uint64,
                                                C.c_int32, C.c_uint32, C.c_uint32, _I]),
            "orc_reject_pair": (None, [C.c_uint64, C.c_int32, C.c_uint32, C.c_uint32, C.c_int64,
                                       C.c_int64, C.c_int64, C.POINTER(C.c_int64), _D]),
            "orc_rejection_ancestors": (None, [C.c_int64, _D, C.c_uint64, C.c_int32, C.c_uint32,
                                               C.c_uint32, _I]),
            "orc_pf_run_ex": (C.c_int32, [P, _D, C.c_int64, C.c_uint32, C.c_uint32, C.c_int32,
                                          C.c_int32, C.c_int32, C.c_double, _D, _D, _D, _I,
                                          _D, _I, _D]),
            "orc_path_slot": (C.c_int64, [C.c_uint64, C.c_int32, C.c_uint32, C.c_uint32,
                                          C.c_int64]),
            "orc_pf_path": (C.c_int32, [P, _D, C.c_int64, C.c_uint32, C.c_uint32, C.c_int32,
                                        _D, _D, C.POINTER(C.c_int64)]),
            "orc_ndtri": (C.c_double, [C.c_double]),
            "orc_wk_theta": (None, [P, C.POINTER(WkMh), _D, _D]),
            "orc_wk_log_prior": (C.c_double, [C.POINTER(WkMh), _D]),
            "orc_kf_pmmh": (C.c_int32, [P, C.POINTER(WkMh), C.c_int32, C.c_int32, _D, _D, _D,
                                        _D, _D, _I]),
            "orc_smc2": (C.c_int32, [P, C.c_int32, C.POINTER(C.c_int64), C.c_int32, _D,
                                     C.c_int32, _D, _D, _D, _D, _D, _D, _U, _D, _D, _D, _I,
                                     _D, _D, _I, _I, _D, _D, _D]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_D)


def _ip(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_I)


class _Prob:
    """Keeps the numpy arrays a ``Problem`` struct points into alive."""

    def __init__(self, pb, seed: Optional[int] = None):
        self.obs_idx = np.ascontiguousarray(pb.obs_idx, dtype=np.int32)
        self.obs = None if pb.obs is None else np.ascontiguousarray(pb.obs, dtype=np.float64)
        self.q = None if pb.q is None else np.ascontiguousarray(pb.q, dtype=np.float64)
        self.s = Problem(pb.model, pb.d, pb.K, pb.T, pb.h, len(self.obs_idx), _ip(self.obs_idx),
                         pb.obs_sd, _dp(self.obs), _dp(self.q),
                         int(pb.seed if seed is None else seed))

    @property
    def ref(self):
        return C.byref(self.s)


# ----------------------------------------------------------------- generator

def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def u01(w: int) -> float:
    return lib().orc_u01(int(w))


def ln(x: float) -> float:
    return lib().orc_ln(float(x))


def sincos2pi(u: float):
    s, c = C.c_double(), C.c_double()
    lib().orc_sincos2pi(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def normals4(seed, tag, blk, it, j, n, b) -> np.ndarray:
    z = np.zeros(4)
    lib().orc_normals4(seed, tag, blk, it, j, n, b, _dp(z))
    return z


def normals_bulk(seed, tag, it, b, n, count) -> np.ndarray:
    z = np.zeros((count, 4))
    lib().orc_normals_bulk(seed, tag, it, b, n, count, _dp(z))
    return z


# ----------------------------------------------------------------- filter pieces

def l96_drift(x, F) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    lib().orc_l96_drift(x.shape[0], _dp(x), float(F), _dp(out))
    return out


def init(pb, theta, N, b=0, it=0) -> np.ndarray:
    P = _Prob(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    x = np.zeros((pb.d, N))
    lib().orc_init(P.ref, _dp(th), N, b, it, _dp(x))
    return x


def propagate(pb, theta, x, t, b=0, it=0) -> np.ndarray:
    P = _Prob(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    N = x.shape[1]
    out = np.zeros_like(x)
    lib().orc_propagate(P.ref, _dp(th), N, b, it, t, _dp(x), _dp(out))
    return out


def init_idx(pb, theta, idx, b=0, it=0) -> np.ndarray:
    """Initial states of particles idx (columns) of filter b."""
    P = _Prob(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    x = np.zeros((pb.d, idx.size))
    lib().orc_init_idx(P.ref, _dp(th), idx.size, idx.ctypes.data_as(C.POINTER(C.c_int64)), b, it,
                       _dp(x))
    return x


def propagate_idx(pb, theta, x, idx, t, b=0, it=0) -> np.ndarray:
    """Propagate columns of x, column c being particle idx[c], from t-1 to t."""
    P = _Prob(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    lib().orc_propagate_idx(P.ref, _dp(th), idx.size, idx.ctypes.data_as(C.POINTER(C.c_int64)),
                            b, it, t, _dp(x), _dp(out))
    return out


def weight(pb, theta, x, t) -> np.ndarray:
    P = _Prob(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    N = x.shape[1]
    lw = np.zeros(N)
    lib().orc_weight(P.ref, _dp(th), N, t, _dp(x), _dp(lw))
    return lw


def resample_u(seed, t, b=0, it=0) -> float:
    return lib().orc_resample_u(int(seed), int(t), int(b), int(it))


def reduce_resample(lw, u):
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    N = lw.shape[0]
    a = np.zeros(N, dtype=np.int32)
    ell, ess = C.c_double(), C.c_double()
    st = lib().orc_reduce_resample(N, _dp(lw), float(u), C.byref(ell), C.byref(ess), _ip(a))
    return st, ell.value, ess.value, a


def gather(x, a) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.int32)
    out = np.zeros_like(x)
    lib().orc_gather(x.shape[0], x.shape[1], _dp(x), _ip(a), _dp(out))
    return out


def pf_run(pb, theta=None, N=None, b=0, it=0, T=None, traces=False, u=None):
    """Run Alg. 2 for one filter; returns a dict of per-step outputs."""
    P = _Prob(pb)
    th = np.ascontiguousarray(pb.theta[b] if theta is None else theta, dtype=np.float64)
    N = int(pb.n_particles[b] if N is None else N)
    T = pb.T if T is None else T
    ell, ess = np.zeros(T), np.zeros(T)
    ll = C.c_double()
    anc = np.zeros((T, N), dtype=np.int32) if traces else None
    lwt = np.zeros((T, N)) if traces else None
    xf = np.zeros((pb.d, N))
    uo = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    st = lib().orc_pf_run(P.ref, _dp(th), N, b, it, T, _dp(ell), _dp(ess), C.byref(ll),
                          _ip(anc), _dp(lwt), _dp(xf), _dp(uo))
    return dict(status=st, ell=ell, ess=ess, loglik=ll.value, anc=anc, lw=lwt, x=xf)


def kf_wk(pb, theta=None):
    P = _Prob(pb)
    th = np.ascontiguousarray(pb.theta[0] if theta is None else theta, dtype=np.float64)
    ell = np.zeros(pb.T)
    ll = lib().orc_kf_wk(P.ref, _dp(th), _dp(ell))
    return ll, ell


def simulate(pb, theta=None, data_seed=None):
    """Truth trajectory [T+1, d] and observations [T, n_obs]."""
    P = _Prob(pb)
    th = np.ascontiguousarray(pb.data_theta if theta is None else theta, dtype=np.float64)
    xt = np.zeros((pb.T + 1, pb.d))
    y = np.zeros((pb.T, len(pb.obs_idx)))
    lib().orc_simulate(P.ref, _dp(th), int(pb.data_seed if data_seed is None else data_seed),
                       _dp(xt), _dp(y))
    return xt, y


def pmmh(pb, N, inputs, chain0=0, n_chains=None, iters=None):
    """Reference PMMH chains (Alg. 3) for chains chain0 .. chain0+n_chains-1."""
    P = _Prob(pb)
    tot = inputs.z.shape[1]
    n_chains = tot - chain0 if n_chains is None else n_chains
    iters = inputs.z.shape[0] if iters is None else iters
    lf0 = np.ascontiguousarray(inputs.log_f0, dtype=np.float64)
    z = np.ascontiguousarray(inputs.z, dtype=np.float64)
    al = np.ascontiguousarray(inputs.alpha, dtype=np.float64)
    lft = np.zeros((iters, n_chains))
    llt = np.zeros((iters, n_chains))
    acc = np.zeros(n_chains, dtype=np.int32)
    lib().orc_pmmh(P.ref, N, chain0, n_chains, tot, iters, _dp(lf0), _dp(z), _dp(al),
                   inputs.step_sd, inputs.f_lo, inputs.f_hi, inputs.sigma, _dp(lft), _dp(llt),
                   _ip(acc))
    return dict(log_f=lft, ll=llt, accepts=acc)


def ndtri(p: float) -> float:
    return lib().orc_ndtri(float(p))


def wk_theta(pb, spec, rczs) -> np.ndarray:
    """Model parameters (a, c, Z, sigma_p, m0, s0) from (R, C, Z, sigma^2)."""
    P = _Prob(pb)
    x = np.ascontiguousarray(rczs, dtype=np.float64)
    th = np.zeros(6)
    lib().orc_wk_theta(P.ref, C.byref(_wk_mh(spec)), _dp(x), _dp(th))
    return th


def wk_log_prior(spec, rczs) -> float:
    x = np.ascontiguousarray(rczs, dtype=np.float64)
    return lib().orc_wk_log_prior(C.byref(_wk_mh(spec)), _dp(x))


def kf_pmmh(pb, spec, inputs, iters=None):
    """Reference marginal Metropolis-Hastings chains on the windkessel's
    (R, C, Z, sigma^2) with the Kalman likelihood (Alg. 3 on Alg. 1)."""
    P = _Prob(pb)
    th0 = np.ascontiguousarray(inputs.theta0, dtype=np.float64)
    n = th0.shape[0]
    iters = inputs.prop.shape[0] if iters is None else iters
    prop = np.ascontiguousarray(inputs.prop[:iters], dtype=np.float64)
    al = np.ascontiguousarray(inputs.alpha[:iters], dtype=np.float64)
    tht = np.zeros((iters, n, 4))
    llt = np.zeros((iters, n))
    acc = np.zeros(n, dtype=np.int32)
    lib().orc_kf_pmmh(P.ref, C.byref(_wk_mh(spec)), n, iters, _dp(th0), _dp(prop), _dp(al),
                      _dp(tht), _dp(llt), _ip(acc))
    return dict(theta=tht, ll=llt, accepts=acc)


def copy_index(k, n_src, n_dst, w) -> int:
    return lib().orc_copy_index(int(k), int(n_src), int(n_dst), int(w))


def smc2(pb, inputs, T=None, n_particles=None):
    """Reference SMC^2 (Alg. 4) over ``inputs.theta0`` for T times; returns
    the final theta-particles, theta-log-weights, likelihoods, accept counts,
    theta-ESS per time, the evidence estimate, per-time traces and the final
    particles [d][sum N]."""
    P = _Prob(pb)
    T = inputs.T if T is None else T
    th0 = np.ascontiguousarray(inputs.theta0, dtype=np.float64)
    B, nth = th0.shape
    n = np.ascontiguousarray(pb.n_particles if n_particles is None else n_particles,
                             dtype=np.int64)
    assert n.shape == (B,)
    z = np.ascontiguousarray(inputs.z, dtype=np.float64)
    la = np.ascontiguousarray(inputs.log_alpha, dtype=np.float64)
    u = np.ascontiguousarray(inputs.u, dtype=np.float64)
    w = np.ascontiguousarray(inputs.w_copy, dtype=np.uint32)
    out = dict(theta=np.zeros((B, nth)), logw=np.zeros(B), loglik=np.zeros(B),
               accepts=np.zeros(B, dtype=np.int32), ess=np.zeros(T),
               anc=np.zeros((T, B), dtype=np.int32), acc=np.zeros((T, B), dtype=np.int32),
               logw_trace=np.zeros((T, B)), theta_trace=np.zeros((T, B, nth)),
               x=np.zeros((pb.d, int(n.sum()))))
    ev = C.c_double()
    st = lib().orc_smc2(P.ref, B, n.ctypes.data_as(C.POINTER(C.c_int64)), nth, _dp(th0), T,
                        _dp(inputs.step_sd), _dp(inputs.lo), _dp(inputs.hi), _dp(z), _dp(la),
                        _dp(u), w.ctypes.data_as(_U), _dp(out["theta"]), _dp(out["logw"]),
                        _dp(out["loglik"]), _ip(out["accepts"]), _dp(out["ess"]),
                        C.byref(ev), _ip(out["anc"]), _ip(out["acc"]), _dp(out["logw_trace"]),
                        _dp(out["theta_trace"]), _dp(out["x"]))
    out["status"] = st
    out["log_evidence"] = ev.value
    return out


def path_slot(seed, s, b, it, N) -> int:
    return lib().orc_path_slot(int(seed), int(s), int(b), int(it), int(N))


def pf_path(pb, theta=None, N=None, b=0, it=0, T=None):
    """Alg. 2 with its single state sample: returns (status, loglik,
    path [T+1, d], particle indices [T+1])."""
    P = _Prob(pb)
    th = np.ascontiguousarray(pb.theta[b] if theta is None else theta, dtype=np.float64)
    N = int(pb.n_particles[b] if N is None else N)
    T = pb.T if T is None else T
    path = np.zeros((T + 1, pb.d))
    idx = np.zeros(T + 1, dtype=np.int64)
    ll = C.c_double()
    st = lib().orc_pf_path(P.ref, _dp(th), N, b, it, T, C.byref(ll), _dp(path),
                           idx.ctypes.data_as(C.POINTER(C.c_int64)))
    return st, ll.value, path, idx


RESAMPLE_SYSTEMATIC, RESAMPLE_STRATIFIED, RESAMPLE_METROPOLIS, RESAMPLE_MULTINOMIAL = 0, 1, 2, 3
RESAMPLE_REJECTION = 4


def strat_u(seed, t, b, it, k) -> float:
    return lib().orc_strat_u(int(seed), int(t), int(b), int(it), int(k))


def stratified_ancestors(lw, seed, t, b=0, it=0):
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    N = lw.shape[0]
    M = lw[lw == lw].max()
    w = np.where(lw == lw, np.exp(lw - M), 0.0)
    W = np.cumsum(w)  # sequential left-to-right sums, as the oracle takes them
    acc = 0.0
    for j in range(N):
        acc = acc + w[j]
        W[j] = acc
    jstar = int(np.flatnonzero(w > 0)[-1])
    a = np.zeros(N, dtype=np.int32)
    lib().orc_stratified_ancestors(N, _dp(W), float(W[-1]), jstar, int(seed), int(t), int(b),
                                   int(it), _ip(a))
    return a


def metropolis_ancestors(lw, steps, seed, t, b=0, it=0):
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    a = np.zeros(lw.shape[0], dtype=np.int32)
    lib().orc_metropolis_ancestors(lw.shape[0], _dp(lw), int(steps), int(seed), int(t), int(b),
                                   int(it), _ip(a))
    return a


def reject_pair(seed, t, b, it, k, r, N):
    j, u = C.c_int64(), C.c_double()
    lib().orc_reject_pair(int(seed), int(t), int(b), int(it), int(k), int(r), int(N),
                          C.byref(j), C.byref(u))
    return j.value, u.value


def rejection_ancestors(lw, seed, t, b=0, it=0):
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    a = np.zeros(lw.shape[0], dtype=np.int32)
    lib().orc_rejection_ancestors(lw.shape[0], _dp(lw), int(seed), int(t), int(b), int(it),
                                  _ip(a))
    return a


def pf_run_ex(pb, theta=None, N=None, b=0, it=0, T=None, resampler=0, steps=0,
              ess_frac=float("inf"), traces=False):
    """Alg. 2 with a resampler choice and ESS-triggered resampling."""
    P = _Prob(pb)
    th = np.ascontiguousarray(pb.theta[b] if theta is None else theta, dtype=np.float64)
    N = int(pb.n_particles[b] if N is None else N)
    T = pb.T if T is None else T
    ell, ess = np.zeros(T), np.zeros(T)
    ll = C.c_double()
    anc = np.zeros((T, N), dtype=np.int32) if traces else None
    lwt = np.zeros((T, N)) if traces else None
    res = np.zeros(T, dtype=np.int32)
    xf = np.zeros((pb.d, N))
    st = lib().orc_pf_run_ex(P.ref, _dp(th), N, b, it, T, int(resampler), int(steps),
                             float(ess_frac), _dp(ell), _dp(ess), C.byref(ll), _ip(anc),
                             _dp(lwt), _ip(res), _dp(xf))
    return dict(status=st, ell=ell, ess=ess, loglik=ll.value, anc=anc, lw=lwt, resampled=res,
                x=xf)


def kf_wk_interval(pb, theta, t, m, V):
    """One Kalman interval; returns (ell_t, m, V)."""
    P = _Prob(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    mm, VV = C.c_double(m), C.c_double(V)
    e = lib().orc_kf_wk_interval(P.ref, _dp(th), int(t), C.byref(mm), C.byref(VV))
    return e, mm.value, VV.value


def smc2_kalman(pb, inputs, T=None):
    """Reference SMC over the parameters with attached Kalman filters
    (windkessel); the same outputs as smc2 plus the final (m, V)."""
    P = _Prob(pb)
    T = inputs.T if T is None else T
    th0 = np.ascontiguousarray(inputs.theta0, dtype=np.float64)
    B, nth = th0.shape
    z = np.ascontiguousarray(inputs.z, dtype=np.float64)
    la = np.ascontiguousarray(inputs.log_alpha, dtype=np.float64)
    u = np.ascontiguousarray(inputs.u, dtype=np.float64)
    out = dict(theta=np.zeros((B, nth)), logw=np.zeros(B), loglik=np.zeros(B),
               accepts=np.zeros(B, dtype=np.int32), ess=np.zeros(T),
               anc=np.zeros((T, B), dtype=np.int32), acc=np.zeros((T, B), dtype=np.int32),
               logw_trace=np.zeros((T, B)), mV=np.zeros((B, 2)))
    ev = C.c_double()
    st = lib().orc_smc2_kalman(P.ref, B, nth, _dp(th0), T, _dp(inputs.step_sd), _dp(inputs.lo),
                               _dp(inputs.hi), _dp(z), _dp(la), _dp(u), _dp(out["theta"]),
                               _dp(out["logw"]), _dp(out["loglik"]), _ip(out["accepts"]),
                               _dp(out["ess"]), C.byref(ev), _ip(out["anc"]), _ip(out["acc"]),
                               _dp(out["logw_trace"]), _dp(out["mV"]))
    out["status"] = st
    out["log_evidence"] = ev.value
    return out


def multi_u(seed, t, b, it, k) -> float:
    return lib().orc_multi_u(int(seed), int(t), int(b), int(it), int(k))


def multinomial_ancestors(lw, seed, t, b=0, it=0):
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    N = lw.shape[0]
    M = lw[lw == lw].max()
    w = np.where(lw == lw, np.exp(lw - M), 0.0)
    W = np.empty(N)
    acc = 0.0
    for j in range(N):
        acc = acc + w[j]
        W[j] = acc
    jstar = int(np.flatnonzero(w > 0)[-1])
    a = np.zeros(N, dtype=np.int32)
    lib().orc_multinomial_ancestors(N, _dp(W), float(W[-1]), jstar, int(seed), int(t), int(b),
                                    int(it), _ip(a))
    return a
