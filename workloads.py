"""Seeded synthetic workloads for the bootstrap particle filter.

This module only builds inputs: model constants, per-filter parameter
vectors, particle counts and the windkessel flow series.  It holds none of
the filter's arithmetic (no propagation, weighting, reduction or
resampling) and imports neither the oracle nor the HIP library, so both
sides can be fed from it.  Observations are *not* made here: simulating
the model is model arithmetic, so each side has its own simulator.

The five workloads follow the paper's two examples:

* windkessel (Sec. 2.1.1, eqs. 2-windkessel / 3-windkessel): a scalar
  linear-Gaussian state with an exact Kalman likelihood;
* Lorenz '96 (Sec. 2.1.2, eq. lorenz96-sde): a chaotic cyclic system
  integrated with fixed-step RK4.

Parameter layouts (one row of ``theta`` per filter):

* windkessel: ``(a, c, Z, sigma_p, m0, s0)`` with ``a = exp(-h/(R C))``
  and ``c = R (1 - a)``, so the exponential of the exact step
  (eq. 2-windkessel) is evaluated once, here, and passed as data;
* Lorenz '96: ``(F, sigma)``; the per-substep noise sd is ``sigma*sqrt(h)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

MODEL_WK = 1
MODEL_L96 = 2
MODEL_L96_STAGE = 3  # Lorenz '96 with the noise inside the RK4 stages (the paper's form)
FP64 = 0
FP32_MIXED = 1
FP32_ACCURATE = 2

N_THETA = {MODEL_WK: 6, MODEL_L96: 2, MODEL_L96_STAGE: 2}


@dataclasses.dataclass
class Problem:
    """One filtering problem: model, sizes, parameters and seeds.

    ``theta`` has shape ``[B, n_theta]``; ``n_particles`` has shape ``[B]``.
    ``data_theta`` is the parameter vector the synthetic truth is simulated
    with; ``obs`` is filled in by whichever simulator the caller uses.
    """
    name: str
    model: int
    d: int
    K: int
    h: float
    obs_idx: np.ndarray
    obs_sd: float
    T: int
    theta: np.ndarray
    n_particles: np.ndarray
    q: Optional[np.ndarray]
    seed: int
    data_seed: int
    data_theta: np.ndarray
    precision: int = FP64
    obs: Optional[np.ndarray] = None

    @property
    def B(self) -> int:
        return int(self.theta.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_idx.shape[0])

    @property
    def n_theta(self) -> int:
        return int(self.theta.shape[1])

    def with_obs(self, obs: np.ndarray) -> "Problem":
        obs = np.ascontiguousarray(obs, dtype=np.float64).reshape(self.T, self.n_obs)
        return dataclasses.replace(self, obs=obs)


# ---------------------------------------------------------------- windkessel

def wk_flow(n_steps: int, h: float, peak: float = 400.0, period: float = 0.8) -> np.ndarray:
    """Flow input F(t_n) = peak*max(0, sin(2*pi*t_n/period))^2, t_n = n*h.

    A periodic pulse standing in for the paper's prescribed flow (eq. flow),
    held constant over each step [t_n, t_n + h).  Returns n_steps + 1
    values, n = 0..n_steps.
    """
    t = np.arange(n_steps + 1, dtype=np.float64) * h
    s = np.sin(2.0 * np.pi * t / period)
    return peak * np.maximum(0.0, s) ** 2


def wk_theta(R: float, C: float, Z: float, sigma_p: float, m0: float, s0: float,
             h: float) -> np.ndarray:
    a = math.exp(-h / (R * C))
    return np.array([a, R * (1.0 - a), Z, sigma_p, m0, s0], dtype=np.float64)


def windkessel(N: int = 1024, T: int = 100, K: int = 10, seed: int = 0, data_seed: int = 1,
               precision: int = FP64, B: int = 1) -> Problem:
    """Linear-Gaussian windkessel workload: R=1, C=1.5, h=0.01, Z=0.03,
    process sd 0.5 on the pressure, observation sd 1, initial N(90, 15^2)
    (the paper's initial block gives mean 90, sd 15)."""
    h = 0.01
    th = wk_theta(1.0, 1.5, 0.03, 0.5, 90.0, 15.0, h)
    return Problem(
        name=f"windkessel_N{N}_T{T}", model=MODEL_WK, d=1, K=K, h=h,
        obs_idx=np.zeros(1, dtype=np.int32), obs_sd=1.0, T=T,
        theta=np.tile(th, (B, 1)), n_particles=np.full(B, N, dtype=np.int64),
        q=wk_flow(T * K, h), seed=seed, data_seed=data_seed, data_theta=th.copy(),
        precision=precision)


def wk_flow_paper(n_steps: int, h: float, f_max: float = 500.0, t_s: float = 0.3,
                  t_d: float = 0.5) -> np.ndarray:
    """The paper's prescribed flow (eq. flow): F(t) = f_max sin^2(pi t /
    (t_s + t_d)) while t mod (t_s + t_d) lies in [0, t_s] (systole), else 0
    (diastole); sampled at t_n = n h and held over each step.  n_steps + 1
    values.  "mod" is read as the remainder."""
    t = np.arange(n_steps + 1, dtype=np.float64) * h
    period = t_s + t_d
    systole = np.mod(t, period) <= t_s
    return np.where(systole, f_max * np.sin(np.pi * t / period) ** 2, 0.0)


def wk_theta_paper(R: float, C: float, Z: float, sigma2: float, m0: float, s0: float,
                   h: float) -> np.ndarray:
    """The paper's parameters (R, C, Z, sigma^2) with the noise on the flow:
    P_p <- a P_p + c (F + xi), xi ~ N(0, sigma^2), is the pressure noise of sd
    c sigma, so sigma_p = R (1 - a) sqrt(sigma^2)."""
    a = math.exp(-h / (R * C))
    c = R * (1.0 - a)
    return np.array([a, c, Z, c * math.sqrt(sigma2), m0, s0], dtype=np.float64)


def windkessel_paper(N: int = 1024, T: int = 100, K: int = 10, seed: int = 0,
                     data_seed: int = 1, precision: int = FP64, B: int = 1, R: float = 1.0,
                     C: float = 1.5, Z: float = 0.03, sigma2: float = 25.0) -> Problem:
    """The paper's windkessel example (Sec. 2.1.1): flow with f_max 500,
    systole 0.3 s, diastole 0.5 s; noise on the flow with variance sigma^2;
    observation sd 2; P_p(t_0) ~ N(90, 15); dt = 0.01."""
    h = 0.01
    th = wk_theta_paper(R, C, Z, sigma2, 90.0, 15.0, h)
    return Problem(
        name=f"windkessel_paper_N{N}_T{T}", model=MODEL_WK, d=1, K=K, h=h,
        obs_idx=np.zeros(1, dtype=np.int32), obs_sd=2.0, T=T,
        theta=np.tile(th, (B, 1)), n_particles=np.full(B, N, dtype=np.int64),
        q=wk_flow_paper(T * K, h), seed=seed, data_seed=data_seed, data_theta=th.copy(),
        precision=precision)


# ---------------------------------------------------------------- Lorenz '96

def lorenz96(d: int = 8, N: int = 65536, T: int = 200, K: int = 8, F: float = 8.0,
             sigma: float = 0.1, obs_every: int = 1, seed: int = 0, data_seed: int = 1,
             precision: int = FP64, B: int = 1, stage_noise: bool = False) -> Problem:
    """Stochastic Lorenz '96 with RK4 step h=0.05, K substeps between
    observations, observation sd 0.5 on components 0, obs_every, 2*obs_every...
    stage_noise: the paper's form, the noise inside the RK4 stages."""
    th = np.array([F, sigma], dtype=np.float64)
    idx = np.arange(0, d, obs_every, dtype=np.int32)
    return Problem(
        name=f"lorenz96{'s' if stage_noise else ''}_d{d}_N{N}_T{T}",
        model=MODEL_L96_STAGE if stage_noise else MODEL_L96, d=d, K=K, h=0.05,
        obs_idx=idx, obs_sd=0.5, T=T, theta=np.tile(th, (B, 1)),
        n_particles=np.full(B, N, dtype=np.int64), q=None, seed=seed,
        data_seed=data_seed, data_theta=th.copy(), precision=precision)


def batched_thetas(B: int, seed: int = 2, f_lo: float = 6.0, f_hi: float = 10.0,
                   s_lo: float = 0.05, s_hi: float = 0.3,
                   counts=(256, 512, 1024, 2048, 4096, 8192)):
    """Parameter particles for the batched (SMC^2-style) workload:
    F ~ U(f_lo, f_hi), sigma ~ U(s_lo, s_hi), N_b uniform over ``counts``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    F = rng.uniform(f_lo, f_hi, size=B)
    s = rng.uniform(s_lo, s_hi, size=B)
    n = rng.choice(np.asarray(counts, dtype=np.int64), size=B)
    return np.stack([F, s], axis=1).astype(np.float64), n.astype(np.int64)


def lorenz96_batched(B: int = 512, T: int = 200, seed: int = 0, data_seed: int = 1,
                     theta_seed: int = 2, precision: int = FP32_MIXED,
                     counts=(256, 512, 1024, 2048, 4096, 8192)) -> Problem:
    """B filters, each with its own (F_b, sigma_b) and N_b, all on the
    d=8 Lorenz '96 data set (truth F=8, sigma=0.1)."""
    base = lorenz96(d=8, N=1, T=T, seed=seed, data_seed=data_seed, precision=precision)
    th, n = batched_thetas(B, theta_seed, counts=counts)
    return dataclasses.replace(base, name=f"lorenz96_batched_B{B}_T{T}", theta=th,
                               n_particles=n)


@dataclasses.dataclass
class PmmhInputs:
    """Random numbers the marginal Metropolis-Hastings layer draws, passed in
    as inputs: initial log F per chain, proposal normals and acceptance
    uniforms per (iteration, chain)."""
    log_f0: np.ndarray        # [chains]
    z: np.ndarray             # [iters, chains]
    alpha: np.ndarray         # [iters, chains], in (0, 1)
    step_sd: float
    f_lo: float
    f_hi: float
    sigma: float


def pmmh_inputs(chains: int = 64, iters: int = 2000, seed: int = 3, step_sd: float = 0.05,
                f_lo: float = 6.0, f_hi: float = 10.0, sigma: float = 0.1) -> PmmhInputs:
    rng = np.random.Generator(np.random.PCG64(seed))
    f0 = rng.uniform(f_lo, f_hi, size=chains)
    z = rng.standard_normal(size=(iters, chains))
    # strictly inside (0, 1): log(alpha) is finite
    alpha = (rng.integers(0, 2 ** 32, size=(iters, chains), dtype=np.uint64).astype(np.float64)
             + 0.5) * 2.0 ** -32
    return PmmhInputs(np.log(f0), z, alpha, step_sd, f_lo, f_hi, sigma)


@dataclasses.dataclass
class WkMh:
    """Priors and proposals of marginal Metropolis-Hastings on the
    windkessel's (R, C, Z, sigma^2) (Sec. 2.1.1, the parameter and proposal
    blocks), with the initial state N(m0, s0^2).  Gamma and Inverse-Gamma are
    read as (shape, scale).  A zero step sd (or a zero ``ig_prop_factor``)
    keeps that parameter fixed."""
    prior_shape: tuple = (2.0, 2.0, 2.0)
    prior_scale: tuple = (0.9, 1.5, 0.03)
    ig_shape: float = 2.0
    ig_scale: float = 25.0
    step_sd: tuple = (0.03, 0.1, 0.002)
    ig_prop_shape: float = 2.0
    ig_prop_factor: float = 3.0
    m0: float = 90.0
    s0: float = 15.0


@dataclasses.dataclass
class WkMhInputs:
    """Random numbers of the windkessel chains, passed in as inputs:
    ``theta0`` [chains, 4] the initial (R, C, Z, sigma^2); ``prop``
    [iters, chains, 4]: uniforms in (0, 1) for R, C, Z and a
    Gamma(ig_prop_shape, 1) variate for sigma^2; ``alpha`` [iters, chains] in
    (0, 1)."""
    theta0: np.ndarray
    prop: np.ndarray
    alpha: np.ndarray


def _open_uniforms(rng, shape) -> np.ndarray:
    """Uniforms strictly inside (0, 1): (k + 1/2) 2^-32 for a 32-bit k."""
    return (rng.integers(0, 2 ** 32, size=shape, dtype=np.uint64).astype(np.float64)
            + 0.5) * 2.0 ** -32


def wk_mh_prior_draws(spec: WkMh, n: int, rng) -> np.ndarray:
    """n draws of (R, C, Z, sigma^2) from the prior."""
    out = np.zeros((n, 4))
    for k in range(3):
        out[:, k] = rng.gamma(spec.prior_shape[k], spec.prior_scale[k], size=n)
    out[:, 3] = spec.ig_scale / rng.gamma(spec.ig_shape, 1.0, size=n)
    return out


def wk_mh_inputs(spec: WkMh, chains: int = 64, iters: int = 1000, seed: int = 5,
                 theta0: Optional[np.ndarray] = None) -> WkMhInputs:
    """Inputs for ``chains`` chains of ``iters`` iterations; without
    ``theta0`` the chains start from prior draws."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if theta0 is None:
        theta0 = wk_mh_prior_draws(spec, chains, rng)
    theta0 = np.array(np.broadcast_to(theta0, (chains, 4)), dtype=np.float64, order="C")
    prop = np.zeros((iters, chains, 4))
    prop[:, :, :3] = _open_uniforms(rng, (iters, chains, 3))
    prop[:, :, 3] = rng.gamma(spec.ig_prop_shape, 1.0, size=(iters, chains))
    return WkMhInputs(theta0, prop, _open_uniforms(rng, (iters, chains)))


@dataclasses.dataclass
class Smc2Inputs:
    """Random numbers the SMC^2 parameter layer (Alg. 4) draws, passed in as
    inputs, plus its random walk and prior box.

    ``theta0`` [B, n_theta]: the initial theta-particles (drawn from the prior);
    ``z`` [T, B, n_theta]: proposal normals; ``log_alpha`` [T, B]: logs of the
    acceptance uniforms; ``u`` [T]: the theta-resampling uniform of each time;
    ``w_copy`` [T, B]: 32-bit words placing the whole-filter copies.
    ``step_sd`` [n_theta] is the random-walk sd (0 keeps a parameter fixed);
    the prior is uniform on [lo, hi] for every moved parameter."""
    theta0: np.ndarray
    z: np.ndarray
    log_alpha: np.ndarray
    u: np.ndarray
    w_copy: np.ndarray
    step_sd: np.ndarray
    lo: np.ndarray
    hi: np.ndarray

    @property
    def T(self) -> int:
        return int(self.z.shape[0])


def smc2_inputs(theta0: np.ndarray, T: int, step_sd, lo, hi, seed: int = 4) -> Smc2Inputs:
    """Inputs for T times of SMC^2 over the theta-particles ``theta0``."""
    theta0 = np.ascontiguousarray(theta0, dtype=np.float64)
    B, n_theta = theta0.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal(size=(T, B, n_theta))
    # uniforms strictly inside (0, 1), so their logs are finite
    alpha = (rng.integers(0, 2 ** 32, size=(T, B), dtype=np.uint64).astype(np.float64)
             + 0.5) * 2.0 ** -32
    u = rng.integers(0, 2 ** 32, size=T, dtype=np.uint64).astype(np.float64) * 2.0 ** -32
    w = rng.integers(0, 2 ** 32, size=(T, B), dtype=np.uint64).astype(np.uint32)
    return Smc2Inputs(theta0, z, np.log(alpha), u, w,
                      np.ascontiguousarray(step_sd, dtype=np.float64).reshape(n_theta),
                      np.ascontiguousarray(lo, dtype=np.float64).reshape(n_theta),
                      np.ascontiguousarray(hi, dtype=np.float64).reshape(n_theta))


def smc2_l96_inputs(theta0: np.ndarray, T: int, seed: int = 4, step_f: float = 0.1,
                    step_s: float = 0.01, f_lo: float = 6.0, f_hi: float = 10.0,
                    s_lo: float = 0.05, s_hi: float = 0.3) -> Smc2Inputs:
    """Lorenz '96 SMC^2: random walk on (F, sigma) within the prior box the
    batched workload's parameters are drawn from."""
    return smc2_inputs(theta0, T, [step_f, step_s], [f_lo, s_lo], [f_hi, s_hi], seed)


def smc2_wk_m0_inputs(base_theta: np.ndarray, B: int, T: int, seed: int = 5,
                      m0_lo: float = 70.0, m0_hi: float = 110.0,
                      step: float = 3.0) -> Smc2Inputs:
    """Windkessel SMC^2 over the initial-pressure mean m0 only (index 4), with
    prior U(m0_lo, m0_hi): the evidence is then a one-dimensional integral of
    the Kalman likelihood."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    th = np.tile(np.asarray(base_theta, dtype=np.float64), (B, 1))
    th[:, 4] = rng.uniform(m0_lo, m0_hi, size=B)
    step_sd = np.zeros(th.shape[1])
    step_sd[4] = step
    lo = np.full(th.shape[1], -np.inf)
    hi = np.full(th.shape[1], np.inf)
    lo[4], hi[4] = m0_lo, m0_hi
    return smc2_inputs(th, T, step_sd, lo, hi, seed)


# ---------------------------------------------------------------- named configs

def config(name: str, **kw) -> Problem:
    """The named workloads, and smaller variants of them through keyword
    arguments: "windkessel" (the linear-Gaussian windkessel, N = 1024),
    "lorenz96_d8" (one Lorenz '96 filter, d = 8, N = 65,536, T = 200),
    "lorenz96_d40_large" (one filter, d = 40, N = 2^20, T = 500, every second
    component observed), "lorenz96_d8_batched" (512 filters of uneven N) and
    "lorenz96_d8_chains" (64 filters of N = 4096, the PMMH chains' shape)."""
    if name == "windkessel":
        return windkessel(**kw)
    if name == "lorenz96_d8":
        return lorenz96(d=8, N=kw.pop("N", 65536), T=kw.pop("T", 200), **kw)
    if name == "lorenz96_d40_large":
        return lorenz96(d=40, N=kw.pop("N", 1 << 20), T=kw.pop("T", 500), obs_every=2,
                        precision=kw.pop("precision", FP32_MIXED), **kw)
    if name == "lorenz96_d8_batched":
        return lorenz96_batched(**kw)
    if name == "lorenz96_d8_chains":
        chains = kw.pop("chains", 64)
        N = kw.pop("N", 4096)
        return lorenz96(d=8, N=N, T=kw.pop("T", 200), B=chains,
                        precision=kw.pop("precision", FP32_MIXED), **kw)
    raise KeyError(name)
