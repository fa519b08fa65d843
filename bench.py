"""Throughput of the MI355X bootstrap particle filter (one JSON line on stdout).

A step is one pass of the whole hot path over the headline batch: every
filter re-initialised (x(t0) drawn), then T observation intervals of
propagate (K substeps) + weight + likelihood increment + ESS + systematic
resampling + ancestor gather (graph replays or eager launches, as the
autotuner measured faster on this host), then the
likelihoods read back (the only host synchronisation).  The rate is in
particle-steps/s, a particle-step being one particle through one
observation interval.  Inputs (observations, parameters) are resident in
HBM before timing starts; the data are simulated on the GPU from the model.

Headline (``value``): the FP32 batched form on the batched workload — 512
Lorenz '96 (d = 8) filters with F ~ U(6, 10), sigma ~ U(0.05, 0.3) and
particle counts uniform over {256, ..., 8192}, T = 200 — next to the FP64
plain filter (one filter at a time, per-filter kernels) and the FP64 batched
form on the same workload, and the FP32 error per step measured at full size
by teacher forcing against the FP64 path.  Secondary legs: the single filter
(d = 8, N = 65,536), the large filter (d = 40, N = 2^20: resample + gather
against HBM, propagation against the FP32 vector peak), and marginal
Metropolis-Hastings chains (64 x N = 4096), whose acceptance is compared
with the oracle's chains on the same inputs.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak
FP32_PEAK_TFLOPS = 157.3
# VALU issue peak in lane-operations/s: the FP32 vector peak counts an FMA as
# 2 FLOP, i.e. 78.6 T lane-operations/s (256 CUs x 2.4 GHz x 128); every VALU
# instruction is counted as one lane-operation.
VALU_PEAK_TOPS = 157.3 / 2
# the per-step log-likelihood bound of the FP32 form (absolute)
FP32_ELL_BOUND = 1e-4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# the sources each profiled kernel family is built from
BATCHED_SOURCES = ("paper_1306_3277_amd/csrc/pf_batched.hip",
                   "paper_1306_3277_amd/csrc/pf_device.hpp",
                   "paper_1306_3277_amd/csrc/pf_internal.hpp")
PLAIN_SOURCES = ("paper_1306_3277_amd/csrc/pf_kernels.hip",
                 "paper_1306_3277_amd/csrc/pf_device.hpp",
                 "paper_1306_3277_amd/csrc/pf_internal.hpp")


def kernel_sources_sha256(sources=BATCHED_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic(summary: str):
    """HBM bytes per launch of a kernel from its committed counter summary
    under profiles/ (memory counters scaled by a plain copy), or None when
    the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                fields[k] = v.strip("` ")
    if fields.get("kernel sources sha256") != kernel_sources_sha256(BATCHED_SOURCES):
        return None
    try:
        return float(fields["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def valu_slots_per_particle_step(model: int, d: int, K: int, n_obs: int, fp32: bool) -> float:
    """Algorithmic VALU operations (lane-instructions) one particle needs for
    one observation interval.  Per generator call (4 words): 10 Philox rounds
    of 2 wide multiplies + 2 three-input xors = 40; FP32 normals: 4 uniforms
    x 2 + 2 Box-Muller pairs x 5 (log, scale, sqrt, cos, sin) = 18; FP64
    normals: 4 uniforms x 2 + 2 pairs x 95 (own log ~32, sincos ~45, sqrt
    ~12, products) = 198.  Lorenz '96 per component per substep, FP32: 4
    stages x (drift 2 + increment 1 + stage input 1) - 1 + 2 (x + cF) + the
    noise (1) and the state update (1) = 19; FP64 (the oracle's expression
    tree, no fusion): 30.  Weight: 3 FP64 operations per observed component
    + 4."""
    philox = 40
    bm_call = 18 if fp32 else 198
    if model == W.MODEL_WK:
        per_sub = philox + bm_call // 2 + (4 if fp32 else 5)
        return K * per_sub + 8
    rk4 = 19 if fp32 else 30
    per_sub = (d // 4) * (philox + bm_call) + rk4 * d
    return K * per_sub + 3 * n_obs + 4


def model_flop_per_particle_step(model: int, d: int, K: int, n_obs: int) -> int:
    """The propagation's algorithmic floating-point work per particle-step,
    random numbers excluded: Lorenz '96 RK4 about 30 FLOP per component per
    substep (four drift evaluations of 3 operations plus the stage inputs and
    the weighted sum), and 4 per observed component for the weight; the
    windkessel step 5 per substep."""
    if model == W.MODEL_WK:
        return 5 * K + 4 * n_obs
    return 30 * d * K + 4 * n_obs


def plain_propagate_bytes(d: int, sx: int, slw: int) -> int:
    """Algorithmic HBM bytes per particle of one plain-layout propagation:
    read the pending ancestor's d state components (the gather of the last
    resampling) and write the d propagated ones and the log-weight; read
    and clear the mark, write the ancestor."""
    return 2 * d * sx + slw + 4 + 4 + 4


def plain_scan_bytes(slw: int) -> int:
    """Algorithmic HBM bytes per particle of the plain-layout scan: read the
    log-weight, write at most one mark."""
    return slw + 4


class Runner:
    """Drives one handle for n consecutive intervals, restarting at T."""

    def __init__(self, f, T):
        self.f, self.T, self.t = f, T, 0

    def run(self, n, graph=True):
        done = 0
        while done < n:
            if self.t >= self.T:
                self.f.reset(0)
                self.t = 0
            k = min(n - done, self.T - self.t)
            if graph:
                self.f.graph_run(k)
            else:
                self.f.advance(k)
            self.t += k
            done += k

    def restart(self):
        self.f.reset(0)
        self.t = 0


def timed(torch, runner, steps, warmup):
    runner.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runner.run(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def filter_passes(f, T, n):
    """n passes of the whole hot path over the workload: every filter
    re-initialised, T intervals replayed from the captured graphs, the
    likelihoods read back (which synchronises the stream)."""
    for _ in range(n):
        f.reset(0)
        f.graph_run(T)
        f.loglik(allow_numeric=True)


def timed_passes(torch, f, T, steps, warmup):
    filter_passes(f, T, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    filter_passes(f, T, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_times(runner, steps):
    """Per-kernel mean durations (us) from HIP events on the handle's stream."""
    f = runner.f
    runner.restart()
    f.timing(True)
    runner.run(steps, graph=False)
    tm = f.timing_get()
    f.timing(False)
    out = {}
    for k in ("propagate", "combine", "scan", "gather", "batched"):
        n = tm[f"{k}_launches"]
        out[k] = tm[f"{k}_ms"] / n * 1e3 if n else 0.0
    out["steps"] = steps
    return out


def teacher_forced_fp32_error(pfm, pb, stream, steps, precision):
    """|ell_t(FP32 batched) - ell_t(FP64 plain)| for every filter and interval,
    each interval started on both sides from the FP64 path's particles rounded
    to FP32 (the FP64 path is the one checked bit for bit against the oracle),
    for the given FP32 form.  Returns the errors [steps, B], the FP64
    increments and the FP64 ESS."""
    f64 = pfm.Filter(pb, precision=W.FP64, layout=pfm.PF_LAYOUT_PLAIN, stream=stream)
    f32 = pfm.Filter(pb, precision=precision, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    err, ell, ess = [], [], []
    for t in range(steps):
        x = f64.get_state().astype(np.float32).astype(np.float64)
        f64.set_state(x)
        f32.set_state(x)
        f64.step()
        f32.step()
        e64, s64 = f64.trace()
        e32, _ = f32.trace()
        err.append(np.abs(e32[:, t] - e64[:, t]))
        ell.append(e64[:, t])
        ess.append(s64[:, t])
        f64.resample()
        f32.resample()
    f64.close()
    f32.close()
    return np.array(err), np.array(ell), np.array(ess)


def tf_summary(err, ell, ess, bound):
    """Distribution of the teacher-forced errors over (interval, filter) pairs
    against the absolute bound, with the pairs that exceed it listed."""
    over = np.argsort(-err.ravel())
    n_over = int(np.sum(err > bound))
    ok = ess >= 2.0
    return {"bound": bound, "max_abs": float(err.max()),
            "p99_abs": float(np.quantile(err, 0.99)), "median_abs": float(np.median(err)),
            "pairs": int(err.size), "pairs_over_bound": n_over,
            "frac_within_bound": float(np.mean(err <= bound)),
            "max_abs_where_ess_ge_2": float(err[ok].max()) if ok.any() else None,
            "pairs_over_bound_where_ess_ge_2": int(np.sum(err[ok] > bound)),
            "worst": [{"err": float(err.ravel()[i]), "ell": float(ell.ravel()[i]),
                       "ess": float(ess.ravel()[i])} for i in over[:max(3, min(n_over, 12))]]}


def plain_hbm(us, byt, n):
    gbs = byt * n / (us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "bytes_per_particle": byt, "us": us}


def large_filter_leg(torch, pfm, stream):
    """One Lorenz '96 (d = 40) filter of 2^20 particles, FP32 mixed.  An
    interval is three kernels: the propagation (which gathers the previous
    interval's particles through the pending ancestors), the combine of its
    4,096 block partials, and the scan that marks the new ancestors.  The
    propagation is priced against the FP32 vector peak and against HBM (it
    moves the state twice), the scan against HBM.  Also measured with spread
    weights (an observation sd of 20 on the same data: ESS near N, so the
    gather reads every particle's row rather than a few heavy particles'
    from cache)."""
    big = W.config("lorenz96_d40_large")
    _, yb = pfm.simulate(big, stream=stream)
    big = big.with_obs(yb)
    nb = int(big.n_particles[0])
    flop_b = model_flop_per_particle_step(big.model, big.d, big.K, big.n_obs)
    slots_b = valu_slots_per_particle_step(big.model, big.d, big.K, big.n_obs, True)

    def measure(pb):
        f = pfm.Filter(pb, stream=stream)
        r = Runner(f, pb.T)
        r.run(3)
        kt = kernel_times(r, 10)
        r.restart()
        dt = min(timed(torch, r, 40, 8) for _ in range(3))  # the fastest of three runs
        _, ess, _ = f.loglik()
        ach = flop_b * nb / (kt["propagate"] * 1e-6) / 1e12
        sl = slots_b * nb / (kt["propagate"] * 1e-6) / 1e12
        out = {
            "us_per_step": dt / 40 * 1e6, "particle_steps_per_s": nb * 40 / dt,
            "ess_last_step": float(ess[0]),
            "propagate": {"bound": "alu", "achieved": ach, "peak": FP32_PEAK_TFLOPS,
                          "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS,
                          "us": kt["propagate"], "flop_per_particle_step": flop_b,
                          "issue_slots": {"ops_per_particle_step": slots_b, "achieved": sl,
                                          "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
                                          "frac": sl / VALU_PEAK_TOPS},
                          "hbm": plain_hbm(kt["propagate"], plain_propagate_bytes(big.d, 4, 8),
                                           nb)},
            "combine_us": kt["combine"],
            "scan": plain_hbm(kt["scan"], plain_scan_bytes(8), nb),
        }
        return f, r, out

    fb, rb, leg = measure(big)
    variants = {}
    # (rejection resampling is left out here: with an ESS of a few particles
    # out of 2^20 each output needs ~N w_max / sum w ~ 1e5 attempts)
    for name, scheme, msteps in (("stratified", 1, 0), ("multinomial", 3, 0),
                                 ("metropolis_8", 2, 8)):
        fb.set_resampler(scheme, msteps)
        rb.restart()
        kv = kernel_times(rb, 10)
        variants[name] = {"scan_us": kv["scan"], "ancestors_us": kv["gather"],
                          "propagate_us": kv["propagate"]}
    fb.close()
    spread = dataclasses.replace(big, obs_sd=20.0)
    fs, rs, leg_s = measure(spread)
    variants_spread = {}
    for name, scheme, msteps in (("stratified", 1, 0), ("multinomial", 3, 0),
                                 ("metropolis_8", 2, 8), ("rejection", 4, 0)):
        fs.set_resampler(scheme, msteps)
        rs.restart()
        kv = kernel_times(rs, 10)
        variants_spread[name] = {"scan_us": kv["scan"], "ancestors_us": kv["gather"],
                                 "propagate_us": kv["propagate"]}
    fs.close()
    leg_s["obs_sd"] = spread.obs_sd
    leg.update({"workload": big.name, "particles": nb, "spread_weights": leg_s,
                "resample_variants": variants,
                "resample_variants_spread_weights": variants_spread})
    fmt = lambda v: ", ".join(f"{k} {x['scan_us'] + x['ancestors_us']:.1f}"
                              for k, x in v.items())
    log("[bench] large filter resampling variants (scan + ancestor kernels, us): " +
        fmt(variants) + "; spread weights: " + fmt(variants_spread))
    for name, lg in (("workload", leg), ("spread", leg_s)):
        p = lg["propagate"]
        log(f"[bench] large filter ({name} weights, ESS {lg['ess_last_step']:.3g}): "
            f"{lg['us_per_step']:.1f} us/interval; propagate+gather {p['us']:.1f} us "
            f"({p['frac']:.0%} of the FP32 peak, {p['hbm']['achieved']:.0f} GB/s), combine "
            f"{lg['combine_us']:.1f} us, scan {lg['scan']['us']:.1f} us")
    return leg


RESAMPLER_CASES = [("systematic", 0, 0, float("inf")), ("stratified", 1, 0, float("inf")),
                   ("multinomial", 3, 0, float("inf")), ("metropolis_8", 2, 8, float("inf")),
                   ("rejection", 4, 0, float("inf")), ("systematic_ess0.5", 0, 0, 0.5)]
# rejection resampling costs ~N attempts per output in a collapsed filter
# (about a quarter of this workload's filters): time only the first
# intervals after one eight-interval warm-up
REJECTION_STEPS, REJECTION_WARMUP = 40, 8


def resampler_leg(torch, pfm, pb, stream, threads, groups, steps=200):
    """Interval time of the batched workload (fast FP32 form, graph replay)
    with each resampling variant, after a whole warm-up pass (rejection
    resampling: 40 intervals after 8)."""
    out = {}
    for name, scheme, msteps, frac in RESAMPLER_CASES:
        f = pfm.Filter(pb, precision=W.FP32_MIXED, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
        f.set_tuning(threads, groups)
        f.set_resampler(scheme, msteps, frac)
        r = Runner(f, pb.T)
        n, w = (REJECTION_STEPS, REJECTION_WARMUP) if scheme == 4 else (steps, pb.T)
        dt = timed(torch, r, n, w)
        f.close()
        out[name] = {"us_per_interval": dt / n * 1e6,
                     "particle_steps_per_s": int(pb.n_particles.sum()) * n / dt}
        if scheme == 4:
            out[name]["intervals"] = f"{w + 1}-{w + n}"
    log("[bench] resamplers (batched, us/interval): " +
        ", ".join(f"{k} {v['us_per_interval']:.1f}" for k, v in out.items()))
    return out


def models_leg(torch, pfm, pb, stream, threads, groups, steps=100):
    """The paper's model forms and the Kalman filter: the batched workload
    with the noise inside the RK4 stages (FP32 mixed), the exact windkessel
    likelihood of 512 parameter sets, and SMC over the windkessel m0 with
    attached Kalman filters."""
    out = {}
    ps = dataclasses.replace(pb, model=W.MODEL_L96_STAGE)
    f = pfm.Filter(ps, precision=W.FP32_MIXED, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    f.set_tuning(threads, groups)
    dt = timed(torch, Runner(f, ps.T), steps, 10)
    f.close()
    out["lorenz96_stage_noise_batched"] = {
        "us_per_interval": dt / steps * 1e6,
        "particle_steps_per_s": int(ps.n_particles.sum()) * steps / dt}
    wk = W.windkessel(N=64, T=100, B=512)
    _, y = pfm.simulate(wk, stream=stream)
    wk = wk.with_obs(y)
    inp = W.smc2_wk_m0_inputs(wk.theta[0], 512, wk.T, seed=9)
    wk = dataclasses.replace(wk, theta=inp.theta0)
    fk = pfm.Filter(wk, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    fk.kalman()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        fk.kalman()
    dtk = (time.perf_counter() - t0) / 10
    fk.smc2(None, inp, T=3, kalman=True, traces=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rk = fk.smc2(None, inp, kalman=True, traces=False)
    dts = time.perf_counter() - t0
    fk.close()
    out["kalman_windkessel_512_filters_T100"] = {"ms_per_call": dtk * 1e3}
    out["smc_kalman_windkessel_512_theta_T100"] = {
        "seconds": dts, "log_evidence": rk["log_evidence"],
        "accept_rate": float(rk["accepts"].sum() / (512 * wk.T))}
    out["kalman_mh_windkessel_512_chains"] = kalman_mh_leg(torch, pfm, stream)
    log(f"[bench] models: L96 stage noise {out['lorenz96_stage_noise_batched']['us_per_interval']:.1f} "
        f"us/interval; Kalman 512 x T100 {dtk * 1e3:.3f} ms; SMC with Kalman filters "
        f"512 x T100 {dts * 1e3:.1f} ms; Kalman MH "
        f"{out['kalman_mh_windkessel_512_chains']['chain_iterations_per_s']:.3e} iterations/s")
    return out


def kalman_mh_leg(torch, pfm, stream, B=512, iters=1000, T=100):
    """Marginal Metropolis-Hastings on the paper's windkessel (R, C, Z,
    sigma^2) with the exact Kalman likelihood: B chains x iters iterations
    on T observations, the paper's priors and proposals, every chain started
    within 20% of the data's parameters; inputs resident on the device."""
    wk = W.windkessel_paper(N=1, T=T, B=B)
    _, y = pfm.simulate(wk, stream=stream)
    wk = wk.with_obs(y)
    spec = W.WkMh()
    truth = np.array([1.0, 1.5, 0.03, 25.0])
    rng = np.random.default_rng(17)
    inp = W.wk_mh_inputs(spec, chains=B, iters=iters, seed=18,
                         theta0=truth * rng.uniform(0.8, 1.2, size=(B, 4)))
    dev = torch.device("cuda")
    th0, pr, al = (torch.from_numpy(a).to(dev) for a in (inp.theta0, inp.prop, inp.alpha))
    f = pfm.Filter(wk, precision=pfm.PF_FP64, stream=stream)
    res = f.kalman_pmmh(spec, th0, pr, al, iters=20)
    out = None
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = f.kalman_pmmh(spec, th0, pr, al, out=out)
        times.append(time.perf_counter() - t0)
    f.close()
    dt = min(times)
    theta = out["theta"][iters // 2:].reshape(-1, 4).cpu().numpy()
    acc = out["accepts"].cpu().numpy()
    del res
    substeps = B * (iters + 1) * T * wk.K
    return {"chains": B, "iterations": iters, "T": T, "K": wk.K, "seconds": dt,
            "chain_iterations_per_s": B * iters / dt, "kalman_substeps_per_s": substeps / dt,
            "accept_rate": float(acc.sum() / (B * iters)),
            "posterior_mean_second_half": dict(zip(["R", "C", "Z", "sigma2"],
                                                   theta.mean(0).round(4).tolist())),
            "truth": dict(zip(["R", "C", "Z", "sigma2"], truth.tolist()))}


def path_leg(torch, pfm, pb, stream, threads, groups, dt_plain_interval):
    """The headline workload with ancestry storage attached (the stepping
    kernels also store every interval's propagated particles and ancestors
    into the history), then the state sample of every filter (Alg. 2, last
    lines)."""
    f = pfm.Filter(pb, precision=W.FP32_MIXED, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    f.set_tuning(threads, groups)
    f.attach_history()
    r = Runner(f, pb.T)
    r.run(pb.T)  # graph capture and first touch
    f.reset(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.graph_run(pb.T)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    path, idx = f.backtrace()
    dtb = time.perf_counter() - t1
    hist_bytes = int(f.history.numel())
    f.close()
    n_tot = int(pb.n_particles.sum())
    rec_bytes = n_tot * (pb.d * 4 + 4)  # the extra stores: particles and ancestors
    per = dt / pb.T
    extra = per - dt_plain_interval
    leg = {"workload": pb.name, "history_bytes": hist_bytes, "T": pb.T,
           "us_per_interval_with_history": per * 1e6,
           "us_per_interval_without": dt_plain_interval * 1e6,
           "us_added_per_interval": extra * 1e6 if dt_plain_interval > 0 else None,
           "record_bytes_per_interval": rec_bytes,
           "backtrace_ms_all_filters": dtb * 1e3, "path_shape": list(path.shape)}
    log(f"[bench] history: {per * 1e6:.1f} us/interval with recording ({hist_bytes / 2**30:.1f} GiB "
        f"history) vs {dt_plain_interval * 1e6:.1f}; backtrace of {pb.B} filters {dtb * 1e3:.2f} ms")
    return leg


def smc2_leg(torch, pfm, pb, stream, T, threads, groups):
    """SMC over the parameters (Alg. 4) with the batched workload's filters as
    the theta-particles' attached filters (FP32 mixed).  Time i re-runs every
    theta-particle's proposal filter over t_{0:i-1}, so the run does
    T(T+1)/2 intervals of filter work over all particles."""
    inp = W.smc2_l96_inputs(pb.theta, T, seed=4)
    fh = pfm.Filter(pb, precision=W.FP32_MIXED, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    fp = pfm.Filter(pb, precision=W.FP32_MIXED, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    for f in (fh, fp):
        f.set_tuning(threads, groups)
    fh.smc2(fp, inp, T=3, traces=False)  # graph capture and first touch, untimed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fh.smc2(fp, inp, T=T, traces=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fh.close()
    fp.close()
    n_tot = int(pb.n_particles.sum())
    intervals = T * (T + 1) // 2
    w = np.exp(r["logw"] - r["logw"].max())
    w /= w.sum()
    leg = {"workload": f"{pb.name} theta-particles", "theta_particles": pb.B,
           "particles": n_tot, "T": T, "seconds": dt,
           "filter_intervals_per_particle": intervals,
           "particle_steps_per_s": n_tot * intervals / dt,
           "theta_steps_per_s": pb.B * T / dt,
           "accept_rate": float(r["accepts"].sum() / (pb.B * T)),
           "log_evidence": r["log_evidence"], "final_theta_ess": float(r["ess"][-1]),
           "posterior_mean": {"F": float(w @ r["theta"][:, 0]),
                              "sigma": float(w @ r["theta"][:, 1])},
           "status": int(r["status"])}
    log(f"[bench] SMC^2: {pb.B} theta-particles x {T} times in {dt:.2f} s = "
        f"{leg['particle_steps_per_s']:.3e} particle-steps/s; accept {leg['accept_rate']:.3f}; "
        f"log evidence {r['log_evidence']:.2f}; posterior mean F {leg['posterior_mean']['F']:.3f}, "
        f"sigma {leg['posterior_mean']['sigma']:.3f}")
    return leg


def host_cpu():
    """The host's core count and CPU model (the oracle's timing host)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "cores_available": len(os.sched_getaffinity(0)),
            "model": model}


def oracle_worker(argv):
    """One oracle process, pinned to one core: filters w, w + P, ... of the
    headline workload (observations from the file the parent wrote), the
    first T / 10 intervals each, for about `seconds`; prints its work and
    time.  Uses no GPU."""
    w, P, seconds, obs_path, core = (int(argv[0]), int(argv[1]), float(argv[2]), argv[3],
                                     int(argv[4]))
    os.sched_setaffinity(0, {core})
    import oracle
    pb = W.config("lorenz96_d8_batched").with_obs(np.load(obs_path, allow_pickle=False))
    t0 = time.perf_counter()
    done_ps, nf, b = 0, 0, w
    while time.perf_counter() - t0 < seconds and b < pb.B:
        oracle.pf_run(pb, theta=pb.theta[b], N=int(pb.n_particles[b]), b=b, T=pb.T // 10)
        done_ps += int(pb.n_particles[b]) * (pb.T // 10)
        nf += 1
        b += P
    print(json.dumps({"ps": done_ps, "s": time.perf_counter() - t0, "filters": nf,
                      "first": w, "stride": P, "core": core,
                      "affinity": sorted(os.sched_getaffinity(0))}), flush=True)


def oracle_procs(pb, seconds, procs):
    """The oracle in `procs` child processes at once, each pinned to its own
    core (process w on the w-th core of this process's affinity set), on
    disjoint filters of the headline workload."""
    import subprocess
    import tempfile
    cores = sorted(os.sched_getaffinity(0))
    fd, path = tempfile.mkstemp(suffix=".npy")
    os.close(fd)
    try:
        np.save(path, np.ascontiguousarray(pb.obs), allow_pickle=False)
        ps = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                                str(w), str(procs), str(seconds), path,
                                str(cores[w % len(cores)])],
                               stdout=subprocess.PIPE, text=True) for w in range(procs)]
        res = []
        for p in ps:
            out, _ = p.communicate(timeout=seconds * 4 + 120)
            if p.returncode != 0:
                raise RuntimeError(f"oracle worker exited with {p.returncode}")
            res.append(json.loads(out.strip().splitlines()[-1]))
    finally:
        os.unlink(path)
    return res


def pick_tuning(passes):
    """The tuning with the lowest best-of-passes time.  Each pass is the
    autotuner's [groups (1, 2, 4)] x [workgroup (256, 512, 1024)] array of ms
    per interval, -1 where a candidate was not run.  Returns (threads,
    groups, per-candidate best times with -1 kept for candidates never run)."""
    t = np.stack([np.asarray(p, dtype=np.float64).reshape(3, 3) for p in passes])
    best = np.min(np.where(t > 0, t, np.inf), axis=0)
    if not np.isfinite(best).any():
        raise ValueError("no autotuning candidate was timed")
    gi, ci = np.unravel_index(int(np.argmin(best)), best.shape)
    return (256, 512, 1024)[ci], (1, 2, 4)[gi], np.where(np.isfinite(best), best, -1.0)


def autotune(f, steps, passes=3):
    """The library's autotuner on handle f, `passes` times (each candidate's
    best pass kept: the leading candidates differ by about one pass's noise);
    the handle is left on the choice.  The replay mode (graph replay or eager
    launches, whichever the library's last pass measured faster) stays when
    that pass chose the same tuning; another tuning goes back to graphs."""
    threads, groups, cand = pick_tuning([f.autotune(steps=steps)[2] for _ in range(passes)])
    f.set_tuning(threads, groups)
    return threads, groups, cand


def replay_mode(f):
    return "eager launches" if f.get_tuning()[2] else "graph replay"


def pmmh_vs_oracle(pfm, y, stream, chains=2, iters=20, T=20):
    """The PMMH chains against the oracle's chains on the same chain inputs
    (initial values, proposal normals, acceptance uniforms) and the same
    generator counters, at the chains' shape (N = 4096, d = 8) over the first
    T observations: the FP64 batched chains decision by decision (their
    likelihood estimates are the oracle's to rounding, so every accept
    decision is the same), and the FP32 chains' acceptance beside them (an
    FP32 filter's particles part from the FP64 ones within a few intervals
    on this chaotic model, so its estimates, and its decisions, differ by
    Monte Carlo noise)."""
    import oracle
    pm = W.config("lorenz96_d8_chains", chains=chains, T=T).with_obs(y[:T])
    inp = W.pmmh_inputs(chains=chains, iters=iters)
    out = {"chains": chains, "iterations": iters, "T": T, "particles": int(pm.n_particles[0])}
    t0 = time.perf_counter()
    r = oracle.pmmh(pm, int(pm.n_particles[0]), inp)
    out["oracle_seconds"] = time.perf_counter() - t0
    out["accept_rate_oracle_fp64"] = float(r["accepts"].sum() / (chains * iters))
    for name, prec in (("fp64", W.FP64), ("fp32", W.FP32_MIXED)):
        f = pfm.Filter(pm, precision=prec, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
        g = f.pmmh(inp)
        f.close()
        out[f"accept_rate_gpu_{name}"] = float(g["accepts"].sum() / (chains * iters))
        out[f"decisions_equal_to_oracle_{name}"] = float(np.mean(
            (np.diff(g["log_f"], axis=0, prepend=inp.log_f0[None, :]) != 0) ==
            (np.diff(r["log_f"], axis=0, prepend=inp.log_f0[None, :]) != 0)))
        out[f"chain_states_identical_{name}"] = float(np.mean(g["log_f"] == r["log_f"]))
        if name == "fp64":
            out["max_rel_ll_diff_fp64"] = float(np.max(np.abs(g["ll"] - r["ll"]) /
                                                       np.maximum(1.0, np.abs(r["ll"]))))
    return out


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--oracle-worker":
        oracle_worker(sys.argv[2:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed passes of the whole filter over the batch (T intervals each)")
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed passes before the timed ones")
    ap.add_argument("--fp64-steps", type=int, default=40,
                    help="intervals timed for the FP64 plain comparison")
    ap.add_argument("--pmmh-iters", type=int, default=2000)
    ap.add_argument("--repeats", type=int, default=5,
                    help="further repeats of the headline's timed region (spread only)")
    ap.add_argument("--tf-steps", type=int, default=8, help="teacher-forced error intervals")
    ap.add_argument("--headline-form", choices=("accurate", "fast"), default="accurate",
                    help="FP32 form of the headline figure (the other one is reported beside "
                         "it): accurate meets the 1e-4 per-step bound on every filter")
    ap.add_argument("--smc2-T", type=int, default=200,
                    help="observation times of the SMC^2 leg (0: skip it)")
    ap.add_argument("--profile-models", action="store_true",
                    help="run only the model-form and Kalman leg")
    ap.add_argument("--profile-path", action="store_true",
                    help="run only the history / state-sample leg (for kernel traces)")
    ap.add_argument("--profile-smc2", action="store_true",
                    help="run only the SMC^2 leg (for kernel traces)")
    ap.add_argument("--pmmh-tuning", default="",
                    help="collective lanes,groups for --profile-pmmh (default: autotune)")
    ap.add_argument("--profile-pmmh", action="store_true",
                    help="run only PMMH on the chains' shape, 512 lanes / 2 groups "
                         "(for kernel traces; --pmmh-iters sets its length)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="headline workload only")
    ap.add_argument("--profile-headline", action="store_true",
                    help="run only the timed FP32 batched passes with a fixed tuning "
                         "(for counter runs)")
    ap.add_argument("--profile-large", action="store_true",
                    help="run only the large single-filter leg (for counter runs)")
    ap.add_argument("--profile-groups", type=int, default=1,
                    help="filter groups of the --profile-headline run")
    ap.add_argument("--profile-plain", choices=("lorenz96_d8", "lorenz96_d40_large",
                                                "lorenz96_d40_large_spread"),
                    help="run only one plain-layout workload, FP32, 40 graph-replayed "
                         "intervals (for kernel-trace and counter runs); _spread: observation "
                         "sd 20, so the weights stay spread and the gather reads every state")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 2 GiB device-to-device copy (scales the memory "
                         "counters) and exit")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="processes of the all-cores oracle figure (0: skip it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the filters of the batched workload shard across "
              "GPUs with no per-step exchange, but this benchmark measures one GPU only. "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size whose source is not cache-resident: the
        # memory counters of this copy fix their scale
        n = 2 << 30
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        evict = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(2)
        dst = torch.empty(n, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del evict
        print(json.dumps({"copy_calibration_bytes": n}), flush=True)
        return
    import paper_1306_3277_amd as pfm
    pfm.load()
    stream = torch.cuda.Stream()
    if args.profile_large:
        print(json.dumps({"profile_large": large_filter_leg(torch, pfm, stream)}), flush=True)
        return
    if args.profile_plain:
        name = args.profile_plain.replace("_spread", "")
        pp = W.config(name, precision=W.FP32_MIXED)
        _, yp = pfm.simulate(pp, stream=stream)
        pp = pp.with_obs(yp)
        if args.profile_plain.endswith("_spread"):
            pp = dataclasses.replace(pp, obs_sd=20.0)
        fp = pfm.Filter(pp, stream=stream)
        # five timed passes of 40 intervals after a warm-up pass; the fastest
        n = min(40, pp.T)
        fp.graph_run(n)
        passes = []
        for _ in range(5):
            fp.reset(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fp.graph_run(n)
            torch.cuda.synchronize()
            passes.append((time.perf_counter() - t0) / n * 1e6)
        _, essp, _ = fp.loglik(allow_numeric=True)
        fp.close()
        print(json.dumps({"profile_plain": args.profile_plain, "us_per_interval": min(passes),
                          "passes_us": passes, "ess_last": float(essp[0])}), flush=True)
        return

    # ---------------------------------------------------------------- headline
    pb = W.config("lorenz96_d8_batched")
    _, y = pfm.simulate(pb, stream=stream)
    pb = pb.with_obs(y)
    n_tot = int(pb.n_particles.sum())
    log(f"[bench] {pb.name}: B={pb.B} particles={n_tot} T={pb.T}")
    if args.profile_models:
        print(json.dumps({"profile_models": models_leg(torch, pfm, pb, stream, 512, 2)}),
              flush=True)
        return
    if args.profile_path:
        print(json.dumps({"profile_path": path_leg(torch, pfm, pb, stream, 512, 2, 0.0)}),
              flush=True)
        return
    if args.profile_smc2:
        print(json.dumps({"profile_smc2": smc2_leg(torch, pfm, pb, stream, args.smc2_T, 512, 2)}),
              flush=True)
        return
    if args.profile_pmmh:
        pm = W.config("lorenz96_d8_chains").with_obs(y)
        fm = pfm.Filter(pm, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
        if args.pmmh_tuning:
            th, gr = (int(v) for v in args.pmmh_tuning.split(","))
            table = None
        else:
            th, gr, table = autotune(fm, pm.T - 1)
        fm.set_tuning(th, gr)
        # the same filters without the chain layer: whole passes (reset,
        # T intervals, likelihoods read back) and bare interval replay
        dtp = timed_passes(torch, fm, pm.T, 10, 2)
        rp = Runner(fm, pm.T)
        rp.restart()
        dti = timed(torch, rp, 400, pm.T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fm.pmmh(W.pmmh_inputs(chains=pm.B, iters=args.pmmh_iters))
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0
        fm.close()
        print(json.dumps({"profile_pmmh": {
            "iterations": args.pmmh_iters, "collective_workgroup": th, "filter_groups": gr,
            "autotune_ms_per_interval": None if table is None else np.asarray(table).tolist(),
            "filters_per_s": pm.B * (args.pmmh_iters + 1) / dtm,
            "ms_per_iteration": dtm / (args.pmmh_iters + 1) * 1e3,
            "ms_per_pass_without_chain": dtp / 10 * 1e3,
            "us_per_interval_replay": dti / 400 * 1e6}}), flush=True)
        return

    head_prec = W.FP32_ACCURATE if args.headline_form == "accurate" else W.FP32_MIXED
    f32 = pfm.Filter(pb, precision=head_prec, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    if args.profile_headline:
        # counter runs replay each kernel under the profiler: a fixed tuning
        # keeps them short (one filter group by default, so that every
        # propagation launch covers the whole batch)
        threads, groups = 512, args.profile_groups
        tune_src = "fixed (profiling run)"
        f32.set_tuning(threads, groups)
    else:
        # every candidate timed over the whole horizon (the weights'
        # concentration, and with it the collective's work, changes along it)
        threads, groups, cand_ms = autotune(f32, pb.T - 1)
        tune_src = "autotuner, whole horizon per candidate, best of 3 passes"
        log(f"[bench] autotune: collective workgroup {threads}, {groups} filter group(s); "
            f"us/interval (rows: 1, 2, 4 groups; cols: 256, 512, 1024 lanes): "
            f"{np.round(cand_ms * 1e3, 1).tolist()}")
    head_replay = replay_mode(f32)
    dt32 = timed_passes(torch, f32, pb.T, args.steps, args.warmup)
    ps_per_step = n_tot * pb.T
    # the same timed region repeated, for the spread of the figure
    reps = [] if args.profile_headline else [
        timed_passes(torch, f32, pb.T, args.steps, 0) / args.steps * 1e3
        for _ in range(args.repeats)]
    if args.profile_headline:
        f32.close()
        print(json.dumps({"profile_headline": pb.name, "ms_per_step": dt32 / args.steps * 1e3}),
              flush=True)
        return
    # per-kernel durations on one stream (no group overlap), for the roofline
    r32 = Runner(f32, pb.T)
    f32.set_tuning(threads, 1)
    kt32 = kernel_times(r32, pb.T)
    f32.set_tuning(threads, groups)
    r32.restart()
    r32.run(pb.T)
    ll32, _, _ = f32.loglik(allow_numeric=True)
    f32.close()
    rate32 = ps_per_step * args.steps / dt32
    log(f"[bench] fp32 batched ({args.headline_form} form): {dt32 / args.steps * 1e3:.3f} ms/step "
        f"({dt32 / args.steps / pb.T * 1e6:.1f} us/interval) {rate32:.4e} p-steps/s; "
        f"propagate {kt32['propagate']:.1f} us, collective {kt32['batched']:.1f} us")

    # the other FP32 form on the same workload
    other_form = "fast" if args.headline_form == "accurate" else "accurate"
    other_prec = W.FP32_MIXED if other_form == "fast" else W.FP32_ACCURATE
    fo = pfm.Filter(pb, precision=other_prec, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    to, go, _ = autotune(fo, pb.T - 1)
    dto = timed_passes(torch, fo, pb.T, args.steps, 2)
    ro = Runner(fo, pb.T)
    fo.set_tuning(to, 1)
    kto = kernel_times(ro, pb.T)
    fo.close()
    rate_o = ps_per_step * args.steps / dto
    log(f"[bench] fp32 batched ({other_form} form): {dto / args.steps / pb.T * 1e6:.1f} "
        f"us/interval {rate_o:.4e} p-steps/s")

    log("[bench] FP64 plain leg starts")
    f64 = pfm.Filter(pb, precision=W.FP64, layout=pfm.PF_LAYOUT_PLAIN, stream=stream)
    r64 = Runner(f64, pb.T)
    dt64 = timed(torch, r64, args.fp64_steps, 2)
    r64.restart()
    r64.run(pb.T)
    ll64, _, _ = f64.loglik(allow_numeric=True)
    f64.close()
    rate64 = n_tot * args.fp64_steps / dt64
    log(f"[bench] fp64 plain: {dt64 / args.fp64_steps * 1e3:.4f} ms/interval {rate64:.4e} p-steps/s")

    tfs = {}
    for form, prec in (("accurate", W.FP32_ACCURATE), ("fast", W.FP32_MIXED)):
        tf = tf_summary(*teacher_forced_fp32_error(pfm, pb, stream, args.tf_steps, prec),
                        FP32_ELL_BOUND)
        tfs[form] = tf
        log(f"[bench] teacher-forced FP32 ({form} form) error over {pb.B} filters x "
            f"{args.tf_steps} intervals: max {tf['max_abs']:.2e}, p99 {tf['p99_abs']:.2e}, "
            f"median {tf['median_abs']:.2e}; {tf['pairs_over_bound']} of {tf['pairs']} pairs "
            f"over {FP32_ELL_BOUND:g} ({tf['pairs_over_bound_where_ess_ge_2']} of them with "
            f"ESS >= 2); worst {tf['worst'][:2]}")

    # FP64 batched (same kernels as the headline, FP64 state and own-math normals)
    log("[bench] FP64 batched leg starts")
    f64b = pfm.Filter(pb, precision=W.FP64, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    t64b, g64b, _ = autotune(f64b, 16, passes=1)
    n64b = max(2, args.steps // 4)
    dt64b = timed_passes(torch, f64b, pb.T, n64b, 1)
    f64b.close()
    rate64b = ps_per_step * n64b / dt64b
    fp64_batched = {"value": rate64b, "unit": "particle-steps/s",
                    "ms_per_step": dt64b / n64b * 1e3, "steps": n64b,
                    "collective_workgroup": t64b, "filter_groups": g64b}
    log(f"[bench] fp64 batched: {dt64b / n64b * 1e3:.2f} ms/step {rate64b:.4e} p-steps/s")

    flop = model_flop_per_particle_step(pb.model, pb.d, pb.K, pb.n_obs)

    def k5a_roofline(kt, form, profile):
        k5a_s = kt["propagate"] / 1e6
        achieved = flop * n_tot / k5a_s / 1e12
        return {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                "traffic": counted_traffic(profile),
                "kernel": f"k_batch_propagate<fp32 {form}, d=8>", "kernel_us": kt["propagate"],
                "flop_per_particle_step": flop, "particles_per_launch": n_tot}
    form_prof = {"accurate": "k_batch_propagate_accurate_lorenz96_d8_batched_B512.md",
                 "fast": "k_batch_propagate_lorenz96_d8_batched_B512.md"}
    roofline = k5a_roofline(kt32, args.headline_form, form_prof[args.headline_form])
    fp32_other = {"form": other_form, "value": rate_o, "unit": "particle-steps/s",
                  "ms_per_step": dto / args.steps * 1e3,
                  "us_per_interval": dto / args.steps / pb.T * 1e6,
                  "collective_workgroup": to, "filter_groups": go, "kernels_us": kto,
                  "roofline": k5a_roofline(kto, other_form, form_prof[other_form]),
                  "loglik_error": tfs[other_form]}

    out = {
        "metric": "particle-steps/sec (FP32 batched vs FP64 plain) at stated loglik error; "
                  "% HBM roofline",
        "value": rate32,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (simulated on the GPU from the model)",
        "config": {"workload": pb.name, "model": "lorenz96", "d": pb.d, "filters": pb.B,
                   "particles": n_tot, "particle_counts": "uniform over 256..8192",
                   "T": pb.T, "substeps": pb.K, "layout": "batched",
                   "step": f"one pass over the batch: init, {pb.T} intervals, likelihood readout",
                   "particle_steps_per_step": ps_per_step,
                   "us_per_interval": dt32 / args.steps / pb.T * 1e6,
                   "collective_workgroup": threads, "filter_groups": groups, "tuning": tune_src,
                   "replay": head_replay,
                   "precision": ("fp32 accurate form: fp32 state in memory, fp32 slopes and "
                                 "normals, fp64 state and increments within each interval, fp64 "
                                 "log-weights/scan/likelihood" if args.headline_form == "accurate"
                                 else "fp32 fast form: fp32 state/propagation, fp64 "
                                      "log-weights/scan/likelihood")},
        "fp64_plain": {"value": rate64, "unit": "particle-steps/s",
                       "ms_per_interval": dt64 / args.fp64_steps * 1e3,
                       "intervals": args.fp64_steps},
        "fp64_batched": fp64_batched,
        f"fp32_{other_form}": fp32_other,
        "fp32_batched_over_fp64_plain": rate32 / rate64,
        "fp32_batched_over_fp64_batched": rate32 / rate64b,
        "loglik_error": {"fp32_teacher_forced_per_step": tfs[args.headline_form],
                         "bound": FP32_ELL_BOUND,
                         "fp64_vs_oracle_rel_bound": 1e-10,
                         "fp32_free_running_median_abs_diff_vs_fp64":
                             float(np.median(np.abs(ll32 - ll64)))},
        "kernels_us": {"fp32_batched": kt32},
        "repeats_ms_per_step": {"values": [round(x, 4) for x in reps],
                                "median": float(np.median(reps)) if reps else None},
        "roofline": roofline,
    }

    if not args.no_legs:
        # ------------------------------------------------------------ single filter
        log("[bench] single-filter leg starts")
        pc = W.config("lorenz96_d8")
        _, yc = pfm.simulate(pc, stream=stream)
        pc = pc.with_obs(yc)
        leg = {"workload": pc.name, "particles": int(pc.n_particles[0])}
        for name, prec in (("fp32", W.FP32_MIXED), ("fp64", W.FP64)):
            f = pfm.Filter(pc, precision=prec, stream=stream)
            r = Runner(f, pc.T)
            dt = timed(torch, r, pc.T, 20)
            leg[name] = {"particle_steps_per_s": pc.n_particles[0] * pc.T / dt,
                         "us_per_step": dt / pc.T * 1e6,
                         "kernels_us": kernel_times(r, 50)}
            f.close()
        leg["fp32_over_fp64"] = (leg["fp32"]["particle_steps_per_s"] /
                                 leg["fp64"]["particle_steps_per_s"])
        out["single_filter"] = leg
        log(f"[bench] single filter: fp32 {leg['fp32']['us_per_step']:.1f} us/step, "
            f"fp64 {leg['fp64']['us_per_step']:.1f} us/step")

        # ------------------------------------------------------------ large filter
        log("[bench] large-filter leg starts")
        out["large_filter"] = large_filter_leg(torch, pfm, stream)

        # ------------------------------------------------------------ PMMH chains
        if args.pmmh_iters > 0:
            log("[bench] PMMH leg starts")
            pm = W.config("lorenz96_d8_chains")
            pm = pm.with_obs(y)  # the d = 8 data set of the batched workload
            inp = W.pmmh_inputs(chains=pm.B, iters=args.pmmh_iters)
            fm = pfm.Filter(pm, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
            pm_threads, pm_groups, _ = autotune(fm, pm.T - 1)
            pm_replay = replay_mode(fm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fm.pmmh(inp)
            torch.cuda.synchronize()
            dtm = time.perf_counter() - t0
            fm.close()
            nfilt = pm.B * (args.pmmh_iters + 1)
            out["pmmh"] = {"chains": pm.B, "iterations": args.pmmh_iters,
                           "collective_workgroup": pm_threads, "filter_groups": pm_groups,
                           "replay": pm_replay,
                           "particles": int(pm.n_particles[0]), "T": pm.T,
                           "filters_per_s": nfilt / dtm,
                           "particle_steps_per_s": nfilt * int(pm.n_particles[0]) * pm.T / dtm,
                           "accept_rate": float(res["accepts"].sum() /
                                                (pm.B * args.pmmh_iters))}
            log(f"[bench] pmmh: {nfilt / dtm:.1f} filters/s, accept "
                f"{out['pmmh']['accept_rate']:.3f}")
            if not args.no_cpu_baseline:
                out["pmmh"]["vs_oracle"] = pmmh_vs_oracle(pfm, y, stream)
                log(f"[bench] pmmh vs oracle chains: {out['pmmh']['vs_oracle']}")

        # the legs below run the fast FP32 form: its tuning and interval time
        if args.headline_form == "fast":
            ft, fg, fdt = threads, groups, dt32 / args.steps / pb.T
        else:
            ft, fg, fdt = to, go, dto / args.steps / pb.T

        # ------------------------------------------------------------ resamplers
        log("[bench] resampler leg starts")
        out["resamplers_batched"] = resampler_leg(torch, pfm, pb, stream, ft, fg)

        # ------------------------------------------------------------ model forms, Kalman
        log("[bench] models leg starts")
        out["models"] = models_leg(torch, pfm, pb, stream, ft, fg)

        # ------------------------------------------------------------ state sample
        log("[bench] history leg starts")
        out["state_sample"] = path_leg(torch, pfm, pb, stream, ft, fg, fdt)

        # ------------------------------------------------------------ SMC^2
        if args.smc2_T > 0:
            log("[bench] SMC^2 leg starts")
            out["smc2"] = smc2_leg(torch, pfm, pb, stream, args.smc2_T, ft, fg)

    if not args.no_cpu_baseline:
        host = host_cpu()
        log(f"[bench] CPU oracle on one pinned core starts (host {host})")
        # bounded sample of the headline workload: whole filters of the batch,
        # taken in order, the first T/10 intervals each, for about cpu_seconds
        r1 = oracle_procs(pb, args.cpu_seconds, 1)[0]
        out["cpu_baseline"] = {"value": r1["ps"] / r1["s"], "unit": "particle-steps/s",
                               "cores": 1, "kind": "oracle", "host": host,
                               "sample": f"{pb.name}: filters 0..{r1['filters'] - 1} of {pb.B}, "
                                         f"first {pb.T // 10} of {pb.T} intervals each, FP64, "
                                         f"one process pinned to core {r1['core']} "
                                         f"({r1['s']:.1f} s)"}
        if args.cpu_procs > 0:
            procs = min(args.cpu_procs, pb.B, host["cores_available"])
            log(f"[bench] CPU oracle on {procs} pinned processes starts")
            res = oracle_procs(pb, args.cpu_seconds / 2, procs)
            out["cpu_baseline_all_cores"] = {
                "value": sum(r["ps"] / r["s"] for r in res), "unit": "particle-steps/s",
                "cores": procs, "kind": "oracle", "host": host,
                "sample": f"{pb.name}: {sum(r['filters'] for r in res)} filters dealt round-robin "
                          f"to {procs} processes run at once, each pinned to its own core, first "
                          f"{pb.T // 10} of {pb.T} intervals each, FP64, about "
                          f"{args.cpu_seconds / 2:.1f} s per process"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
