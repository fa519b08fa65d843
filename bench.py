"""Throughput of the MI355X bootstrap particle filter (one JSON line on stdout).

A step is one observation interval of the whole hot path for every particle
of the workload: propagate (K substeps) + weight + likelihood increment +
ESS + systematic resampling + ancestor gather.  Inputs (observations,
parameters, particles) are resident in HBM before timing starts; the data
are simulated on the GPU from the model.

Headline (``value``): the FP32 batched form on the batched workload — 512
Lorenz '96 (d = 8) filters with F ~ U(6, 10), sigma ~ U(0.05, 0.3) and
particle counts uniform over {256, ..., 8192}, T = 200 — in particle-steps/s,
next to the FP64 plain filter (one filter at a time, per-filter kernels) on
the same workload, and the FP32 error per step measured at full size by
teacher forcing against the FP64 path.  Secondary legs: the single filter
(d = 8, N = 65,536), the large filter (d = 40, N = 2^20: resample + gather
against HBM, propagation against the VALU issue rate), and marginal
Metropolis-Hastings chains (64 x N = 4096).
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
# VALU peak in lane-operations/s: the FP32 vector peak of 157.3 TFLOP/s counts
# an FMA as 2 FLOP, i.e. 78.6 T lane-operations/s (256 CUs x 2.4 GHz x 128);
# every VALU instruction is counted as one lane-operation.
VALU_PEAK_TOPS = 157.3 / 2


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


def resample_gather_bytes(d: int, sx: int, slw: int) -> int:
    """Algorithmic HBM bytes per particle of one plain-layout resample +
    gather: read the log-weight (scan), write and read the stratum count,
    write the ancestor, read and write the d state components."""
    return slw + 4 + 4 + 4 + 2 * d * sx


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


def teacher_forced_fp32_error(pfm, pb, stream, steps):
    """|ell_t(FP32 batched) - ell_t(FP64 plain)| for every filter and interval,
    each interval started on both sides from the FP64 path's particles rounded
    to FP32 (the FP64 path is the one checked bit for bit against the oracle).
    Returns the errors [steps, B], the FP64 increments and the FP64 ESS."""
    f64 = pfm.Filter(pb, precision=W.FP64, layout=pfm.PF_LAYOUT_PLAIN, stream=stream)
    f32 = pfm.Filter(pb, precision=W.FP32_MIXED, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
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


def tf_summary(err, ell, ess, bound, rel_bound):
    """Distribution of the teacher-forced errors over (interval, filter) pairs;
    the combined bound is max(bound, rel_bound |ell_t|)."""
    comb = np.maximum(bound, rel_bound * np.abs(ell))
    worst = np.argsort(-(err / comb).ravel())[:3]
    ok = ess >= 2.0
    return {"max_abs": float(err.max()), "p99_abs": float(np.quantile(err, 0.99)),
            "median_abs": float(np.median(err)),
            "frac_within_abs_bound": float(np.mean(err <= bound)),
            "max_abs_where_ess_ge_2": float(err[ok].max()) if ok.any() else None,
            "rel_bound": rel_bound,
            "frac_within_combined_bound": float(np.mean(err <= comb)),
            "max_ratio_to_combined_bound": float((err / comb).max()),
            "worst": [{"err": float(err.ravel()[i]), "ell": float(ell.ravel()[i]),
                       "ess": float(ess.ravel()[i])} for i in worst],
            "pairs": int(err.size)}


def large_filter_leg(torch, pfm, stream):
    """One Lorenz '96 (d = 40) filter of 2^20 particles, FP32 mixed: resample +
    gather priced against HBM, propagation against the VALU issue rate."""
    big = W.config("lorenz96_d40_large")
    _, yb = pfm.simulate(big, stream=stream)
    big = big.with_obs(yb)
    fb = pfm.Filter(big, stream=stream)
    rb = Runner(fb, big.T)
    rb.run(3)
    kb = kernel_times(rb, 10)
    dtb = timed(torch, rb, 20, 2)
    variants = {}
    for name, scheme, msteps in (("stratified", 1, 0), ("multinomial", 3, 0),
                                 ("metropolis_8", 2, 8)):
        fb.set_resampler(scheme, msteps)
        rb.restart()
        kv = kernel_times(rb, 10)
        variants[name] = {"resample_gather_us": kv["scan"] + kv["gather"]}
    fb.close()
    nb = int(big.n_particles[0])
    rs_us = kb["scan"] + kb["gather"]
    byt = resample_gather_bytes(big.d, 4, 8)
    gbs = byt * nb / (rs_us * 1e-6) / 1e9
    slots_b = valu_slots_per_particle_step(big.model, big.d, big.K, big.n_obs, True)
    ach_b = slots_b * nb / (kb["propagate"] * 1e-6) / 1e12
    leg = {
        "workload": big.name, "particles": nb, "us_per_step": dtb / 20 * 1e6,
        "particle_steps_per_s": nb * 20 / dtb,
        "resample_gather": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                            "bytes_per_particle": byt, "us": rs_us,
                            "scan_us": kb["scan"], "gather_us": kb["gather"]},
        "propagate": {"bound": "alu", "achieved": ach_b, "peak": VALU_PEAK_TOPS,
                      "unit": "TOP/s", "frac": ach_b / VALU_PEAK_TOPS,
                      "us": kb["propagate"], "ops_per_particle_step": slots_b},
        "combine_us": kb["combine"],
        "resample_variants": variants,
    }
    log("[bench] large filter resample+gather variants (us): " +
        ", ".join(f"{k} {v['resample_gather_us']:.1f}" for k, v in variants.items()))
    log(f"[bench] large filter: resample+gather {rs_us:.1f} us = {gbs:.0f} GB/s "
        f"({gbs / HBM_PEAK_GBS:.0%}); propagate {kb['propagate']:.1f} us "
        f"({ach_b / VALU_PEAK_TOPS:.0%} of VALU issue)")
    return leg


RESAMPLER_CASES = [("systematic", 0, 0, float("inf")), ("stratified", 1, 0, float("inf")),
                   ("multinomial", 3, 0, float("inf")), ("metropolis_8", 2, 8, float("inf")),
                   ("systematic_ess0.5", 0, 0, 0.5)]


def resampler_leg(torch, pfm, pb, stream, threads, groups, steps=100):
    """Interval time of the batched workload (FP32 mixed, graph replay) with
    each resampling variant."""
    out = {}
    for name, scheme, msteps, frac in RESAMPLER_CASES:
        f = pfm.Filter(pb, precision=W.FP32_MIXED, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
        f.set_tuning(threads, groups)
        f.set_resampler(scheme, msteps, frac)
        r = Runner(f, pb.T)
        dt = timed(torch, r, steps, 10)
        f.close()
        out[name] = {"us_per_interval": dt / steps * 1e6,
                     "particle_steps_per_s": int(pb.n_particles.sum()) * steps / dt}
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
    log(f"[bench] models: L96 stage noise {out['lorenz96_stage_noise_batched']['us_per_interval']:.1f} "
        f"us/interval; Kalman 512 x T100 {dtk * 1e3:.3f} ms; SMC with Kalman filters "
        f"512 x T100 {dts * 1e3:.1f} ms")
    return out


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


def oracle_worker(argv):
    """One process of the all-cores oracle figure: filters w, w + P, ... of
    the headline workload (observations from the file the parent wrote), the
    first T / 10 intervals each, for about `seconds`; prints its work and
    time.  Uses no GPU."""
    w, P, seconds, obs_path = int(argv[0]), int(argv[1]), float(argv[2]), argv[3]
    import oracle
    pb = W.config("lorenz96_d8_batched").with_obs(np.load(obs_path, allow_pickle=False))
    t0 = time.perf_counter()
    done_ps, nf, b = 0, 0, w
    while time.perf_counter() - t0 < seconds and b < pb.B:
        oracle.pf_run(pb, theta=pb.theta[b], N=int(pb.n_particles[b]), b=b, T=pb.T // 10)
        done_ps += int(pb.n_particles[b]) * (pb.T // 10)
        nf += 1
        b += P
    print(json.dumps({"ps": done_ps, "s": time.perf_counter() - t0, "filters": nf}), flush=True)


def oracle_all_cores(pb, seconds, procs):
    """The oracle run by `procs` child processes at once on disjoint filters:
    the aggregate rate of the host's cores."""
    import subprocess
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".npy")
    os.close(fd)
    try:
        np.save(path, np.ascontiguousarray(pb.obs), allow_pickle=False)
        ps = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                                str(w), str(procs), str(seconds), path],
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


def autotune_worker(argv):
    """Child process of autotune_isolated: the autotuner on the headline
    workload ("lorenz96_d8_batched") or the PMMH shape ("lorenz96_d8_chains",
    on the headline's data); prints the choice and the candidates' times as
    one JSON line."""
    which = argv[0]
    import torch
    import paper_1306_3277_amd as pfm
    torch.cuda.set_device(0)
    pfm.load()
    stream = torch.cuda.Stream()
    pb = W.config("lorenz96_d8_batched")
    _, y = pfm.simulate(pb, stream=stream)
    pb = pb.with_obs(y)
    if which == "lorenz96_d8_chains":
        pb = W.config("lorenz96_d8_chains").with_obs(y)
    f = pfm.Filter(pb, precision=W.FP32_MIXED, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    # three passes over the candidates, each candidate's best time kept: the
    # leading candidates differ by about as much as one pass's noise
    passes = [f.autotune(steps=pb.T - 1)[2] for _ in range(3)]
    f.close()
    threads, groups, cand = pick_tuning(passes)
    print(json.dumps({"threads": threads, "groups": groups, "cand_ms": cand.tolist()}), flush=True)


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


def autotune_isolated(which):
    """The autotuner run in a child process, so that a failure inside it
    cannot end the benchmark (the autotuner has ended processes with a host
    segmentation fault, cause not found).  Returns (threads, groups,
    candidate times) or None if the child failed."""
    import subprocess
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--autotune-worker", which],
                           capture_output=True, text=True, timeout=600)
    except subprocess.TimeoutExpired:
        return None
    if r.returncode != 0:
        log(f"[bench] autotune child exited with {r.returncode}: {r.stderr.strip()[-300:]}")
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return d["threads"], d["groups"], np.array(d["cand_ms"])


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--oracle-worker":
        oracle_worker(sys.argv[2:])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--autotune-worker":
        autotune_worker(sys.argv[2:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=2000,
                    help="untimed intervals before the timed ones (the device clocks settle)")
    ap.add_argument("--fp64-steps", type=int, default=40,
                    help="intervals timed for the FP64 plain comparison")
    ap.add_argument("--pmmh-iters", type=int, default=2000)
    ap.add_argument("--repeats", type=int, default=5,
                    help="further repeats of the headline's timed region (spread only)")
    ap.add_argument("--tf-steps", type=int, default=8, help="teacher-forced error intervals")
    ap.add_argument("--smc2-T", type=int, default=200,
                    help="observation times of the SMC^2 leg (0: skip it)")
    ap.add_argument("--profile-models", action="store_true",
                    help="run only the model-form and Kalman leg")
    ap.add_argument("--profile-path", action="store_true",
                    help="run only the history / state-sample leg (for kernel traces)")
    ap.add_argument("--profile-smc2", action="store_true",
                    help="run only the SMC^2 leg (for kernel traces)")
    ap.add_argument("--profile-pmmh", action="store_true",
                    help="run only PMMH on the chains' shape, 512 lanes / 2 groups "
                         "(for kernel traces; --pmmh-iters sets its length)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="headline workload only")
    ap.add_argument("--fp64-batched-leg", action="store_true",
                    help="also time the FP64 batched layout on the headline workload "
                         "(off by default: a run with it ended in a host segmentation "
                         "fault whose cause is not found)")
    ap.add_argument("--profile-headline", action="store_true",
                    help="run only the timed FP32 batched intervals (for counter runs)")
    ap.add_argument("--profile-large", action="store_true",
                    help="run only the large single-filter leg (for counter runs)")
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
        fm.set_tuning(512, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fm.pmmh(W.pmmh_inputs(chains=pm.B, iters=args.pmmh_iters))
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0
        fm.close()
        print(json.dumps({"profile_pmmh": {"iterations": args.pmmh_iters,
                                           "filters_per_s": pm.B * (args.pmmh_iters + 1) / dtm}}),
              flush=True)
        return

    f32 = pfm.Filter(pb, precision=W.FP32_MIXED, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
    if args.profile_headline:
        # counter runs replay each kernel under the profiler: a fixed tuning
        # keeps them short
        threads, groups = 512, 2
        tune_src = "fixed (profiling run)"
        f32.set_tuning(threads, groups)
    else:
        # the tuner replays every candidate over the whole horizon (the
        # weights' concentration, and with it the collective's work, changes
        # along it)
        tuned = autotune_isolated("lorenz96_d8_batched")
        if tuned is None:
            threads, groups = 512, 2
            tune_src = "default (the autotuner's child process failed)"
            log("[bench] autotune failed; collective workgroup 512, 2 filter groups")
        else:
            tune_src = "autotuner in a child process, whole horizon per candidate, best of 3 passes"
            threads, groups, cand_ms = tuned
            log(f"[bench] autotune: collective workgroup {threads}, {groups} filter group(s); "
                f"us/interval (rows: 1, 2, 4 groups; cols: 256, 512, 1024 lanes): "
                f"{np.round(cand_ms * 1e3, 1).tolist()}")
        f32.set_tuning(threads, groups)
    r32 = Runner(f32, pb.T)
    dt32 = timed(torch, r32, args.steps, args.warmup)
    # the same timed region repeated, for the spread of the figure
    reps = [] if args.profile_headline else [
        timed(torch, r32, args.steps, 0) / args.steps * 1e3 for _ in range(args.repeats)]
    # per-kernel durations on one stream (no group overlap), for the roofline
    f32.set_tuning(threads, 1)
    kt32 = kernel_times(r32, min(args.steps, pb.T))
    f32.set_tuning(threads, groups)
    r32.restart()
    r32.run(pb.T)
    ll32, _, _ = f32.loglik()
    f32.close()
    rate32 = n_tot * args.steps / dt32
    log(f"[bench] fp32 batched: {dt32 / args.steps * 1e3:.4f} ms/step {rate32:.4e} p-steps/s; "
        f"propagate {kt32['propagate']:.1f} us, collective {kt32['batched']:.1f} us")

    if args.profile_headline:
        print(json.dumps({"profile_headline": pb.name, "ms_per_step": dt32 / args.steps * 1e3}),
              flush=True)
        return

    log("[bench] FP64 plain leg starts")
    f64 = pfm.Filter(pb, precision=W.FP64, layout=pfm.PF_LAYOUT_PLAIN, stream=stream)
    r64 = Runner(f64, pb.T)
    dt64 = timed(torch, r64, args.fp64_steps, 2)
    r64.restart()
    r64.run(pb.T)
    ll64, _, _ = f64.loglik()
    f64.close()
    rate64 = n_tot * args.fp64_steps / dt64
    log(f"[bench] fp64 plain: {dt64 / args.fp64_steps * 1e3:.4f} ms/step {rate64:.4e} p-steps/s")

    tf = tf_summary(*teacher_forced_fp32_error(pfm, pb, stream, args.tf_steps), 1e-4, 1e-6)
    log(f"[bench] teacher-forced FP32 error over {pb.B} filters x {args.tf_steps} intervals: "
        f"max {tf['max_abs']:.2e}, p99 {tf['p99_abs']:.2e}, median {tf['median_abs']:.2e}, "
        f"within 1e-4: {tf['frac_within_abs_bound']:.4f}; within max(1e-4, 1e-6 |ell|): "
        f"{tf['frac_within_combined_bound']:.4f} (worst ratio {tf['max_ratio_to_combined_bound']:.2f}); "
        f"max where ESS >= 2: {tf['max_abs_where_ess_ge_2']:.2e}; worst {tf['worst']}")

    # FP64 batched (same kernels as the headline, FP64 state and own-math normals)
    fp64_batched = None
    if args.fp64_batched_leg:
        f64b = pfm.Filter(pb, precision=W.FP64, layout=pfm.PF_LAYOUT_BATCHED, stream=stream)
        f64b.autotune(steps=4)
        r64b = Runner(f64b, pb.T)
        dt64b = timed(torch, r64b, args.fp64_steps, 4)
        f64b.close()
        rate64b = n_tot * args.fp64_steps / dt64b
        fp64_batched = {"value": rate64b, "unit": "particle-steps/s",
                        "ms_per_step": dt64b / args.fp64_steps * 1e3, "steps": args.fp64_steps}
        log(f"[bench] fp64 batched: {dt64b / args.fp64_steps * 1e3:.4f} ms/step "
            f"{rate64b:.4e} p-steps/s")

    slots = valu_slots_per_particle_step(pb.model, pb.d, pb.K, pb.n_obs, True)
    k5a_s = kt32["propagate"] / 1e6
    achieved = slots * n_tot / k5a_s / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK_TOPS,
                "traffic": counted_traffic("k_batch_propagate_lorenz96_d8_batched_B512.md"),
                "kernel": "k_batch_propagate<fp32, d=8>", "kernel_us": kt32["propagate"],
                "ops_per_particle_step": slots, "particles_per_launch": n_tot}

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
                   "collective_workgroup": threads, "filter_groups": groups, "tuning": tune_src,
                   "precision": "fp32 state/propagation, fp64 log-weights/scan/likelihood"},
        "fp64_plain": {"value": rate64, "unit": "particle-steps/s",
                       "ms_per_step": dt64 / args.fp64_steps * 1e3, "steps": args.fp64_steps},
        "fp64_batched": fp64_batched,
        "fp32_batched_over_fp64_plain": rate32 / rate64,
        "fp32_batched_over_fp64_batched": rate32 / fp64_batched["value"] if fp64_batched else None,
        "loglik_error": {"fp32_teacher_forced_per_step": tf, "bound": 1e-4,
                         "fp64_vs_oracle_rel_bound": 1e-10,
                         "fp32_free_running_median_abs_diff_vs_fp64":
                             float(np.median(np.abs(ll32 - ll64)))},
        "kernels_us": {"fp32_batched": kt32},
        "repeats_ms_per_step": {"values": [round(x, 5) for x in reps],
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
            tuned = autotune_isolated("lorenz96_d8_chains")
            pm_threads, pm_groups = (512, 2) if tuned is None else tuned[:2]
            fm.set_tuning(pm_threads, pm_groups)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fm.pmmh(inp)
            torch.cuda.synchronize()
            dtm = time.perf_counter() - t0
            fm.close()
            nfilt = pm.B * (args.pmmh_iters + 1)
            out["pmmh"] = {"chains": pm.B, "iterations": args.pmmh_iters,
                           "collective_workgroup": pm_threads, "filter_groups": pm_groups,
                           "particles": int(pm.n_particles[0]), "T": pm.T,
                           "filters_per_s": nfilt / dtm,
                           "particle_steps_per_s": nfilt * int(pm.n_particles[0]) * pm.T / dtm,
                           "accept_rate": float(res["accepts"].sum() /
                                                (pm.B * args.pmmh_iters))}
            log(f"[bench] pmmh: {nfilt / dtm:.1f} filters/s, accept "
                f"{out['pmmh']['accept_rate']:.3f}")

        # ------------------------------------------------------------ resamplers
        log("[bench] resampler leg starts")
        out["resamplers_batched"] = resampler_leg(torch, pfm, pb, stream, threads, groups)

        # ------------------------------------------------------------ model forms, Kalman
        log("[bench] models leg starts")
        out["models"] = models_leg(torch, pfm, pb, stream, threads, groups)

        # ------------------------------------------------------------ state sample
        log("[bench] history leg starts")
        out["state_sample"] = path_leg(torch, pfm, pb, stream, threads, groups,
                                       dt32 / args.steps)

        # ------------------------------------------------------------ SMC^2
        if args.smc2_T > 0:
            log("[bench] SMC^2 leg starts")
            out["smc2"] = smc2_leg(torch, pfm, pb, stream, args.smc2_T, threads, groups)

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle sample starts")
        import oracle
        # bounded sample of the headline workload: whole filters of the batch,
        # taken in order, all T intervals, until about cpu_seconds of work
        t0 = time.perf_counter()
        done_ps = 0
        nf = 0
        while time.perf_counter() - t0 < args.cpu_seconds and nf < pb.B:
            b = nf
            oracle.pf_run(pb, theta=pb.theta[b], N=int(pb.n_particles[b]), b=b, T=pb.T // 10)
            done_ps += int(pb.n_particles[b]) * (pb.T // 10)
            nf += 1
        dtc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done_ps / dtc, "unit": "particle-steps/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{pb.name}: filters 0..{nf - 1} of {pb.B}, first "
                                         f"{pb.T // 10} of {pb.T} intervals each, FP64, one "
                                         f"thread ({dtc:.1f} s)"}
        if args.cpu_procs > 0:
            log(f"[bench] CPU oracle on {args.cpu_procs} processes starts")
            procs = min(args.cpu_procs, pb.B)
            res = oracle_all_cores(pb, args.cpu_seconds / 2, procs)
            out["cpu_baseline_all_cores"] = {
                "value": sum(r["ps"] / r["s"] for r in res), "unit": "particle-steps/s",
                "cores": procs, "kind": "oracle",
                "sample": f"{pb.name}: {sum(r['filters'] for r in res)} filters dealt round-robin "
                          f"to {procs} processes run at once, first {pb.T // 10} of {pb.T} "
                          f"intervals each, FP64, about {args.cpu_seconds / 2:.1f} s per process"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
