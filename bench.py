"""Throughput of the MI355X bootstrap particle filter.

A step is one observation interval of the whole hot path for every particle
of the workload: propagate (K substeps) + weight + likelihood increment +
ESS + systematic resampling + ancestor gather.  Inputs (observations,
parameters, particles) are resident in HBM before timing starts; the data
are simulated on the GPU.

Default workload: Lorenz '96, d = 8, N = 65,536, T = 200 (FP32 mixed path),
with the FP64 plain filter timed on the same workload for comparison, plus
the resample + gather HBM rate on the large single filter (d = 40,
N = 2^20).  One JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
# VALU issue slots per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def valu_slots_per_particle_step(model: int, d: int, K: int, n_obs: int, fp32: bool) -> float:
    """Algorithmic VALU issue slots (lane-instructions) one particle needs for
    one observation interval.  Per generator call (4 words): 10 Philox rounds
    of 2 wide multiplies + 4 xors = 60; FP32 normals: 4 uniforms x 3 + 2
    Box-Muller pairs x 7 (log, scale, sqrt, cos, sin, 2 products) = 26; FP64
    normals: 4 uniforms x 2 + 2 pairs x 95 (own log ~32, sincos ~45, sqrt ~12,
    products) = 198.  Lorenz '96 RK4 per component: drift 3 ops x 4 stages +
    4 accumulations + 3 stage inputs + the noise = 20 (FP32, fused) or 30
    (FP64, unfused).  Weight: 3 FP64 ops per observed component."""
    philox = 60
    bm_call = 26 if fp32 else 198
    if model == W.MODEL_WK:
        per_sub = philox + bm_call // 2 + (4 if fp32 else 5)
        return K * per_sub + 8
    rk4 = 20 if fp32 else 30
    per_sub = (d // 4) * (philox + bm_call) + rk4 * d
    return K * per_sub + 3 * n_obs + 4


def resample_gather_bytes(d: int, sx: int, slw: int) -> int:
    """Algorithmic HBM bytes per particle of one resample + gather: read the
    log-weight (scan), write and read the stratum count, write the ancestor,
    read and write the d state components."""
    return slw + 4 + 4 + 4 + 2 * d * sx


def run_steps(f, T: int, n: int, use_graph: bool = True):
    """n consecutive observation intervals, restarting the filter at T."""
    done = 0
    while done < n:
        if f.t_host >= T:
            f.reset(0)
            f.t_host = 0
        k = min(n - done, T - f.t_host)
        if use_graph:
            f.graph_run(k)
        else:
            f.advance(k)
        f.t_host += k
        done += k


def make_filter(pfm, pb, precision, stream):
    f = pfm.Filter(pb, precision=precision, stream=stream)
    f.t_host = 0
    return f


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the d=40, N=2^20 HBM leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; the multi-GPU layout is a design "
              "only (filters shard across GPUs with no per-step exchange). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1306_3277_amd as pfm
    torch.cuda.set_device(0)
    pfm.load()
    stream = torch.cuda.Stream()

    pb = W.config(args.workload)
    if pb.B != 1:
        raise SystemExit("bench.py: use a single-filter workload (c1, c2 or c3)")
    with torch.cuda.stream(stream):
        _, y = pfm.simulate(pb, stream=stream)
    pb = pb.with_obs(y)
    N = int(pb.n_particles[0])
    log(f"[bench] workload {args.workload}: {pb.name} d={pb.d} N={N} T={pb.T} K={pb.K}")

    results = {}
    for name, prec in (("fp32", W.FP32_MIXED), ("fp64", W.FP64)):
        f = make_filter(pfm, pb, prec, stream)
        run_steps(f, pb.T, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_steps(f, pb.T, args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # one full filter run for the log-likelihood
        f.reset(0)
        f.t_host = 0
        run_steps(f, pb.T, pb.T)
        ll, ess, _ = f.loglik()
        # per-kernel durations, measured with HIP events on the filter's stream
        f.reset(0)
        f.t_host = 0
        f.timing(True)
        run_steps(f, pb.T, min(pb.T, args.steps), use_graph=False)
        tm = f.timing_get()
        f.timing(False)
        results[name] = dict(seconds=dt, rate=N * args.steps / dt, loglik=float(ll[0]),
                             timing=tm)
        log(f"[bench] {name}: {dt * 1e3 / args.steps:.4f} ms/step "
            f"{N * args.steps / dt:.4e} particle-steps/s loglik {ll[0]:.6f} "
            f"K1 {tm['propagate_ms'] / max(1, tm['propagate_launches']) * 1e3:.2f} us "
            f"K2 {tm['combine_ms'] / max(1, tm['combine_launches']) * 1e3:.2f} us "
            f"K3 {tm['scan_ms'] / max(1, tm['scan_launches']) * 1e3:.2f} us "
            f"K4 {tm['gather_ms'] / max(1, tm['gather_launches']) * 1e3:.2f} us")
        f.close()

    r32 = results["fp32"]
    tm = r32["timing"]
    k1_s = tm["propagate_ms"] / tm["propagate_launches"] / 1e3
    slots = valu_slots_per_particle_step(pb.model, pb.d, pb.K, pb.n_obs, True)
    achieved = slots * N / k1_s / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                "kernel": "k_propagate_weight<fp32>", "kernel_us": k1_s * 1e6,
                "ops_per_particle_step": slots}

    out = {
        "metric": "particle-steps/sec (FP32 batched vs FP64 plain) at stated loglik error; "
                  "% HBM roofline",
        "value": r32["rate"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["seconds"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (simulated on the GPU from the model)",
        "config": {"workload": pb.name, "model": "lorenz96" if pb.model == 2 else "windkessel",
                   "d": pb.d, "particles": N, "T": pb.T, "substeps": pb.K,
                   "precision": "fp32 state/log-weights, fp64 scan/likelihood"},
        "fp64_plain": {"value": results["fp64"]["rate"], "unit": "particle-steps/s",
                       "ms_per_step": results["fp64"]["seconds"] * 1e3 / args.steps},
        "fp32_over_fp64": r32["rate"] / results["fp64"]["rate"],
        "loglik": {"fp32": r32["loglik"], "fp64": results["fp64"]["loglik"],
                   "fp32_teacher_forced_bound_per_step": 1e-4},
        "roofline": roofline,
    }

    if not args.no_large:
        big = W.config("c3")
        with torch.cuda.stream(stream):
            _, yb = pfm.simulate(big, stream=stream)
        big = big.with_obs(yb)
        fb = make_filter(pfm, big, W.FP32_MIXED, stream)
        run_steps(fb, big.T, 3)
        fb.timing(True)
        run_steps(fb, big.T, 10, use_graph=False)
        tb = fb.timing_get()
        fb.close()
        nb = 1 << 20
        n_st = tb["propagate_launches"]
        rs = (tb["scan_ms"] + tb["gather_ms"]) / n_st / 1e3
        k1b = tb["propagate_ms"] / n_st / 1e3
        step_s = (tb["propagate_ms"] + tb["combine_ms"] + tb["scan_ms"] + tb["gather_ms"]) / n_st / 1e3
        byt = resample_gather_bytes(big.d, 4, 8)
        gbs = byt * nb / rs / 1e9
        slots_b = valu_slots_per_particle_step(big.model, big.d, big.K, big.n_obs, True)
        out["large_filter"] = {
            "workload": big.name, "particles": nb, "step_us": step_s * 1e6,
            "particle_steps_per_s": nb / step_s,
            "resample_gather": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                                "bytes_per_particle": byt, "us": rs * 1e6,
                                "scan_us": tb["scan_ms"] / n_st * 1e3,
                                "gather_us": tb["gather_ms"] / n_st * 1e3},
            "propagate": {"bound": "alu", "achieved": slots_b * nb / k1b / 1e12,
                          "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                          "frac": slots_b * nb / k1b / 1e12 / VALU_PEAK_TOPS, "us": k1b * 1e6},
            "combine_us": tb["combine_ms"] / n_st * 1e3,
        }
        log(f"[bench] large filter: resample+gather {rs * 1e6:.1f} us = {gbs:.0f} GB/s; "
            f"propagate {k1b * 1e6:.1f} us")

    if not args.no_cpu_baseline:
        import oracle
        # bounded sample of the same workload: all N particles over the first
        # T' intervals, T' sized for about cpu_seconds of work
        t_probe = time.perf_counter()
        oracle.pf_run(pb, T=1)
        per_step = time.perf_counter() - t_probe
        Tp = max(1, min(pb.T, int(args.cpu_seconds / max(per_step, 1e-6))))
        t0 = time.perf_counter()
        oracle.pf_run(pb, T=Tp)
        dtc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": N * Tp / dtc, "unit": "particle-steps/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{pb.name}: all {N} particles, first {Tp} of {pb.T} "
                                         f"intervals, FP64, one thread ({dtc:.1f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
