"""Throughput benchmark of the batched reversible-jump photon-path sampler.

Workload: 65,536 chains in 256 groups of 256 (one source/sensor pair and one
homogeneous medium per group: scattering length log-U[10,50] m, absorption
length log-U[50,200] m, g ~ U[0.8,0.95], sensor radius 0.165 m at U[5,100] m),
vertex cap 256, FP32 evaluation with FP64 statistics; synthetic seeded inputs.

One benchmark step = one pass of the hot path over the batch:
  rjpath_run_chains (1000 sampler steps for every chain: perturbation /
  birth / death proposals, local log-density, accept, statistics)
  + rjpath_intensity (anchor quadrature, reduction, jackknife)
  + rjpath_grad (score pass over every path).
The default 10 timed steps after 1 warm-up step are the workload's 10^4
sampler steps per chain with a 10% burn-in.

Prints one JSON line: path-density evaluations per second (one evaluation =
one proposal's log-density change, accepted or not), plus ESS/s of the
detected intensity at 1% error, the roofline of the step kernel and the FP64
oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12  # MI355X published dense FP32 vector rate (FLOP/s)

# Algorithmic FP32 work per proposal (FLOPs, FMA = 2, one transcendental = 1),
# counted from the arithmetic of the method ("Roofline"):
FLOP_PERTURB = 217.0        # Gaussian step + two segments + three turns, old and new
FLOP_JUMP_BASE = 208.0      # mean of birth (235) and death (180): proposal, segments, turns, Jacobian
FLOP_JUMP_PER_VERTEX = 1.0  # birth scan of the cached depths (2 per vertex over half the path, half the jumps)


# Sources of the step kernel the benchmark times (the FP32 plain-sampler
# variant for homogeneous media); the HBM traffic recorded under profiles/ is
# reported only while their digest matches the one recorded with it.
KERNEL_SOURCES = ["include/rjpath.h", "paper_1811_04156_amd/csrc/rj_internal.h",
                  "paper_1811_04156_amd/csrc/rj_device.h", "paper_1811_04156_amd/csrc/rj_step.h",
                  "paper_1811_04156_amd/csrc/rj_run.h", "paper_1811_04156_amd/csrc/rj_run_f32.hip"]
TRAFFIC_PROFILE = "profiles/run_kernel_hom_f32_config2_traffic.md"


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per launch of the step kernel from the FETCH_SIZE / WRITE_SIZE
    counter runs recorded under profiles/, or None when the kernel sources
    have changed since (or nothing was recorded)."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_PROFILE)) as fh:
            text = fh.read()
    except OSError:
        return None
    rec = {}
    for line in text.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            rec[k.strip(" -*`")] = v.strip(" `")
    if rec.get("kernel_source_sha256") != kernel_digest():
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chunk", type=int, default=1000, help="sampler steps per benchmark step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-extras", action="store_true", help="skip the layered and grad-vs-plain measurements")
    ap.add_argument("--autotune", action="store_true",
                    help="time the launch configurations first (default: the library's measured default)")
    ap.add_argument("--occupancy-probe", action="store_true",
                    help="also time the config-2 kernel (cap 12, all paths in LDS) at one and two resident "
                         "waves per SIMD (65,536 and 131,072 chains)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device copy of this size (calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(w, budget_s):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    the first chain of every 16th chain group, sampler steps until ~budget_s."""
    from oracle import oracle as O
    idx = np.arange(0, len(w["c_target"]), 256 * 16)
    ws = dict(w)
    ws["c_target"] = np.asarray(w["c_target"])[idx]
    orc = O.Oracle(ws)
    st = O.initial_state(ws)
    threads = os.cpu_count() or 1
    steps, done, t_used = 200, 0, 0.0
    while t_used < budget_s:
        t0 = time.perf_counter()
        orc.run(ws, st, steps, step0=done, threads=threads)
        dt = time.perf_counter() - t0
        t_used += dt
        done += steps
        if dt < budget_s / 8:
            steps *= 2
    evals = len(idx) * done
    return dict(value=evals / t_used, unit="path-density evals/s", cores=min(threads, len(idx)), kind="oracle",
                sample=f"{len(idx)} chains (one per 16 chain groups) x {done} steps, FP64, {t_used:.1f} s")


def _ess_run(s, steps, chunk):
    """Times `steps` sampler steps in chunks; returns (seconds, median se/I).
    se/I does not depend on the anchor, so unit anchors are used."""
    import torch
    s._anchor = np.ones(s.T)
    s.stats.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // chunk):
        s.run(chunk)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = s.intensity()
    r = res["se"] / res["I"]
    ok = np.isfinite(r) & (r > 0)
    return dt, float(np.median(r[ok])) if ok.any() else float("nan"), int(ok.sum())


def grad_vs_plain(steps=3000, chunk=500):
    """Config 4's layered medium and cone-source geometry (262,144 chains):
    the plain sampler vs the gradient-informed one (joint Langevin interior
    moves, step size tuned towards 57.4% acceptance), each after the same
    sector-tilt tuning and burn-in; ESS/s at 1% relative error of the median
    target, ESS/s := 1 / (r^2 t)."""
    from paper_1811_04156_amd import tune as tuning
    from paper_1811_04156_amd import workloads as W
    from paper_1811_04156_amd.rjpath import Sampler
    out = {}
    for name in ("plain", "mala"):
        w = W.config4()
        w.update(burn_in=0, sampler=0)
        s = Sampler(w, device="cuda:0", precision="f32")
        tuning.tune_tilt(s, rounds=3, steps=300)
        h = None
        if name == "mala":
            h, acc = tuning.tune_mala(s, h0=0.02, rounds=6, steps=150)
        s.run(500)  # burn-in
        dt, r, nt = _ess_run(s, steps, chunk)
        st = s.stats.cpu().numpy()
        out[name] = {"seconds": dt, "median_rel_err": r, "targets": nt, "ess_per_s": 1.0 / (r * r * dt),
                     "t_1pct_s": dt * (r / 0.01) ** 2, "evals_per_s": s.C * steps / dt,
                     "mean_vertices": float(st[:, 5].sum() / max(1.0, st[:, 0].sum()))}
        if h is not None:
            out[name].update(mala_h=h, mala_acceptance=float(st[:, 14].sum() / max(1.0, st[:, 13].sum())))
    out["ess_ratio_mala_over_plain"] = out["mala"]["ess_per_s"] / out["plain"]["ess_per_s"]
    return out


def occupancy_probe(steps=1000):
    """The step kernel on config 2's media with cap 12 (every path fits its 12
    LDS slots, so the work per chain-step is the same at every occupancy), at
    one resident wave per SIMD (65,536 chains) and two (131,072 chains): how
    much of a SIMD's issue rate one wave leaves unused."""
    import torch
    from paper_1811_04156_amd import workloads as W
    from paper_1811_04156_amd.rjpath import Sampler
    out = {}
    for pg in (256, 512):
        w = W.config2(per_group=pg, cap=12)
        w["burn_in"] = 0
        s = Sampler(w, device="cuda:0", precision="f32")
        s.run(2000, block=64, v_lds=12)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            s.run(steps, block=64, v_lds=12)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 3
        out[f"{s.C}_chains"] = {"ms_per_launch": dt * 1e3, "ns_per_chain_step": dt * 1e9 / (s.C * steps)}
    a, b = out["65536_chains"], out["131072_chains"]
    out["two_wave_speedup_per_chain_step"] = a["ns_per_chain_step"] / b["ns_per_chain_step"]
    return out


def layered_throughput(steps=1000):
    """Config 3 (2^20 chains, 100 layers, cap 512) sampler throughput."""
    import torch
    from paper_1811_04156_amd import workloads as W
    from paper_1811_04156_amd.rjpath import Sampler
    w = W.config3()
    w["burn_in"] = 0
    s = Sampler(w, device="cuda:0", precision="f32")
    s.run(200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = s.stats.cpu().numpy()
    return {"evals_per_s": s.C * steps / dt, "chains": s.C, "steps": steps,
            "mean_vertices": float(st[:, 5].sum() / max(1.0, st[:, 0].sum()))}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each GPU would run its own share "
              "of the chains; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1811_04156_amd import workloads as W
    from paper_1811_04156_amd.rjpath import Sampler

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = W.config2()
    w["burn_in"] = args.warmup * args.chunk
    from paper_1811_04156_amd import tune as tuning
    s = Sampler(w, device="cuda:0", precision="f32")
    stream = torch.cuda.current_stream()
    C = s.C
    # untimed set-up: sector tilt and launch configuration (pilot steps are
    # ordinary sampler steps; their statistics are discarded)
    # (the pilot rounds are full-length launches, so every dispatch of the step
    # kernel in this program is one benchmark chunk)
    torch.cuda.synchronize()
    t_tune = time.perf_counter()
    tuning.tune_tilt(s, rounds=3, steps=args.chunk)
    block, vlds = (0, 0)
    if args.autotune:
        block, vlds = tuning.tune_launch(s, steps=4800)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t_tune
    s.w["burn_in"] = s.step + args.warmup * args.chunk
    # warm-up (burn-in) steps, untimed
    for _ in range(args.warmup):
        s.run(args.chunk)
        s.intensity()
        s.grad(logp=False, score=True)
    torch.cuda.synchronize()
    k_ms = []
    n_mean = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.run(args.chunk)
        e1.record(stream)
        res = s.intensity()
        s.grad(logp=False, score=True)
        k_ms.append((e0, e1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kern = [a.elapsed_time(b) for a, b in k_ms]
    sampler_steps = args.steps * args.chunk
    evals = C * sampler_steps
    value = evals / wall
    # ESS/s of the detected intensity at 1% relative error (median target)
    r = res["se"] / res["I"]
    ok = np.isfinite(r) & (r > 0)
    r_med = float(np.median(r[ok])) if ok.any() else float("nan")
    t_sampling = wall  # statistics accumulate over the timed steps only (burn-in excluded)
    t1pct = t_sampling * (r_med / 0.01) ** 2
    ess_s = 1e4 / t1pct
    # roofline of the step kernel: algorithmic FLOPs per launch / mean launch time
    stats = s.stats.cpu().numpy()
    nbar = stats[:, 5].sum() / max(1.0, stats[:, 0].sum())
    mix_p = w["n_perturb"] / w["cycle_len"]
    flop_per_prop = mix_p * FLOP_PERTURB + (1 - mix_p) * (FLOP_JUMP_BASE + FLOP_JUMP_PER_VERTEX * nbar)
    flop_launch = flop_per_prop * C * args.chunk
    k_mean = float(np.mean(kern)) * 1e-3
    achieved = flop_launch / k_mean
    acc = stats[:, 9:12].sum(0) / np.maximum(1, stats[:, 6:9].sum(0))
    out = {
        "metric": "path-density evals/s + ESS/s of detected intensity at 1% err, grad vs plain",
        "value": value,
        "unit": "path-density evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched plain RJMCMC, 65,536 chains x 256 homogeneous groups, cap 256, "
                               "1e4 sampler steps (1e3 per bench step), FP32 eval / FP64 stats",
                   "chains": C, "sampler_steps_per_bench_step": args.chunk, "cap": int(w["cap"])},
        "ess_per_s": ess_s,
        "t_1pct_s": t1pct,
        "median_rel_err": r_med,
        "mean_vertices": nbar,
        "acceptance": {"perturb": acc[0], "birth": acc[1], "death": acc[2]},
        "kernel_ms_per_launch": float(np.mean(kern)),
        "tuning": {"seconds": t_tune, "block_chains": block or "default (64)", "v_lds": vlds or "default (32)",
                   "tilted_targets": int((s.logw.cpu().numpy().max(1) > 0).sum()) if s.logw is not None else 0},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": recorded_traffic()},
    }
    if not args.no_extras:
        out["layered_config3"] = layered_throughput()
        out["grad_vs_plain"] = grad_vs_plain()
    if args.occupancy_probe:
        out["occupancy_probe"] = occupancy_probe()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
