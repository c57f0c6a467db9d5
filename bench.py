"""Throughput benchmark of the batched reversible-jump photon-path sampler.

Headline workload: the ragged layered batch -- 2^20 chains over 1000
source/sensor pairs (20-degree cone sources at random depth and azimuth,
sensors of radius 0.165 m at 10-150 m) in 100 horizontal layers of 10 m
(scattering length log-U[10,60] m, absorption length log-U[40,250] m,
g = 0.9), vertex cap 512, FP32 evaluation with FP64 statistics; synthetic
seeded inputs.

One benchmark step = one pass of the whole hot path over the batch, replayed
from two captured graphs on one stream:
  graph 1: rjpath_run_chains -- 1000 sampler steps of every chain
           (perturbation / birth / death proposals, local log-density,
           accept, statistics), launched with the autotuned configuration;
  graph 2: rjpath_grad (score pass over every path, summed per target) and
           rjpath_intensity_noalloc (reduction, jackknife, ESS on the device).
Before timing: sector-tilt pilot rounds, the launch autotuner and the
proposal tuner (interior step, move mix, end-point concentration, scored by
the intensity's ESS per second, the three best candidates tried again on
trials four times as long; their trials are ordinary sampler steps) and
`warmup` benchmark steps of burn-in.  The default 10 timed steps are the workload's 10^4 sampler steps.

Prints one JSON line: path-density evaluations per second (one evaluation =
one proposal whose log-density change was computed, accepted or not), the
ESS/s of the detected intensity at 1% relative error of the median target
(measured from the per-step intensity history), the roofline of the step
kernel, extra measurements (the 65,536-chain homogeneous batch; the
gradient-informed vs the plain sampler on 262,144 chains until 1% error) and
the FP64 oracle timed on the host cores on a bounded sample.
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

# Algorithmic FP32 work per evaluated proposal of a homogeneous medium (an
# add, multiply, FMA or transcendental counts one):
#  perturbation: about 130 add/mul/FMA (two segments and three turns, old and
#    new, the Gaussian or end-point step) + about 13 transcendentals;
#  birth / death: about 150 add/mul/FMA + 21 transcendentals, plus the birth's
#    scan of the cached segment depths (2 per vertex).
# Layered media add a few operations per layer crossed (not counted).
FLOP_PERTURB = 143.0
FLOP_JUMP_BASE = 171.0
FLOP_JUMP_PER_VERTEX = 2.0

# Sources of the step kernel the benchmark times (FP32, plain sampler); the HBM
# traffic recorded under profiles/ is reported only while their digest matches
# the one recorded with it.
KERNEL_SOURCES = ["include/rjpath.h", "paper_1811_04156_amd/csrc/rj_internal.h",
                  "paper_1811_04156_amd/csrc/rj_device.h", "paper_1811_04156_amd/csrc/rj_step.h",
                  "paper_1811_04156_amd/csrc/rj_run.h", "paper_1811_04156_amd/csrc/rj_run_f32.hip"]
TRAFFIC_PROFILE = "profiles/run_kernel_lay_f32_layered_batch_traffic.md"


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
    ap.add_argument("--no-extras", action="store_true", help="skip the homogeneous batch and grad-vs-plain legs")
    ap.add_argument("--sampler", choices=("plain", "langevin", "tree"), default="plain",
                    help="interior move of the headline leg (plain Gaussian step, single-vertex Langevin, or "
                         "tree-coordinate whole-path move on the first step of every cycle)")
    ap.add_argument("--tree-h", type=float, default=0.3, help="variance scale of the tree-coordinate move")
    ap.add_argument("--n-perturb", type=int, default=None,
                    help="fixed number of perturbation steps per cycle of 5 for the headline leg (0: jumps only, "
                         "5: perturbations only; skips the proposal tuner)")
    ap.add_argument("--lmala-h", type=float, default=0.05,
                    help="step-size scale of the single-vertex Langevin sampler in the grad-vs-plain leg")
    ap.add_argument("--proposal-trial", type=int, default=3000,
                    help="sampler steps per candidate and pass of the proposal tuner")
    ap.add_argument("--final-factor", type=int, default=16,
                    help="trial length of the tuner's second stage, in first-stage trials")
    ap.add_argument("--ess-max-steps", type=int, default=200,
                    help="further benchmark steps allowed after the timed ones to reach 1%% error (ESS/s)")
    ap.add_argument("--gvp-max-steps", type=int, default=1_600_000,
                    help="sampler-step cap of each grad-vs-plain run (stops earlier at 1%% error)")
    ap.add_argument("--occupancy-probe", action="store_true",
                    help="also time the homogeneous step kernel (cap 12, all paths in LDS) at one and two resident "
                         "waves per SIMD (65,536 and 131,072 chains)")
    ap.add_argument("--only-homogeneous", action="store_true",
                    help="run only the 65,536-chain homogeneous batch leg (for profiling its step kernel)")
    ap.add_argument("--hom-max-steps", type=int, default=40_000,
                    help="sampler-step cap of the homogeneous batch's run to 1%% error")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device copy of this size (calibrates HBM byte counters)")
    return ap.parse_args()


def progress(msg):
    """One line per finished leg on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def evaluated(stats):
    """Proposals whose log-density change was computed: counted steps minus
    jumps that proposed nothing (a birth at the cap, a death at n = 2)."""
    return float(stats[:, 0].sum() - stats[:, 15].sum())


def flop_per_launch(stats, n_perturb, cycle_len):
    """Algorithmic FP32 operations of the counted proposals (see FLOP_*)."""
    nbar = stats[:, 5].sum() / max(1.0, stats[:, 0].sum())
    perturb = float(stats[:, 6].sum())
    jumps = float(stats[:, 7].sum() + stats[:, 8].sum() - stats[:, 15].sum())
    return perturb * FLOP_PERTURB + jumps * (FLOP_JUMP_BASE + FLOP_JUMP_PER_VERTEX * nbar), nbar


def cpu_baseline(w, budget_s):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    one chain from each of 16 pairs spread over the batch (the pairs' chains
    are independent), sampler steps until ~budget_s."""
    from oracle import oracle as O
    pairs = np.unique(np.asarray(w["c_target"]))[:: max(1, len(np.unique(w["c_target"])) // 16)][:16]
    ws = dict(w)
    ws["c_target"] = pairs.astype(np.int32)
    ws["burn_in"] = 0
    orc = O.Oracle(ws)
    st = O.initial_state(ws)
    threads = os.cpu_count() or 1
    steps, done, t_used, ev = 200, 0, 0.0, 0.0
    while t_used < budget_s:
        t0 = time.perf_counter()
        stats, _ = orc.run(ws, st, steps, step0=done, threads=threads)
        dt = time.perf_counter() - t0
        t_used += dt
        done += steps
        ev += evaluated(stats)
        if dt < budget_s / 8:
            steps *= 2
    return dict(value=ev / t_used, unit="path-density evals/s", cores=min(threads, len(pairs)), kind="oracle",
                cpu_model=cpu_model(), host_threads=threads,
                sample=f"{len(pairs)} chains (one each of {len(pairs)} pairs spread over the batch) x {done} steps, "
                       f"FP64, {t_used:.1f} s")


def median_r(I, se):
    with np.errstate(divide="ignore", invalid="ignore"):  # targets without an estimate drop out below
        r = se / I
    ok = np.isfinite(r) & (r > 0)
    return float(np.median(r[ok])) if ok.any() else float("nan"), int(ok.sum())


def proposal_candidates(w, sampler):
    """Proposal parameters the tuner tries (the workload's own first): the
    interior step, the mix of perturbation and jump steps, the end-point
    concentration and, for the Langevin and tree moves, their step-size scale."""
    base = {k: w[k] for k in ("sigma", "kappa_end", "cycle_len", "n_perturb", "mala_h")}
    out = [dict(base)]

    def add(c):
        if c not in out:
            out.append(c)

    if sampler == "langevin":
        # every interior step of this sampler is the Langevin one, whose scale
        # is mala_h (sigma is unused): its step size crossed with the mix
        for h in (0.02, 0.05, 0.1, 0.2, 0.5, 1.0):
            for npert in (2, 3, 4):
                add(dict(base, mala_h=h, cycle_len=5, n_perturb=npert))
    else:
        # the same mixes as the Langevin grid, crossed with the Gaussian step
        for sig in (0.5, 1.0, 2.0, 4.0, 8.0, 16.0):
            for npert in (2, 3, 4):
                add(dict(base, sigma=sig, cycle_len=5, n_perturb=npert))
    for kap in (5.0, 60.0):
        add(dict(base, kappa_end=kap))
    if sampler == "tree":
        for h in (0.1, 1.0):
            add(dict(base, mala_h=h))
    return out


def tune_two_stage(s, cands, trial, run=None, top=3, factor=16):
    """The proposal tuner in two stages: every candidate on trials of `trial`
    steps, then the `top` best of those again on trials `factor` times as
    long, the pick being the best of the second stage (a short trial's ESS/s
    estimate can rank near-equal candidates either way).  Returns the pick's
    index into `cands`, the first stage's scores and the finalists' indices."""
    _, sc1 = s.tune_proposal(cands, trial, run=run)
    fin = [int(i) for i in np.argsort(-np.asarray(sc1), kind="stable")[:min(top, len(cands))]]
    b2, _ = s.tune_proposal([cands[i] for i in fin], trial * factor, run=run)
    return fin[b2], sc1, fin


def layered_headline(args):
    import torch
    from paper_1811_04156_amd import workloads as W
    from paper_1811_04156_amd.rjpath import Sampler
    from paper_1811_04156_amd.rjpath import LMALA, PLAIN, TREE
    w = W.layered_batch()
    samp = {"plain": PLAIN, "langevin": LMALA, "tree": TREE}[args.sampler]
    w.update(burn_in=0, sampler=samp, mala_h=args.tree_h if args.sampler == "tree" else args.lmala_h)
    s = Sampler(w, device="cuda:0", precision="f32")
    C = s.C
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    # untimed set-up: sector tilt (pilot rounds), launch autotuner (ordinary steps)
    s.tune_tilt(rounds=3, steps=args.chunk)
    block, vlds = s.autotune(2400)
    if args.n_perturb is None:
        cands = proposal_candidates(w, args.sampler)
        best, scores, finalists = tune_two_stage(s, cands, args.proposal_trial, factor=args.final_factor)
        s.w.update(cands[best])
    else:
        # a fixed move mix (profiling one move class): no proposal tuning
        cands, best, scores, finalists = [dict()], 0, np.ones(1), [0]
        s.w.update(cycle_len=5, n_perturb=args.n_perturb)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    s.anchor()  # computed once, before capture
    # statistics count from the first timed step on (the tuner's steps counted)
    s.stats.zero_()
    s.w["burn_in"] = s.step + args.warmup * args.chunk
    g_run = s.capture_run(args.chunk)
    g_stats, out = s.capture_stats(score=True, intensity=True, groups=16)
    for _ in range(args.warmup):
        s.replay(g_run)
        g_stats.replay()
    s.score_acc.zero_()
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    hist_I = torch.empty((args.steps, s.T), dtype=torch.float64, device=s.dev)
    hist_se = torch.empty_like(hist_I)
    e_start = ev()
    marks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_start.record(stream)
    for i in range(args.steps):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        s.replay(g_run)
        e1.record(stream)
        g_stats.replay()
        hist_I[i].copy_(out["I"], non_blocking=True)
        hist_se[i].copy_(out["se"], non_blocking=True)
        e2.record(stream)
        marks.append((e0, e1, e2))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b, _ in marks]
    t_at = [e_start.elapsed_time(c) * 1e-3 for _, _, c in marks]
    stats = s.stats.cpu().numpy()
    hI, hs = hist_I.cpu().numpy(), hist_se.cpu().numpy()
    rs = [median_r(hI[i], hs[i])[0] for i in range(args.steps)]
    hit = [i for i, r in enumerate(rs) if r <= 0.01]
    t1, r1, ext, extra_steps = (t_at[hit[0]], rs[hit[0]], 1.0, 0) if hit else (None, None, None, 0)
    # not at 1% yet: keep replaying the same two graphs (same work per step)
    # until the median target gets there, timed from the first timed step on
    r_last, t_last = rs[-1], t_at[-1]
    while t1 is None and extra_steps < args.ess_max_steps:
        for _ in range(10):
            s.replay(g_run)
            g_stats.replay()
        extra_steps += 10
        e = ev()
        e.record(stream)
        torch.cuda.synchronize()
        r_last, _ = median_r(out["I"].cpu().numpy(), out["se"].cpu().numpy())
        t_last = e_start.elapsed_time(e) * 1e-3
        if r_last <= 0.01:
            t1, r1 = t_last, r_last
    if t1 is None:
        ext = (r_last / 0.01) ** 2
        t1, r1 = t_last * ext, 0.01
    elif ext is None:
        ext = 1.0
    evals = evaluated(stats)
    flop, nbar = flop_per_launch(stats, w["n_perturb"], w["cycle_len"])
    k_mean = float(np.mean(kern_ms)) * 1e-3
    achieved = flop / args.steps / k_mean
    acc = stats[:, 9:12].sum(0) / np.maximum(1, stats[:, 6:9].sum(0))
    return {
        "value": evals / wall,
        "ms_per_step": wall / args.steps * 1e3,
        "config": {"workload": "ragged layered batch: 2^20 chains over 1000 cone-source/sensor pairs at 10-150 m, "
                               "100 layers x 10 m, cap 512, 1e3 sampler steps per bench step, FP32 eval / FP64 "
                               "stats, graph-replayed hot path with the autotuned launch",
                   "chains": C, "pairs": s.T, "layers": int(s.medium.L_total), "cap": int(w["cap"]),
                   "sampler_steps_per_bench_step": args.chunk, "interior_move": args.sampler,
                   "launch": {"block_chains": block, "v_lds": vlds, "graph": True},
                   "proposal": {k: s.w[k] for k in ("sigma", "kappa_end", "cycle_len", "n_perturb", "mala_h")},
                   "proposal_tuning": {"candidates": len(cands), "trial_steps": args.proposal_trial,
                                       "finalists": len(finalists), "final_trial_steps": args.final_factor * args.proposal_trial,
                                       "best_score_over_default": float(scores[best] / scores[0])}},
        # 1 / (r^2 t) with the error measured where it first reaches 1% (the
        # checks come every 10 benchmark steps after the timed ones)
        "ess_per_s": 1.0 / (r1 * r1 * t1),
        "t_1pct_s": t1,
        "median_rel_err_at_t_1pct": r1,
        "t_1pct_measured": ext == 1.0,
        "t_1pct_extrapolation_factor": ext,
        "t_1pct_bench_steps": (hit[0] + 1) if hit else args.steps + extra_steps,
        "median_rel_err": rs[-1],
        "median_rel_err_by_step": rs,
        "mean_vertices": nbar,
        "acceptance": {"perturb": acc[0], "birth": acc[1], "death": acc[2]},
        "kernel_ms_per_launch": float(np.mean(kern_ms)),
        "setup_seconds": t_setup,
        "evaluated_fraction": evals / max(1.0, float(stats[:, 0].sum())),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": recorded_traffic()},
    }, w


def _until_1pct(s, run, chunk, max_steps):
    """Runs the sampler in chunks until the median target's relative error is
    at most 1% (or max_steps); returns (steps, seconds, r).  The intensity
    checks are part of the timed work."""
    import torch
    s.stats.zero_()
    s._anchor = np.ones(s.T)  # se / I does not depend on the anchor
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, r = 0, float("nan")
    while done < max_steps:
        s.run(chunk, run=run)
        done += chunk
        res = s.intensity()
        r, _ = median_r(res["I"], res["se"])
        if r <= 0.01:
            break
    torch.cuda.synchronize()
    return done, time.perf_counter() - t0, r


def grad_vs_plain(h, max_steps, tree_h=0.3, trial=3000, factor=16):
    """262,144 chains on the layered batch's medium and cone-source geometry:
    the plain sampler vs the single-vertex Langevin (gradient-informed)
    sampler and the tree-coordinate sampler (a whole-path move on the first
    step of every cycle), each after the same sector-tilt tuning, 3000
    burn-in steps and the two-stage proposal tuner over its own candidates
    (as the headline leg's), run until the median target's relative error reaches
    1%.  ESS/s := 1 / (r^2 t) at that point."""
    from paper_1811_04156_amd import workloads as W
    from paper_1811_04156_amd.rjpath import LMALA, PLAIN, TREE, Sampler
    out = {}
    for name, samp, hh in (("plain", PLAIN, h), ("langevin", LMALA, h), ("tree", TREE, tree_h)):
        w = W.layered_batch_langevin()
        w.update(burn_in=0, sampler=0)
        s = Sampler(w, device="cuda:0", precision="f32")
        s.tune_tilt(rounds=3, steps=300)
        run = dict(sampler=samp, mala_h=hh, burn_in=0)
        s.run(3000, run=run)
        cands = proposal_candidates(dict(w, mala_h=hh), name)
        best, _, _ = tune_two_stage(s, cands, trial, run=run, factor=factor)
        run.update(cands[best])
        steps, sec, r = _until_1pct(s, run, 4000, max_steps)
        progress(f"grad-vs-plain: {name} sampler, {steps} steps, {sec:.1f} s, r = {r:.4f}")
        st = s.stats.cpu().numpy()
        out[name] = {"steps": steps, "seconds": sec, "median_rel_err": r, "reached_1pct": r <= 0.01,
                     "proposal": {k: cands[best][k] for k in ("sigma", "kappa_end", "cycle_len", "n_perturb", "mala_h")},
                     "ess_per_s": 1.0 / (r * r * sec), "evals_per_s": evaluated(st) / sec,
                     # mixing per step (lower is better) and cost per step: ESS/s = 1 / (their product)
                     "r2_times_steps": r * r * steps, "us_per_step": sec / steps * 1e6,
                     "perturb_acceptance": float(st[:, 9].sum() / max(1.0, st[:, 6].sum())),
                     "mean_vertices": float(st[:, 5].sum() / max(1.0, st[:, 0].sum()))}
    out["ess_ratio_langevin_over_plain"] = out["langevin"]["ess_per_s"] / out["plain"]["ess_per_s"]
    out["ess_ratio_tree_over_plain"] = out["tree"]["ess_per_s"] / out["plain"]["ess_per_s"]
    return out


def homogeneous_batch(chunk=1000, max_steps=40_000):
    """The 65,536-chain batch of 256 homogeneous groups (cap 256): sampler
    throughput and time to 1% error after tilt tuning and 1000 burn-in steps."""
    import torch
    from paper_1811_04156_amd import workloads as W
    from paper_1811_04156_amd.rjpath import Sampler
    w = W.homogeneous_groups()
    w["burn_in"] = 0
    s = Sampler(w, device="cuda:0", precision="f32")
    s.tune_tilt(rounds=3, steps=chunk)
    s.run(chunk)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.stats.zero_()
    e0.record(stream)
    s.run(chunk)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1)
    st = s.stats.cpu().numpy()
    flop, nbar = flop_per_launch(st, w["n_perturb"], w["cycle_len"])
    steps, sec, r = _until_1pct(s, {}, chunk, max_steps)
    st2 = s.stats.cpu().numpy()
    return {"workload": "65,536 chains x 256 homogeneous groups, cap 256", "chains": s.C,
            "evals_per_s_kernel": evaluated(st) / (k_ms * 1e-3),
            "evals_per_s_with_checks": evaluated(st2) / sec, "kernel_ms_per_launch": k_ms,
            "roofline_frac": flop / (k_ms * 1e-3) / PEAK_FP32, "steps_to_1pct": steps, "seconds_to_1pct": sec,
            "median_rel_err": r, "ess_per_s": 1.0 / (r * r * sec), "mean_vertices": nbar}


def occupancy_probe(steps=1000):
    """The step kernel on the homogeneous batch's media with cap 12 (every
    path fits its 12 LDS slots, so the work per chain-step is the same at
    every occupancy), at one resident wave per SIMD (65,536 chains) and two
    (131,072 chains)."""
    import torch
    from paper_1811_04156_amd import workloads as W
    from paper_1811_04156_amd.rjpath import Sampler
    out = {}
    for pg in (256, 512):
        w = W.homogeneous_groups(per_group=pg, cap=12)
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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each GPU would run its own share "
              "of the chains and the per-target sums would be all-reduced)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only_homogeneous:
        print(json.dumps({"homogeneous_batch": homogeneous_batch(max_steps=args.hom_max_steps)}), flush=True)
        return
    head, w = layered_headline(args)
    progress(f"headline leg done: {head['value']:.4g} evals/s, {head['ess_per_s']:.4g} ESS/s")
    out = {
        "metric": "path-density evals/s + ESS/s of detected intensity at 1% err, grad vs plain",
        "value": head.pop("value"),
        "unit": "path-density evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
    }
    out.update(head)
    if not args.no_extras:
        out["homogeneous_batch"] = homogeneous_batch(max_steps=args.hom_max_steps)
        progress("homogeneous batch done")
        out["grad_vs_plain"] = grad_vs_plain(args.lmala_h, args.gvp_max_steps, tree_h=args.tree_h,
                                             trial=args.proposal_trial, factor=args.final_factor)
        progress("grad-vs-plain leg done")
    if args.occupancy_probe:
        out["occupancy_probe"] = occupancy_probe()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
