"""The paper's two-region test at full scale (Sec. "Implementation",
Fig. setup; Table "results"): relative light yield B of the sensor at
(60, 7, 104) m to the one at (0, 0, 120) m, for a scan of the scattering
coefficient b1 of the half-space x >= 0.

Each b1 runs `copies` independent copies of the sensor pair (the paper ran
four chains), `chains` chains per sensor and copy, with the tree-coordinate
sampler (whole-path moves; the local moves alone equilibrate the 120 m paths
far more slowly), a burn-in, then windows of sampling with a bridge sample of
every chain every `every` steps.  Prints one JSON line per window and per b1:
B per copy, its mean and the standard error over copies, and the mean vertex
count.  Everything runs in librjpath (rjpath_run_chains,
rjpath_yield_accumulate, rjpath_yield)."""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import workloads as W
from .rjpath import TREE, Sampler


def replicate(w, k, chains):
    """k independent copies of each target of w, `chains` chains each."""
    w = dict(w)
    T = len(w["t_src"])
    for key in list(w):
        if key.startswith("t_") and isinstance(w[key], np.ndarray) and len(w[key]) == T:
            w[key] = np.concatenate([w[key]] * k)
    w["c_target"] = np.repeat(np.arange(k * T, dtype=np.int32), chains)
    return w


def run_b1(b1, copies=4, chains=8192, burn=150_000, windows=3, window_steps=150_000, every=1000, h=0.3,
           scale=1.0, seed=11, log=print):
    t0 = time.perf_counter()
    w = replicate(W.two_region(b1=b1, scale=scale, chains_per_sensor=1, cap=512, seed=seed), copies, chains)
    w.update(burn_in=0, sampler=TREE, mala_h=h)
    s = Sampler(w, precision="f32")
    for _ in range(5):
        s.run(burn // 5)
        log(json.dumps(dict(b1=b1, phase="burn-in", step=s.step, mean_n=round(s.n.float().mean().item(), 2),
                            seconds=round(time.perf_counter() - t0, 1))))
    tabs = s.yield_pairs([(2 * j, 2 * j + 1) for j in range(copies)])
    per_window = []
    total = None
    for k in range(windows):
        acc = None
        for _ in range(window_steps // every):
            s.run(every)
            acc, _ = s.yield_accumulate(tabs, acc=acc, groups=16)
        total = acc.clone() if total is None else total + acc
        B, _ = s.light_yield(acc)
        per_window.append(B)
        log(json.dumps(dict(b1=b1, phase="window", window=k, B=[round(x, 4) for x in B.tolist()],
                            mean_n=round(s.n.float().mean().item(), 2), seconds=round(time.perf_counter() - t0, 1))))
    B, se = s.light_yield(total)
    st = s.stats.cpu().numpy()
    out = dict(b1=b1, phase="result", B=B.tolist(), B_mean=float(B.mean()),
               B_se_over_copies=float(B.std(ddof=1) / np.sqrt(copies)), B_jackknife_se=se.tolist(),
               window_means=[float(x.mean()) for x in per_window], mean_n=float(s.n.float().mean().item()),
               tree_acceptance=float(st[:, 14].sum() / max(1.0, st[:, 13].sum())),
               steps=s.step, chains=s.C, seconds=time.perf_counter() - t0)
    log(json.dumps(out))
    return out


def main():
    ap = argparse.ArgumentParser(description="Relative light yield of the paper's two-region test")
    ap.add_argument("--b1", default="0.1,0.2,0.3,0.4,0.5")
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--chains", type=int, default=8192)
    ap.add_argument("--burn", type=int, default=150_000)
    ap.add_argument("--windows", type=int, default=3)
    ap.add_argument("--window-steps", type=int, default=150_000)
    ap.add_argument("--h", type=float, default=0.3)
    args = ap.parse_args()
    for b1 in [float(x) for x in args.b1.split(",")]:
        run_b1(b1, args.copies, args.chains, args.burn, args.windows, args.window_steps, h=args.h,
               log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
