"""Run-time tuning of the sampler (host policy; every step runs in librjpath).

- sector tilt: a short pilot flattens each target's sector histogram between
  its anchor sector n0 and its mode, so that distant targets visit n0 often
  enough for the anchored estimator (I = I_n0 E[1/w(n)] / E[1(n=n0)/w(n0)]
  stays exact for any tilt w);
- launch configuration: rjpath_autotune over chains-per-block x LDS slots;
- Langevin step size: multiplicative adaptation towards the acceptance 0.574
  that is optimal for MALA in high dimension (Roberts and Rosenthal 1998).
All pilot steps are ordinary sampler steps and may serve as burn-in; the
per-chain statistics are restored afterwards so that no pilot sample (taken
under a different tilt or step size) enters the estimator.
"""
from __future__ import annotations

import numpy as np


def tune_tilt(s, rounds=4, steps=400, max_logw=40.0, floor_push=3.0):
    """Sets s.logw by `rounds` pilot runs of `steps` steps (histograms of the
    sector n after every step).  Returns the (T, cap+1) table."""
    T, cap = s.T, s.cap
    n0 = np.asarray(s.w["t_n0"], int)
    logw = np.zeros((T, cap + 1)) if s.logw is None else s.logw.cpu().numpy().copy()
    saved = s.stats.clone()
    for _ in range(rounds):
        s.set_logw(logw)
        _, hist = s.run(steps, run=dict(burn_in=0), hist=True)
        h = hist.cpu().numpy().astype(np.float64)
        for t in range(T):
            ht = h[t]
            if ht.sum() == 0:
                continue
            mode = int(np.argmax(ht))
            lo = int(n0[t])
            if mode <= lo:
                continue
            for n in range(lo, mode):
                if ht[n] > 0:
                    logw[t, n] += np.log(ht[mode] / ht[n])
                else:
                    logw[t, n] += floor_push
            np.clip(logw[t], 0.0, max_logw, out=logw[t])
    s.set_logw(logw)
    s.stats.copy_(saved)
    return logw


def tune_launch(s, steps=240, run=None):
    """Measured launch configuration (chains per block, LDS vertex slots)."""
    saved = s.stats.clone()
    r = dict(run or {})
    r.setdefault("burn_in", 0)
    out = s.autotune(steps, r)
    s.stats.copy_(saved)
    return out


def tune_mala(s, h0=0.05, rounds=6, steps=200, target=0.574):
    """Adapts the Langevin step size h (m^2) towards the target acceptance of
    the joint interior moves; returns h and the last measured acceptance."""
    h = float(h0)
    acc = float("nan")
    saved = s.stats.clone()
    for _ in range(rounds):
        before = s.stats[:, 13:15].sum(0).cpu().numpy()
        s.run(steps, run=dict(sampler=1, mala_h=h, burn_in=0))
        after = s.stats[:, 13:15].sum(0).cpu().numpy()
        prop, accd = after - before
        if prop <= 0:
            break
        acc = accd / prop
        # multiplicative Robbins-Monro-like update, bounded per round
        h *= float(np.clip(np.exp(2.0 * (acc - target)), 0.3, 3.0))
    s.stats.copy_(saved)
    s.w = dict(s.w)
    s.w.update(sampler=1, mala_h=h)
    return h, acc
