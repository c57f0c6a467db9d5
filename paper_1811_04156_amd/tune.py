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
    """Sets the sampler's sector tilt by `rounds` pilot rounds of `steps`
    steps (rjpath_tune_tilt); returns the (T, cap+1) table."""
    logw, _ = s.tune_tilt(rounds=rounds, steps=steps, max_logw=max_logw, floor_push=floor_push, run=dict(burn_in=0))
    return logw.cpu().numpy()


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
