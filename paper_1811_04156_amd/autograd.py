"""Differentiable detected intensity for bulk-medium calibration.

I_t(theta) = integral of p over all paths of target t, with theta the
per-layer (scattering length, absorption length, g) of the media.  Because
the integrand is p itself, d log I / d theta = E_p[d log p / d theta] (score
identity); the expectation is taken over the sampler's paths with the
per-path score from rjpath_grad (recomputed from the vertices, no tape).
The forward pass runs the batched sampler with the given parameters.
"""
from __future__ import annotations

import numpy as np
import torch

from .rjpath import Sampler
from . import tune as tuning


def run_intensity_and_score(w, theta, chunks=4, chunk_steps=500, burn_in=500, tilt=True, precision="f32",
                            device="cuda", anchor=None, groups=16):
    """Samples the workload under theta ((L, 3): lambda_s, lambda_a, g) and
    returns (I, se, dlogI (T, L, 3), sampler).  The score sums accumulate on
    the device across the chunks (rjpath_grad) and rjpath_dlogi_dtheta forms the
    ratio; this function only sequences the calls."""
    th = theta.detach().to("cpu", torch.float64).numpy()
    ww = dict(w)
    ww["lam_s"], ww["lam_a"], ww["g"] = th[:, 0].copy(), th[:, 1].copy(), th[:, 2].copy()
    ww["burn_in"] = 0
    s = Sampler(ww, device=device, precision=precision)
    if tilt:
        tuning.tune_tilt(s)
    s.run(burn_in)
    s.stats.zero_()
    score = torch.zeros((s.T, 1 + 3 * s.medium.L_total), dtype=torch.float64, device=s.dev)
    for _ in range(chunks):
        s.run(chunk_steps)
        s.grad(logp=False, score=score)
    if anchor is not None:
        s._anchor = np.asarray(anchor, np.float64)
    res = s.intensity(groups=groups)
    dlogI = s.dlogI(score).cpu().numpy()
    return res["I"], res["se"], dlogI, s


class RJPathIntensity(torch.autograd.Function):
    """I = RJPathIntensity.apply(theta, w, cfg): theta (L, 3) tensor of
    per-layer (lambda_s, lambda_a, g); returns the (T,) detected intensities.
    backward: dL/dtheta = sum_t gI_t * I_t * d log I_t / d theta."""

    @staticmethod
    def forward(ctx, theta, w, cfg):
        I, se, dlogI, _ = run_intensity_and_score(w, theta, **(cfg or {}))
        It = torch.as_tensor(I, dtype=torch.float64)
        ctx.save_for_backward(It, torch.as_tensor(dlogI, dtype=torch.float64))
        ctx.se = se
        ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
        return It.to(theta.device)

    @staticmethod
    def backward(ctx, gI):
        I, dlogI = ctx.saved_tensors
        g = gI.detach().to("cpu", torch.float64)
        grad = (g[:, None, None] * I[:, None, None] * dlogI).sum(0)
        return grad.to(ctx.theta_device, ctx.theta_dtype), None, None
