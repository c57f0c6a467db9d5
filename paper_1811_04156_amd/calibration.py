"""Bulk-medium calibration with the differentiated sampler.

The paper motivates path integrals by the calibration of a large scattering
bulk: light is injected by sources inside it and the detected intensities
are matched by simulation (Introduction).  Here the per-layer scattering and
absorption lengths theta = (lambda_s, lambda_a) of a layered medium are fitted
to synthetic intensities by gradient descent:

  loss(theta) = sum_t (log I_t(theta) - log D_t)^2 / (r_t^2 + r_D,t^2)

with I_t the detected intensity of target t (anchored sector estimator,
rjpath_intensity), r_t its relative standard error, D_t the intensities
measured at the ground truth, and the gradient from the score identity
d log I_t / d theta = E_p[d log p / d theta] (rjpath_grad summed over the
sampled paths, rjpath_dlogi_dtheta).  Intensities constrain combinations of
scattering and absorption; the arrival delays separate them (Sec.
"Comparison of timing distributions"), so the fit can add the mean path
length m_t of the detected light, sum_t (m_t - M_t)^2 / (s_m^2 + s_M^2), with
d m_t / d theta = E_p[L d log p / d theta] - E_p[L] E_p[d log p / d theta]
(rjpath_score_length, rjpath_dlength_dtheta).  Every estimate runs in librjpath; this
module sequences the calls and takes the optimiser step (Adam on log theta,
so the lengths stay positive).

The chains are kept across iterations: after each parameter update they start
from their last paths (equilibrated for nearby parameters), which a short
burn-in then adapts.
"""
from __future__ import annotations

import json
import time

import numpy as np
import torch

from .rjpath import Medium, Sampler


class Calibrator:
    """Sampler state of one calibration batch whose medium parameters change."""

    def __init__(self, w, theta, device="cuda", tilt_rounds=3, tilt_steps=300):
        self.w = dict(w)
        self.L = len(w["lam_s"])
        self.s = Sampler(self._with(theta), device=device, precision="f32")
        self.tilt_rounds, self.tilt_steps = tilt_rounds, tilt_steps
        self.theta = np.array(theta, np.float64)

    def _with(self, theta):
        ww = dict(self.w)
        ww["lam_s"], ww["lam_a"] = np.array(theta[:, 0]), np.array(theta[:, 1])
        return ww

    def set_theta(self, theta):
        """Replaces the medium tables (chains keep their paths)."""
        self.theta = np.array(theta, np.float64)
        old = self.s.medium
        self.s.w = self._with(self.theta)
        self.s.medium = Medium(self.s.w, self.s._stream_ptr())
        old.close()
        self.s._anchor = None

    def measure(self, burn=600, chunks=4, chunk_steps=500, tilt=True, groups=16, timing=False):
        """Intensities, their standard errors and d log I / d (lambda_s,
        lambda_a) per target at the current parameters; with `timing` also the
        mean path length of the detected light (the mean arrival delay times
        the speed of light in the bulk), its standard error over the chunks and
        its gradient."""
        s = self.s
        if tilt:
            s.logw = None  # tuned afresh for the current parameters
            s.tune_tilt(rounds=self.tilt_rounds, steps=self.tilt_steps)
        s.run(burn, run=dict(burn_in=s.step + burn))
        s.stats.zero_()
        P = 1 + 3 * s.medium.L_total
        score = torch.zeros((s.T, P), dtype=torch.float64, device=s.dev)
        score_L = torch.zeros((s.T, P), dtype=torch.float64, device=s.dev) if timing else None
        m_chunks = []
        for _ in range(chunks):
            s.run(chunk_steps, run=dict(burn_in=0))
            if timing:
                sc = torch.zeros_like(score)
                sl = torch.zeros_like(score)
                s.grad(logp=False, score=sc)
                s.score_length(sl)
                score += sc
                score_L += sl
                m_chunks.append(s.dlength(sc, sl)[0].cpu().numpy())
            else:
                s.grad(logp=False, score=score)
        res = s.intensity(groups=groups)
        dlogI = s.dlogI(score).cpu().numpy()  # (T, L, 3): lambda_s, lambda_a, g
        if not timing:
            return res["I"], res["se"], dlogI[:, :, :2]
        m, dm = s.dlength(score, score_L)
        mc = np.array(m_chunks)
        se_m = mc.std(axis=0, ddof=1) / np.sqrt(len(mc))
        return res["I"], res["se"], dlogI[:, :, :2], m.cpu().numpy(), se_m, dm.cpu().numpy()[:, :, :2]


def timing_loss_and_grad(m, sm, dm, M, sM, theta):
    """Chi-square loss of the mean path lengths and its gradient with respect
    to log theta (d m / d log theta = theta d m / d theta)."""
    ok = np.isfinite(m) & np.isfinite(M) & np.isfinite(sm) & np.isfinite(sM)
    ok &= np.all(np.isfinite(dm.reshape(len(m), -1)), axis=1)
    v = sm[ok] ** 2 + sM[ok] ** 2
    res = m[ok] - M[ok]
    loss = float(np.sum(res * res / v))
    g = np.einsum("t,tlk->lk", 2 * res / v, dm[ok]) * theta
    return loss, g, float(np.sqrt(np.mean((res / M[ok]) ** 2)))


def loss_and_grad(I, se, dlogI, D, sD, theta):
    """Chi-square loss in log I and its gradient with respect to log theta
    (targets without a finite estimate on either side are left out)."""
    ok = np.isfinite(I) & np.isfinite(D) & (I > 0) & (D > 0) & np.isfinite(se) & np.isfinite(sD)
    ok &= np.all(np.isfinite(dlogI.reshape(len(I), -1)), axis=1)
    r2 = (se[ok] / I[ok]) ** 2 + (sD[ok] / D[ok]) ** 2
    res = np.log(I[ok]) - np.log(D[ok])
    loss = float(np.sum(res * res / r2))
    g = np.einsum("t,tlk->lk", 2 * res / r2, dlogI[ok]) * theta  # d/d log theta
    return loss, g, int(ok.sum()), float(np.sqrt(np.mean(res * res)))


class Adam:
    def __init__(self, shape, lr=0.05, b1=0.9, b2=0.999, eps=1e-8):
        self.m, self.v, self.t = np.zeros(shape), np.zeros(shape), 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, x, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return x - self.lr * mh / (np.sqrt(vh) + self.eps)


def perturbed_start(w, seed, spread=0.2):
    """Ground truth times exp(N(0, spread^2)) per parameter, seeded."""
    rng = np.random.default_rng(seed)
    truth = np.stack([w["lam_s"], w["lam_a"]], axis=1)
    return truth, truth * np.exp(rng.normal(0.0, spread, truth.shape))


def crossed_layers(w):
    """Layers whose centre lies between the lowest and the highest point of
    the source-sensor pairs along the layer axis (the layers the data can
    constrain)."""
    ax = np.asarray(w["m_axis"][0])
    u = np.concatenate([np.asarray(w["t_src"]) @ ax, np.asarray(w["t_sensor"]) @ ax])
    e = np.asarray(w["edges"], np.float64)
    c = 0.5 * (e[:-1] + e[1:])
    return (c >= u.min()) & (c <= u.max())


def fit(w, iters=20, lr=0.05, seed=7, spread=0.2, device="cuda", data_chunks=8, chunks=4, timing=False, log=None):
    """Fits (lambda_s, lambda_a) of every layer from the perturbed start to
    the intensities (and, with `timing`, the mean path lengths of the detected
    light) measured at the ground truth; returns a report."""
    truth, theta0 = perturbed_start(w, seed, spread)
    cal = Calibrator(w, truth, device=device)
    t0 = time.perf_counter()
    data = cal.measure(burn=2000, chunks=data_chunks, timing=timing)  # the synthetic measurement
    D, sD = data[0], data[1]
    t_data = time.perf_counter() - t0
    cal.set_theta(theta0)
    opt = Adam(theta0.shape, lr=lr)
    phi = np.log(theta0)
    hist = []
    inside = crossed_layers(w)
    for it in range(iters):
        t1 = time.perf_counter()
        meas = cal.measure(chunks=chunks, timing=timing)
        I, se, dlogI = meas[:3]
        loss, g, nt, rms = loss_and_grad(I, se, dlogI, D, sD, cal.theta)
        rec = dict(iter=it, loss=loss, targets=nt, rms_log_intensity_residual=rms)
        if timing:
            lt, gt, rms_t = timing_loss_and_grad(meas[3], meas[4], meas[5], data[3], data[4], cal.theta)
            loss += lt
            g = g + gt
            rec.update(loss=loss, timing_loss=lt, rms_rel_length_residual=rms_t)
        err = np.log(cal.theta / truth)
        rec.update(rms_log_param_error=float(np.sqrt(np.mean(err * err))),
                   rms_log_lambda_s_error=float(np.sqrt(np.mean(err[:, 0] ** 2))),
                   rms_log_lambda_a_error=float(np.sqrt(np.mean(err[:, 1] ** 2))),
                   rms_log_param_error_crossed_layers=float(np.sqrt(np.mean(err[inside] ** 2))),
                   seconds=time.perf_counter() - t1)
        hist.append(rec)
        if log:
            log(hist[-1])
        phi = opt.step(phi, g)
        cal.set_theta(np.exp(phi))
    e0 = np.log(theta0 / truth)
    return dict(targets=int(cal.s.T), chains=int(cal.s.C), layers=cal.L, params=2 * cal.L, iters=iters, lr=lr,
                timing=timing, crossed_layers=int(inside.sum()),
                start_rms_log_param_error=float(np.sqrt(np.mean(e0 ** 2))),
                start_rms_log_param_error_crossed_layers=float(np.sqrt(np.mean(e0[inside] ** 2))),
                final_theta=cal.theta.tolist(), history=hist, data_seconds=t_data)


def main():
    import argparse
    from . import workloads as W
    ap = argparse.ArgumentParser(description="Calibration fit of per-layer scattering and absorption lengths")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--lr", type=float, default=0.05)
    ap.add_argument("--chains-per-target", type=int, default=512)
    ap.add_argument("--sources", type=int, default=50)
    ap.add_argument("--timing", action="store_true", help="also fit the mean path lengths (arrival delays)")
    args = ap.parse_args()
    w = W.string_calibration(chains_per_target=args.chains_per_target, n_sources=args.sources)
    rep = fit(w, iters=args.iters, lr=args.lr, timing=args.timing,
              log=lambda h: print(json.dumps(h), flush=True))
    rep.pop("final_theta")
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
