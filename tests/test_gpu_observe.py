"""The snapshot estimators on the device: the relative light yield of two
sensors by the geometric bridge over the cylinder map T (Sec. "Comparison of
relative light yield"; App. "Relative light yield transformation") and the
per-target path-length histograms (Sec. "Comparison of timing
distributions"), on the paper's two-region scenario (Sec. "Implementation",
Fig. setup) with the sensor positions scaled down so that the oracle's analog
tracer reaches it (tests/golden/two_region.txt, written by
tests/golden/make_two_region.py from the oracle alone)."""
import math
import os

import numpy as np
import pytest

from paper_1811_04156_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SCALE = 0.1


@pytest.fixture(scope="module")
def rj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_04156_amd import rjpath
    rjpath.load()
    return rjpath


def _replicate(w, k, chains):
    """k independent copies of each target (copy j of target t is target
    j * T + t), `chains` chains each: independent estimates whose spread
    gives a standard error."""
    from paper_1811_04156_amd.table1 import replicate
    return replicate(w, k, chains)


def _golden():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "two_region.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [float(x) for x in line.split()]
        out[(v[0], int(v[1]))] = dict(I=v[2], se=v[3], lh=np.array(v[4:]).reshape(-1, 2))
    return out


def _path_len(n, V):
    L = np.zeros(len(n))
    for i in range(len(n)):
        d = np.diff(V[i, : n[i]], axis=0)
        L[i] = np.sqrt((d * d).sum(1)).sum()
    return L


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bridge_log_ratio_parity(rj, prec):
    """Each chain's log r (both sides, sensors of different radii so that the
    end point's area factor is exercised) against the oracle's on the same
    path: FP64 to 1e-8; FP32 within the a-priori rounding bound of the two
    full-path densities (both paths' coordinates rounded to FP32: the bound of
    the lock-step tests, summed over every vertex of the chain's path under
    its own target and of its image under the other); the same paths outside
    T's domain (-inf); the bridge sums equal the chains' sqrt(r) and counts."""
    from gpu_helpers import BASE_BOUND, EPS32, K_BOUND
    from oracle import oracle as O
    w = W.two_region(b1=0.3, scale=SCALE, radius=(0.15, 0.3), chains_per_sensor=512, cap=64)
    w["burn_in"] = 0
    s = rj.Sampler(w, precision=prec)
    s.run(400)
    tabs = s.yield_pairs([(0, 1)])
    acc, lr = s.yield_accumulate(tabs, groups=8, logr=True)
    lr = lr.cpu().numpy()
    n, V = s.get_state()
    orc = O.Oracle(w)
    tgt = np.asarray(w["c_target"])
    worst, worst_ratio, outside, errs = 0.0, 0.0, 0, []
    for c in range(0, s.C, 7):
        side = int(tgt[c])
        x = V[c, : n[c]]
        ref = orc.yield_log_ratio(0, 1, side, x)
        if not np.isfinite(ref):
            assert lr[c] == -np.inf, (c, lr[c], ref)
            outside += 1
            continue
        err = abs(lr[c] - ref)
        worst = max(worst, err)
        errs.append(err)
        if prec == "f32":
            y, _ = orc.yield_map(0, 1, x, inverse=side == 1)
            b = 0.0
            for t, v in ((side, x), (1 - side, y)):
                g = orc.grad(t, v, params=False)
                b += float(np.sum(np.abs(g).sum(1) * (np.abs(v).sum(1) + 1.0)))
            bound = 2 * BASE_BOUND + K_BOUND * EPS32 * b
            worst_ratio = max(worst_ratio, err / bound)
    print(f"{prec}: worst |log r - oracle| {worst:.2e} (median {np.median(errs):.1e}), worst ratio to the "
          f"FP32 bound {worst_ratio:.3f}, {outside} paths outside the map's domain")
    if prec == "f64":
        assert worst < 1e-8
    else:
        assert worst_ratio < 1.0 and np.median(errs) < 1e-4
    a = acc.cpu().numpy()
    for side in (0, 1):
        m = tgt == side
        sr = np.where(np.isfinite(lr[m]), np.exp(0.5 * lr[m]), 0.0)
        assert a[0, side, :, 1].sum() == m.sum()
        assert a[0, side, :, 0].sum() == pytest.approx(sr.sum(), rel=1e-12)


@pytest.mark.parametrize("chains", [700, 100])
def test_length_hist_counts_every_path(rj, chains):
    """rjpath_length_hist: bins and normaliser equal a histogram of the
    read-back paths' lengths, with a sector tilt weighting each chain by
    exp(-log w(n)); 700 chains per target exercise the blocks' LDS tables,
    100 the per-lane atomics of blocks that span more than two targets."""
    w = _replicate(W.two_region(b1=0.3, scale=SCALE, chains_per_sensor=1, cap=64), 3, chains)
    w["burn_in"] = 0
    s = rj.Sampler(w, precision="f32")
    rng = np.random.default_rng(1)
    s.set_logw(rng.uniform(0, 3, (s.T, s.cap + 1)))
    s.run(300)
    h = s.length_hist(40, 11.0, 0.5).cpu().numpy()
    n, V = s.get_state()
    L = _path_len(n, V)
    wt = np.exp(-s.logw.cpu().numpy()[np.asarray(w["c_target"]), n])
    tgt = np.asarray(w["c_target"])
    for t in range(s.T):
        m = tgt == t
        b = np.floor((L[m] - 11.0) / 0.5)
        ok = (b >= 0) & (b < 40)
        ref = np.bincount(b[ok].astype(int), weights=wt[m][ok], minlength=40)
        np.testing.assert_allclose(h[t, :40], ref, rtol=1e-12, atol=1e-300)
        assert h[t, 40] == pytest.approx(wt[m].sum(), rel=1e-12)


def _scenario_run(rj, b1, copies=8, chains=4096, burn=20000, snaps=40, every=250):
    # the tree-coordinate sampler: the local moves alone take ~10^6 steps to
    # equilibrate the path length at a few optical depths
    w = _replicate(W.two_region(b1=b1, scale=SCALE, chains_per_sensor=1, cap=128), copies, chains)
    w.update(burn_in=0, sampler=rj.TREE, mala_h=0.3)
    s = rj.Sampler(w, precision="f32")
    s.tune_tilt(rounds=3, steps=300)
    s.run(burn)
    s.stats.zero_()
    tabs = s.yield_pairs([(2 * j, 2 * j + 1) for j in range(copies)])
    acc = None
    hist = None
    for _ in range(snaps):
        s.run(every)
        acc, _ = s.yield_accumulate(tabs, acc=acc, groups=16)
        hist = s.length_hist(47, 0.0, 1.0, hist=hist)
    B, seB = s.light_yield(acc)
    res = s.intensity(groups=16)
    return s, B, seB, res, hist.cpu().numpy()


@pytest.mark.parametrize("b1", [0.1, 0.3])
def test_two_region_yield_and_intensity_vs_tracer(rj, b1):
    """Scaled two-region scenario, 8 independent copies of each sensor pair:
    the device intensities of both sensors (anchored estimator) and the bridge
    estimate of B = I_1 / I_0 agree with the analog tracer within 3 combined
    standard errors, and the bridge agrees with the ratio of the anchored
    intensities."""
    gold = _golden()
    g0, g1 = gold[(b1, 0)], gold[(b1, 1)]
    s, B, seB, res, _ = _scenario_run(rj, b1)
    I = res["I"].reshape(-1, 2)  # copy j: (sensor 0, sensor 1)
    copies = I.shape[0]
    Im, Ise = I.mean(0), I.std(0, ddof=1) / math.sqrt(copies)
    Bm, Bse = B.mean(), B.std(ddof=1) / math.sqrt(copies)
    Rt = g1["I"] / g0["I"]
    Rt_se = Rt * math.hypot(g0["se"] / g0["I"], g1["se"] / g1["I"])
    Ra = I[:, 1] / I[:, 0]
    Ram, Rase = Ra.mean(), Ra.std(ddof=1) / math.sqrt(copies)
    print(f"b1 {b1}: I0 device {Im[0]:.5e} +- {Ise[0] / Im[0]:.2%}, tracer {g0['I']:.5e} +- {g0['se'] / g0['I']:.2%}; "
          f"I1 device {Im[1]:.5e} +- {Ise[1] / Im[1]:.2%}, tracer {g1['I']:.5e} +- {g1['se'] / g1['I']:.2%}")
    print(f"  B bridge {Bm:.5f} +- {Bse / Bm:.2%} (jackknife per copy {np.median(seB / B):.2%}), "
          f"anchored ratio {Ram:.5f} +- {Rase / Ram:.2%}, tracer {Rt:.5f} +- {Rt_se / Rt:.2%}")
    for k, g in ((0, g0), (1, g1)):
        assert abs(Im[k] - g["I"]) < 3 * math.hypot(Ise[k], g["se"])
    assert abs(Bm - Rt) < 3 * math.hypot(Bse, Rt_se)
    assert abs(Bm - Ram) < 3 * math.hypot(Bse, Rase)
    # the per-copy jackknife error is of the size of the spread between copies
    assert 0.3 < np.median(seB) / B.std(ddof=1) < 3.0


def test_two_region_length_distribution_vs_tracer(rj):
    """Path-length distribution of the detected light at both sensors
    (1 m bins): device histogram (8 independent copies) against the tracer's
    detected weight per bin normalised by its intensity; bins with at least
    0.1% of the light (the forward-peaked light arrives within a few metres of
    the straight distance, the tail is what scattering adds) are compared bin
    by bin (|z| < 4.5, mean z^2 < 2.5)."""
    gold = _golden()
    b1 = 0.3
    _, _, _, _, h = _scenario_run(rj, b1)
    h = h.reshape(-1, 2, 48)
    for k in (0, 1):
        p = h[:, k, :47] / h[:, k, 47:48]
        pm, pse = p.mean(0), p.std(0, ddof=1) / math.sqrt(p.shape[0])
        g = gold[(b1, k)]
        q = g["lh"][:47, 0] / g["I"]
        qse = np.sqrt((g["lh"][:47, 1] / g["I"]) ** 2 + (q * g["se"] / g["I"]) ** 2)
        sel = q > 0.001
        z = (pm[sel] - q[sel]) / np.hypot(pse[sel], qse[sel])
        print(f"sensor {k}: {sel.sum()} bins, max |z| {np.abs(z).max():.2f}, mean z^2 {np.mean(z * z):.2f}; "
              f"mean length device {np.sum(pm * (np.arange(47) + 0.5)):.3f} m")
        assert sel.sum() >= 5
        assert np.abs(z).max() < 4.5
        assert np.mean(z * z) < 2.5
