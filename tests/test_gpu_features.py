"""Device-side estimator, tuning and autograd checks against the oracle."""
import math

import numpy as np
import pytest

from paper_1811_04156_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_04156_amd import rjpath
    rjpath.load()
    return rjpath


def test_autograd_pure_absorber(rj):
    """No scattering: only the direct sector exists, I = I_2, and
    d log I / d lambda_a = E[L] / lambda_a^2; compared with central
    differences of the oracle's I_2 quadrature."""
    from oracle import oracle as O
    from paper_1811_04156_amd.autograd import RJPathIntensity
    w = W.single_target(2.0, 0.165, math.inf, 20.0, 0.9, chains=512, cap=8, seed=2)
    theta = torch.tensor([[math.inf, 20.0, 0.9]], dtype=torch.float64, requires_grad=True)
    cfg = dict(chunks=2, chunk_steps=200, burn_in=100, tilt=False)
    I = RJPathIntensity.apply(theta, w, cfg)
    I.sum().backward()
    orc = O.Oracle(w)
    I2 = orc.anchor_I2(0)
    assert I.item() == pytest.approx(I2, rel=1e-6)
    h = 1e-4 * 20.0
    wp, wm = dict(w), dict(w)
    wp["lam_a"], wm["lam_a"] = np.array([20.0 + h]), np.array([20.0 - h])
    dI = (O.Oracle(wp).anchor_I2(0) - O.Oracle(wm).anchor_I2(0)) / (2 * h)
    assert theta.grad[0, 1].item() == pytest.approx(dI, rel=2e-3)
    assert theta.grad[0, 0].item() == 0.0  # no scattering vertex, b = 0


def test_graph_replays_match_eager_runs(rj):
    """A captured chunk (sampler steps + score pass) replayed three times,
    with eager work and synchronisations between replays, reproduces three
    eager calls: same paths and counts, FP64 sums to rounding."""
    w = W.config2(groups=8, per_group=256)
    w["burn_in"] = 0
    eager = rj.Sampler(w, precision="f32")
    graph = rj.Sampler(w, precision="f32")
    eager.run(50)
    graph.run(50)
    g, score_acc = graph.capture(200)
    score_eager = torch.zeros_like(score_acc)
    for _ in range(3):
        eager.run(200)
        _, _, sc = eager.grad(logp=False, score=True)
        score_eager += sc
        graph.replay(g)
        torch.cuda.synchronize()
        _ = graph.stats.sum().item()  # eager work between replays
        used = (torch.arange(w["cap"], device=eager.n.device)[:, None] < eager.n[None, :])[..., None]
        assert torch.equal(eager.n, graph.n)
        assert torch.equal(eager.verts[..., :3] * used, graph.verts[..., :3] * used)
        assert torch.equal(eager.stats[:, [0, 5, 6, 7, 8, 9, 10, 11]], graph.stats[:, [0, 5, 6, 7, 8, 9, 10, 11]])
    assert graph.step == eager.step
    assert torch.allclose(score_eager, score_acc, rtol=1e-10, atol=0)


def test_tilt_leaves_the_intensity_unchanged(rj):
    """The tilted sampler estimates the same intensity with a smaller error
    for a distant target."""
    from paper_1811_04156_amd import tune
    w = W.single_target(40.0, 0.165, 10.0, 80.0, 0.9, chains=4096, cap=64, seed=5, burn_in=0)
    out = {}
    for tilt in (False, True):
        s = rj.Sampler(w, precision="f32")
        if tilt:
            tune.tune_tilt(s, rounds=4, steps=400)
        s.run(3000)  # burn-in from the straight starting path
        s.stats.zero_()
        s.run(4000)
        out[tilt] = s.intensity(groups=16)
    a, b = out[False], out[True]
    assert np.isfinite(b["I"][0]) and b["se"][0] > 0
    if np.isfinite(a["I"][0]) and a["se"][0] > 0:
        assert abs(a["I"][0] - b["I"][0]) < 3.5 * math.hypot(a["se"][0], b["se"][0])
        assert b["se"][0] / b["I"][0] < a["se"][0] / a["I"][0]


def test_fp32_intensity_matches_oracle_estimator(rj):
    """Config-2 targets: device estimate (many chains) vs the oracle's
    estimator (fewer chains), within 3.5 combined standard errors."""
    from oracle import oracle as O
    w = W.config2(groups=256, per_group=1)
    pick = [int(t) for t in np.argsort(np.linalg.norm(w["t_sensor"], axis=1))[:6]]  # the nearest targets
    wg = dict(w)
    wg["c_target"] = np.repeat(np.array(pick, np.int32), 4096)
    wg["burn_in"] = 0
    s = rj.Sampler(wg, precision="f32")
    s.run(3000)  # burn-in from the straight starting path
    s.stats.zero_()
    s.run(4000)
    res = s.intensity(groups=16)
    # the oracle on its own chains (stream ids offset so the two samples are independent)
    wo = dict(w)
    wo["c_target"] = np.repeat(np.array(pick, np.int32), 256)
    wo["burn_in"] = 3000
    orc = O.Oracle(wo)
    st = O.initial_state(wo)
    stats, _ = orc.run(wo, st, 7000, chain_ids=np.arange(len(wo["c_target"])) + 1_000_000)
    anchors = [orc.anchor_I2(t) for t in range(len(w["t_src"]))]
    Io, seo = O.intensity(wo, stats, anchors)
    for t in pick:
        assert res["anchor"][t] == pytest.approx(anchors[t], rel=1e-6)
        assert abs(res["I"][t] - Io[t]) < 3.5 * math.hypot(res["se"][t], seo[t]), (t, res["I"][t], Io[t])
