"""Detailed balance of the oracle's reversible-jump kernel, checked against the
densities of its own proposals, and distributional pins of the Langevin moves
and of the intensity gradient.  CPU only.

Detailed balance of a Metropolis-Hastings-Green kernel holds when, for every
pair of paths (x, y) that one move connects,

    pi(x) Q(x -> y) min(1, A) = pi(y) Q(y -> x) min(1, 1/A),

i.e. when the ratio A the sampler uses equals pi(y) Q(y -> x) / (pi(x) Q(x -> y)).
Here Q is measured from the sampler's own proposal map: the oracle builds each
proposal from continuous uniforms, so the density of the proposed vertex is
the inverse Jacobian determinant of that map, taken by finite differences.
Nothing of the printed Jacobian of the bi-spherical map or of the auxiliary
densities q(s), q(t), q(phi) (App. "Dimension matching transformation") enters
the expected value: a wrong term there, a wrong sign of t, a transposed focus
or a wrong segment probability (App. "Jump proposal") breaks the identity.
"""
import math

import numpy as np
import pytest

from paper_1811_04156_amd import workloads as W
from test_oracle_pins import _layered, _random_path

PERTURB, BIRTH, DEATH, JOINT = 0, 1, 2, 3


def _run(w, **over):
    r = {k: w[k] for k in ("seed", "burn_in", "cycle_len", "n_perturb", "birth_frac", "sigma", "kappa_end",
                           "sampler", "mala_h")}
    r.update(over)
    return r


def _workloads():
    """A homogeneous medium with the paper's detection response and vMF
    emission, and a layered medium with the simplified-Liu mixture."""
    a = W.single_target(3.0, 0.165, 2.0, 20.0, 0.9, chains=1, cap=8, emit_kind=W.EMIT_VMF, emit_param=4.0,
                        emit_dir=(0.1, 0.2, 0.97), det_kind=W.DET_PAPER)
    rng = np.random.default_rng(11)
    b = _layered(None, rng.uniform(1.0, 4.0, 6), rng.uniform(10, 40, 6), g=0.85, dz=1.5)
    b["g"] = np.linspace(0.8, 0.95, 6)
    b["f_sl"] = np.array([0.45, 0.0, 0.3, 0.45, 0.0, 0.2])
    b["t_src"] = np.array([[0.0, 0.0, 1.2]])
    b["t_sensor"] = b["t_src"] + np.array([[1.0, 0.5, 3.5]])
    b["cap"] = 8
    return [a, b]


def _paths(orc, w, rng, nmax, count):
    eta = w["t_sensor"][0] - w["t_src"][0]
    out = []
    while len(out) < count:
        n = int(rng.integers(2, nmax + 1))
        v = _random_path(rng, n, eta, float(w["t_radius"][0]))
        if n > 2:
            v[1:-1] = v[1:-1] * 0.5 + rng.normal(size=(n - 2, 3)) * 0.6  # stay close to the short axis
        d = v[-2] - eta
        v[-1] = eta + float(w["t_radius"][0]) * d / np.linalg.norm(d)
        if np.isfinite(orc.logp(0, v)):
            out.append(v)
    return out


def _jac_det(F, u, h=5e-4):
    """|det dF/du| by fourth-order central differences."""
    u = np.asarray(u, float)
    cols = []
    for i in range(len(u)):
        e = np.zeros_like(u)
        e[i] = h
        cols.append((-F(u + 2 * e) + 8 * F(u + e) - 8 * F(u - e) + F(u - 2 * e)) / (12 * h))
    return abs(np.linalg.det(np.array(cols).T))


def _area(F, u, h=5e-4):
    """Area element |dF/du0 x dF/du1| of a map onto a surface."""
    u = np.asarray(u, float)
    d = []
    for i in range(2):
        e = np.zeros(2)
        e[i] = h
        d.append((-F(u + 2 * e) + 8 * F(u + e) - 8 * F(u - e) + F(u - 2 * e)) / (12 * h))
    return np.linalg.norm(np.cross(d[0], d[1]))


@pytest.mark.parametrize("frac", [0.5, 0.3])
@pytest.mark.parametrize("which", [0, 1])
def test_birth_death_detailed_balance(oracle_mod, which, frac):
    w = _workloads()[which]
    cap = int(w["cap"])
    rng = np.random.default_rng(20 + which)
    logw = rng.uniform(0.0, 2.0, (1, cap + 1))  # an arbitrary sector tilt: the chain samples p(f) w(n)
    orc = oracle_mod.Oracle(w, logw=logw)
    run = _run(w, birth_frac=frac)
    pb = oracle_mod.birth_thresh(frac) / 2.0**32
    checked = 0
    for x in _paths(orc, w, rng, 5, 12):
        n = len(x)
        S = sum(orc.tau(0, x[l], x[l + 1], "b") for l in range(n - 1))
        for k in range(n - 1):
            u = rng.uniform(0.2, 0.8, 3)
            y, logA, mv = orc.propose(run, 0, x, BIRTH, k, u)
            assert mv == 2 and len(y) == n + 1
            assert np.array_equal(np.delete(y, k + 1, axis=0), x)
            lpx, lpy = orc.logp(0, x), orc.logp(0, y)
            if not np.isfinite(lpy):
                assert logA == -math.inf
                continue
            # density of the new vertex: inverse Jacobian of the sampler's map u -> f'
            det = _jac_det(lambda uu: orc.propose(run, 0, x, BIRTH, k, uu)[0][k + 1], u)
            q_fwd = pb * orc.tau(0, x[k], x[k + 1], "b") / S / det  # choose birth, segment k, then f'
            q_rev = (1.0 - pb) / (n + 1 - 2)                         # choose death, vertex k+1 of y
            pi_x, pi_y = lpx + logw[0, n], lpy + logw[0, n + 1]
            expect = pi_y + math.log(q_rev) - pi_x - math.log(q_fwd)
            assert logA == pytest.approx(expect, abs=2e-7), (n, k, u)
            # the death of the new vertex is the exact reverse move
            xb, logAd, mvd = orc.propose(run, 0, y, DEATH, k + 1, [])
            assert mvd == 3 and np.allclose(xb, x, atol=0)
            assert logAd == pytest.approx(-logA, abs=1e-10)
            # pi(x) K(x->y) = pi(y) K(y->x) with the measured densities
            lhs = pi_x + math.log(q_fwd) + min(0.0, logA)
            rhs = pi_y + math.log(q_rev) + min(0.0, logAd)
            assert lhs == pytest.approx(rhs, abs=2e-7)
            checked += 1
    assert checked >= 25


def test_death_and_birth_at_sector_edges(oracle_mod):
    """A birth at the cap and a death at n = 2 are rejected proposals (the
    density is zero beyond the cap and no vertex can be removed at n = 2)."""
    w = W.single_target(3.0, 0.165, 2.0, 20.0, 0.9, chains=4, cap=3, burn_in=0, seed=5)
    orc = oracle_mod.Oracle(w)
    st = oracle_mod.initial_state(w)
    _, tr = orc.run(w, st, 2000, trace=True)
    n = np.full(4, 2)
    for s in range(2000):
        for c in range(4):
            mv, acc = tr[c, s, 0], tr[c, s, 1]
            if mv == 2 and n[c] == 3:
                assert acc == 0 and tr[c, s, 3] == -math.inf
            if mv == 3 and n[c] == 2:
                assert acc == 0 and tr[c, s, 3] == -math.inf
            if acc:
                n[c] += 1 if mv == 2 else (-1 if mv == 3 else 0)
    assert np.array_equal(n, st["n"])


@pytest.mark.parametrize("which", [0, 1])
def test_interior_perturbation_is_a_symmetric_gaussian(oracle_mod, which):
    """The interior step is sigma * xi with xi ~ N(0, I) (moments of 20,000
    proposals from uniform draws), and its ratio is the density ratio alone."""
    w = _workloads()[which]
    orc = oracle_mod.Oracle(w)
    rng = np.random.default_rng(30 + which)
    x = next(p for p in _paths(orc, w, rng, 5, 20) if len(p) >= 4)
    sigma = 0.37
    run = _run(w, sigma=sigma, sampler=0)
    N = 20000
    xi = np.zeros((N, 3))
    for i in range(N):
        j = 1 + i % (len(x) - 2)
        y, logA, mv = orc.propose(run, 0, x, PERTURB, j, rng.uniform(0, 1, 4))
        assert mv == 0
        assert np.array_equal(np.delete(y, j, axis=0), np.delete(x, j, axis=0))
        xi[i] = (y[j] - x[j]) / sigma
        if i < 300:
            lpy = orc.logp(0, y)
            ref = lpy - orc.logp(0, x) if np.isfinite(lpy) else -math.inf
            assert logA == pytest.approx(ref, abs=1e-12)
    assert np.all(np.abs(xi.mean(0)) < 4.5 / math.sqrt(N))
    assert np.all(np.abs(np.cov(xi.T) - np.eye(3)) < 4.5 * math.sqrt(2.0 / N))
    kurt = ((xi - xi.mean(0)) ** 4).mean(0) / xi.var(0) ** 2
    assert np.all(np.abs(kurt - 3.0) < 4.5 * math.sqrt(24.0 / N))


@pytest.mark.parametrize("kappa", [5.0, 20.0])
def test_end_point_step_is_a_symmetric_vmf(oracle_mod, kappa):
    """The end-point move on the sensor: the density of the proposed normal,
    from the area element of the sampler's map, is the von Mises-Fisher
    density kappa e^{kappa (nu . nu' - 1)} / (2 pi (1 - e^{-2 kappa})) (which
    depends on nu . nu' alone, so the move is symmetric), and its ratio is the
    density ratio alone."""
    w = _workloads()[0]
    orc = oracle_mod.Oracle(w)
    rng = np.random.default_rng(40)
    eta, R = w["t_sensor"][0] - w["t_src"][0], float(w["t_radius"][0])
    run = _run(w, kappa_end=kappa)
    for x in _paths(orc, w, rng, 4, 6):
        n = len(x)
        nu = (x[-1] - eta) / R
        for _ in range(6):
            u = rng.uniform(0.1, 0.9, 2)
            F = lambda uu: (orc.propose(run, 0, x, PERTURB, n - 1, np.r_[uu, 0.5, 0.5])[0][-1] - eta) / R
            y, logA, mv = orc.propose(run, 0, x, PERTURB, n - 1, np.r_[u, 0.5, 0.5])
            assert mv == 1
            nn = F(u)
            assert abs(np.linalg.norm(nn) - 1) < 1e-12
            dens = 1.0 / _area(F, u)
            vmf = kappa * math.exp(kappa * (nu @ nn - 1)) / (2 * math.pi * (1 - math.exp(-2 * kappa)))
            assert dens == pytest.approx(vmf, rel=1e-7)
            lpy = orc.logp(0, y)
            ref = lpy - orc.logp(0, x) if np.isfinite(lpy) else -math.inf
            assert logA == pytest.approx(ref, abs=1e-12)


def _fd_grad(orc, v, ks, h=1e-6):
    g = np.zeros((len(v), 3))
    for k in ks:
        for i in range(3):
            a, b = v.copy(), v.copy()
            a[k, i] += h
            b[k, i] -= h
            g[k, i] = (orc.logp(0, a) - orc.logp(0, b)) / (2 * h)
    return g


def _box_muller3(u):
    r1, r2 = math.sqrt(-2 * math.log(u[0])), math.sqrt(-2 * math.log(u[2]))
    return np.array([r1 * math.cos(2 * math.pi * u[1]), r1 * math.sin(2 * math.pi * u[1]),
                     r2 * math.cos(2 * math.pi * u[3])])


def _log_gauss3(z, mean, h):
    d = z - mean
    return -1.5 * math.log(2 * math.pi * h) - d @ d / (2 * h)


@pytest.mark.parametrize("which", [0, 1])
def test_joint_langevin_ratio(oracle_mod, which):
    """Joint Langevin move: the proposal is x + (h/2) grad log p + sqrt(h) xi
    with the gradient taken here by central differences of log p, and the
    ratio is pi(y) N(x; y + (h/2) grad(y), h) / (pi(x) N(y; x + (h/2) grad(x), h))."""
    w = _workloads()[which]
    orc = oracle_mod.Oracle(w)
    rng = np.random.default_rng(50 + which)
    h = 0.004
    run = _run(w, sampler=1, mala_h=h)
    checked = 0
    for x in _paths(orc, w, rng, 5, 10):
        n = len(x)
        if n < 3:
            continue
        U = rng.uniform(0.05, 0.95, 4 * (n - 2))
        y, logA, mv = orc.propose(run, 0, x, JOINT, 0, U)
        assert mv == 4
        inner = range(1, n - 1)
        gx = _fd_grad(orc, x, inner)
        for k in inner:
            xi = _box_muller3(U[4 * (k - 1): 4 * k])
            assert np.allclose(y[k], x[k] + 0.5 * h * gx[k] + math.sqrt(h) * xi, atol=1e-8 * (1 + np.abs(gx[k]).max()))
        assert np.array_equal(y[[0, n - 1]], x[[0, n - 1]])
        lpy = orc.logp(0, y)
        if not np.isfinite(lpy):
            assert logA == -math.inf
            continue
        gy = _fd_grad(orc, y, inner)
        ref = lpy - orc.logp(0, x)
        for k in inner:
            ref += _log_gauss3(x[k], y[k] + 0.5 * h * gy[k], h) - _log_gauss3(y[k], x[k] + 0.5 * h * gx[k], h)
        assert logA == pytest.approx(ref, abs=1e-6)
        checked += 1
    assert checked >= 5


@pytest.mark.parametrize("which", [0, 1])
def test_single_vertex_langevin_ratio(oracle_mod, which):
    """Single-vertex Langevin move at interior vertex j with step size
    h(x) = mala_h * min(|f_j - f_{j-1}|, |f_{j+1} - f_j|)^2: proposal
    x_j + (h/2) d log p / d f_j + sqrt(h) xi, ratio with both Gaussian
    densities (each with its own h, so their normalisations enter)."""
    w = _workloads()[which]
    orc = oracle_mod.Oracle(w)
    rng = np.random.default_rng(60 + which)
    c = 0.05
    run = _run(w, sampler=2, mala_h=c)

    def hof(v, j):
        return c * min(np.linalg.norm(v[j] - v[j - 1]), np.linalg.norm(v[j + 1] - v[j])) ** 2

    checked = 0
    for x in _paths(orc, w, rng, 5, 14):
        n = len(x)
        for j in range(1, n - 1):
            u = rng.uniform(0.05, 0.95, 4)
            y, logA, mv = orc.propose(run, 0, x, PERTURB, j, u)
            assert mv == 6
            assert np.array_equal(np.delete(y, j, axis=0), np.delete(x, j, axis=0))
            gx = _fd_grad(orc, x, [j])[j]
            hx = hof(x, j)
            assert np.allclose(y[j], x[j] + 0.5 * hx * gx + math.sqrt(hx) * _box_muller3(u),
                               atol=1e-8 * (1 + hx * np.abs(gx).max()))
            lpy = orc.logp(0, y)
            if not np.isfinite(lpy):
                assert logA == -math.inf
                continue
            gy = _fd_grad(orc, y, [j])[j]
            hy = hof(y, j)
            ref = lpy - orc.logp(0, x) + _log_gauss3(x[j], y[j] + 0.5 * hy * gy, hy) - \
                _log_gauss3(y[j], x[j] + 0.5 * hx * gx, hx)
            assert logA == pytest.approx(ref, abs=1e-6)
            checked += 1
    assert checked >= 10


# --------------------------------------------------------------------------
# distributional pins against the analog tracer
# --------------------------------------------------------------------------
def _sector_snapshots(oracle_mod, w, steps, every=10):
    """Runs the oracle sampler and returns, per chain and snapshot, the vertex
    count and the path length (after burn-in)."""
    orc = oracle_mod.Oracle(w)
    st = oracle_mod.initial_state(w)
    burn = int(w["burn_in"])
    orc.run(w, st, burn)
    ns, Ls = [], []
    for s in range(burn, steps, every):
        orc.run(w, st, every, step0=s)
        n = st["n"].copy()
        v = st["verts"]
        seg = np.linalg.norm(np.diff(v, axis=1), axis=2)
        mask = np.arange(v.shape[1] - 1)[None, :] < (n - 1)[:, None]
        ns.append(n)
        Ls.append((seg * mask).sum(1))
    return orc, np.array(ns).T, np.array(Ls).T  # (chains, snapshots)


def _group_se(per_group):
    per_group = np.asarray(per_group)
    return per_group.std(ddof=1) / math.sqrt(len(per_group))


@pytest.mark.slow
@pytest.mark.parametrize("sampler,h", [(1, 0.01), (2, 0.3), (3, 0.3)])
def test_langevin_sector_occupancy_matches_tracer(oracle_mod, sampler, h):
    """With every interior perturbation a Langevin move (joint, or single
    vertex), or with the tree-coordinate move of the whole path on the first
    step of every cycle, the chain on paths with n <= 4 spends time in sectors 3 and 4
    relative to sector 2 as I_3 / I_2 and I_4 / I_2, and its mean path length
    in sector 3 is the tracer's, whose photons detected after exactly one and
    two scatterings measure the same quantities."""
    w = W.single_target(1.5, 0.165, 10.0, 60.0, 0.9, chains=256, cap=4, burn_in=500, seed=8, sampler=sampler,
                        mala_h=h)
    orc, n, L = _sector_snapshots(oracle_mod, w, 6500)
    tr = orc.trace_full(0, 20_000_000, esc=400.0)
    b, bL = tr["bucket"], tr["bucket_L"]
    groups = np.arange(n.shape[0]) % 16
    for m in (3, 4):
        ratio = (n == m).sum() / (n == 2).sum()
        per = [(n[groups == g] == m).sum() / (n[groups == g] == 2).sum() for g in range(16)]
        rt = b[m - 2, 0] / b[0, 0]
        se_t = rt * math.hypot(b[m - 2, 1] / b[m - 2, 0], b[0, 1] / b[0, 0])
        assert abs(ratio - rt) < 3.5 * math.hypot(_group_se(per), se_t), (m, ratio, rt)
    Lc = L[n == 3].mean()
    per = [L[groups == g][n[groups == g] == 3].mean() for g in range(16)]
    Lt = bL[1, 0] / b[1, 0]
    se_t = Lt * math.hypot(bL[1, 1] / bL[1, 0], b[1, 1] / b[1, 0])
    assert abs(Lc - Lt) < 3.5 * math.hypot(_group_se(per), se_t), (Lc, Lt)


def test_absorption_score_is_minus_path_length(oracle_mod):
    """d log p / d a = -L for every path (a enters p only through e^{-a L});
    with a = 1 / lambda_a, d log p / d lambda_a = a^2 L."""
    w = W.single_target(4.0, 0.165, 3.0, 30.0, 0.9, chains=1, cap=16, emit_kind=W.EMIT_VMF, emit_param=3.0,
                        det_kind=W.DET_PAPER)
    orc = oracle_mod.Oracle(w)
    rng = np.random.default_rng(70)
    a = 1 / 30.0
    for x in _paths(orc, w, rng, 8, 20):
        gv, ds, da, dg = orc.grad(0, x)
        L = np.linalg.norm(np.diff(x, axis=0), axis=1).sum()
        assert da[0] == pytest.approx(a * a * L, rel=1e-13)
        # b enters as b^N e^{-b L}: d log p / d b = N / b - L
        b = 1 / 3.0
        assert ds[0] == pytest.approx(-b * b * ((len(x) - 2) / b - L), rel=1e-12, abs=1e-15)


@pytest.mark.slow
def test_intensity_gradient_matches_tracer(oracle_mod):
    """The score-identity estimator d log I / d theta = E_p[d log p / d theta]
    over the oracle sampler's paths against the tracer's own derivatives of
    the detected intensity: dI/da = -E[w L] (the weight is e^{-a L}) and
    dI/db = E[w (N/b - L)] (the flights are drawn from b e^{-b l})."""
    lam_s, lam_a = 4.0, 25.0
    a, b = 1 / lam_a, 1 / lam_s
    w = W.single_target(2.0, 0.165, lam_s, lam_a, 0.9, chains=256, cap=64, burn_in=800, seed=12)
    orc, n, L = _sector_snapshots(oracle_mod, w, 8000, every=20)
    # per-path scores (pinned against the oracle's gradient routine above):
    # d log p / d lambda_a = a^2 L and d log p / d lambda_s = -b^2 (N/b - L)
    groups = np.arange(n.shape[0]) % 16
    sa = a * a * L
    sb = -b * b * ((n - 2) / b - L)
    tr = orc.trace_full(0, 24_000_000, esc=500.0)
    I, wL, wN = tr["I"], tr["wL"], tr["wN"]
    ta = a * a * wL[0] / I[0]
    tb = -b * b * (wN[0] / b - wL[0]) / I[0]
    se_ta = ta * math.hypot(wL[1] / wL[0], I[1] / I[0])
    se_tb = abs(tb) * (math.hypot(wN[1] / b, wL[1]) / abs(wN[0] / b - wL[0]) + I[1] / I[0])
    for est, ref, se_ref in ((sa, ta, se_ta), (sb, tb, se_tb)):
        per = [est[groups == g].mean() for g in range(16)]
        assert abs(est.mean() - ref) < 3.5 * math.hypot(_group_se(per), se_ref), (est.mean(), ref, se_ref)
    assert abs(sa.mean() / ta - 1) < 0.03
