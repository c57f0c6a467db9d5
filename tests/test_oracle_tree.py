"""Pins of the oracle's tree coordinates and of the global move built on them
(App. "Path space coordinate system"; Sec. "Path proposal distribution").
CPU only.

  - coordinates -> path -> coordinates is the identity, and both directions
    report the same log-Jacobian;
  - the reported log-Jacobian equals the log-determinant of the numerical
    derivative of the whole map (all interior coordinates -> all interior
    vertices), so the product form, the sech^2 reading of the printed cosh^2
    and the frame hand-down from parent to child are checked together;
  - the move is a Gaussian random walk of variance mala_h / n in (zeta, t, phi)
    with the end point moved on the sensor, and its log A equals
    log p(y) - log p(x) + log|det| at y - log|det| at x with both
    determinants taken numerically.
The distribution the move leaves invariant is pinned against the tracer in
test_oracle_balance.py (sector occupancy and path length).
"""
import math

import numpy as np
import pytest

from paper_1811_04156_amd import workloads as W


def _path(rng, n, eta, R):
    v = np.zeros((n, 3))
    for i in range(1, n - 1):
        v[i] = eta * (i / (n - 1)) + rng.normal(size=3) * 0.4
    nu = -eta / np.linalg.norm(eta) + rng.normal(size=3) * 0.5
    v[-1] = eta + R * nu / np.linalg.norm(nu)
    return v


def _interior_map(O, f0, fend, z, t, ph):
    def fn(u):
        zz, tt, pp = z.copy(), t.copy(), ph.copy()
        n = len(z)
        zz[1:n - 1], tt[1:n - 1], pp[1:n - 1] = u[0::3], u[1::3], u[2::3]
        return O.tree_path(f0, fend, zz, tt, pp)[0][1:n - 1].reshape(-1)
    return fn


def _num_logdet(fn, u, h=1e-6):
    J = np.zeros((len(u), len(u)))
    for i in range(len(u)):
        up, um = u.copy(), u.copy()
        up[i] += h
        um[i] -= h
        J[:, i] = (fn(up) - fn(um)) / (2 * h)
    return np.linalg.slogdet(J)[1]


@pytest.fixture(scope="module")
def setup(oracle_mod):
    w = W.single_target(3.0, 0.3, 2.0, 20.0, 0.9, chains=1, cap=16, emit_kind=W.EMIT_VMF, emit_param=4.0,
                        emit_dir=(0.1, 0.2, 0.97), det_kind=W.DET_PAPER)
    eta = w["t_sensor"][0] - w["t_src"][0]
    return oracle_mod, w, eta, float(w["t_radius"][0])


def test_round_trip(setup):
    O, w, eta, R = setup
    rng = np.random.default_rng(1)
    for _ in range(60):
        n = int(rng.integers(2, 14))
        x = _path(rng, n, eta, R)
        z, t, ph, lj = O.tree_coords(x)
        y, lj2 = O.tree_path(x[0], x[-1], z, t, ph)
        np.testing.assert_allclose(y, x, atol=1e-10)
        assert abs(lj - lj2) < 1e-10 * max(1.0, abs(lj))
        assert np.all(np.abs(ph[1:n - 1]) <= math.pi)


@pytest.mark.parametrize("n", [3, 4, 5, 7])
def test_jacobian_of_the_whole_map(setup, n):
    O, w, eta, R = setup
    rng = np.random.default_rng(10 + n)
    for _ in range(6):
        x = _path(rng, n, eta, R)
        z, t, ph, lj = O.tree_coords(x)
        u = np.stack([z[1:n - 1], t[1:n - 1], ph[1:n - 1]], axis=1).reshape(-1)
        ld = _num_logdet(_interior_map(O, x[0], x[-1], z, t, ph), u)
        assert abs(ld - lj) < 1e-6 * max(1.0, abs(lj)), (ld, lj)


def test_move_is_a_coordinate_random_walk_with_numerical_jacobians(setup):
    O, w, eta, R = setup
    orc = O.Oracle(w)
    h = 0.3
    run = dict(seed=0, burn_in=0, cycle_len=5, n_perturb=3, birth_frac=0.5, sigma=1.0, kappa_end=20.0,
               sampler=3, mala_h=h)
    rng = np.random.default_rng(4)
    checked = 0
    for _ in range(24):
        n = int(rng.integers(3, 7))
        x = _path(rng, n, eta, R)
        u = rng.uniform(0.02, 0.98, 2 + 4 * (n - 2))
        y, logA, mv = orc.propose(run, 0, x, 4, 0, u)
        assert mv == 7 and y is not None and len(y) == n
        assert abs(np.linalg.norm(y[-1] - eta) - R) < 1e-12
        zx, tx, px, _ = O.tree_coords(x)
        zy, ty, py, _ = O.tree_coords(y)
        sig = math.sqrt(h / n)
        for k in range(1, n - 1):
            q = u[2 + 4 * (k - 1): 6 + 4 * (k - 1)]
            r1, r2 = math.sqrt(-2 * math.log(q[0])), math.sqrt(-2 * math.log(q[2]))
            xi = np.array([r1 * math.cos(2 * math.pi * q[1]), r1 * math.sin(2 * math.pi * q[1]),
                           r2 * math.cos(2 * math.pi * q[3])])
            assert abs(zy[k] - zx[k] - sig * xi[0]) < 1e-8
            assert abs(ty[k] - tx[k] - sig * xi[1]) < 1e-8
            dphi = (py[k] - px[k] - sig * xi[2] + math.pi) % (2 * math.pi) - math.pi
            assert abs(dphi) < 1e-8
        if not np.isfinite(orc.logp(0, y)):
            assert logA == -np.inf  # e.g. the new end point faces away from the last segment
            continue
        checked += 1
        ux = np.stack([zx[1:n - 1], tx[1:n - 1], px[1:n - 1]], axis=1).reshape(-1)
        uy = np.stack([zy[1:n - 1], ty[1:n - 1], py[1:n - 1]], axis=1).reshape(-1)
        ldx = _num_logdet(_interior_map(O, x[0], x[-1], zx, tx, px), ux)
        ldy = _num_logdet(_interior_map(O, y[0], y[-1], zy, ty, py), uy)
        ref = orc.logp(0, y) - orc.logp(0, x) + ldy - ldx
        assert abs(logA - ref) < 1e-5 * max(1.0, abs(ref)), (logA, ref)
    assert checked >= 10
