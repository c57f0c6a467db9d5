"""The oracle's light-yield map T between paths ending on two sensors of one
source (App. "Relative light yield transformation") and the bridge ratio it
feeds (Sec. "Comparison of relative light yield").  CPU only.

Pins, none of which re-types the map:
  - T^-1 . T is the identity and the two report the same log-Jacobian;
  - the determinant of the numerical derivative of one interior vertex's
    image equals the reported per-vertex factor, and the area ratio of the end
    point's image, measured from two tangent directions, equals the reported
    end factor (with two different sensor radii);
  - the path along the straight axis toward sensor 0 becomes a circular arc
    that leaves the source along the emission axis and passes through the
    centre of sensor 1, ending one sensor radius (of arc) short of it;
  - on the direct sector (n = 2), integrating p_1(T x) |dT/dx| over sensor 0's
    surface by plain Monte Carlo gives sensor 1's direct intensity from the
    anchor quadrature (change of variables), and p_0 gives sensor 0's;
  - the two sides of the bridge ratio are reciprocal: side 1 at T x equals
    minus side 0 at x.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_1811_04156_amd import workloads as W

R0, R1 = 0.15, 0.4


@pytest.fixture(scope="module")
def sc():
    w = W.two_region(b1=0.2, scale=0.1, radius=(R0, R1), chains_per_sensor=1, cap=16)
    return w, Oracle(w)


def _geom(w):
    eta0 = w["t_sensor"][0] - w["t_src"][0]
    eta1 = w["t_sensor"][1] - w["t_src"][1]
    return eta0, eta1


def _near_axis_path(rng, w, n):
    """A path whose interior vertices scatter around the straight axis toward
    sensor 0 (inside the map's domain) and whose end lies on sensor 0's
    surface on the side facing the source."""
    eta0, _ = _geom(w)
    D = np.linalg.norm(eta0)
    k = eta0 / D
    v = np.zeros((n, 3))
    for i in range(1, n - 1):
        v[i] = k * D * rng.uniform(0.1, 0.9) + rng.normal(size=3) * 0.05 * D
    nu = -k + rng.normal(size=3) * 0.4
    nu /= np.linalg.norm(nu)
    v[-1] = eta0 + R0 * nu
    return v


def test_round_trip_and_end_on_sensor1(sc):
    w, orc = sc
    _, eta1 = _geom(w)
    rng = np.random.default_rng(3)
    for _ in range(50):
        x = _near_axis_path(rng, w, int(rng.integers(2, 9)))
        y, lj = orc.yield_map(0, 1, x)
        xb, lj2 = orc.yield_map(0, 1, y, inverse=True)
        assert np.isfinite(lj)
        np.testing.assert_allclose(xb, x, atol=1e-9 * np.linalg.norm(eta1))
        assert abs(lj - lj2) < 1e-9 * max(1.0, abs(lj))
        assert abs(np.linalg.norm(y[-1] - eta1) - R1) < 1e-10
        assert np.all(y[0] == 0)


def test_interior_vertex_jacobian_by_differences(sc):
    w, orc = sc
    rng = np.random.default_rng(4)
    end_term = 2 * math.log(R1 / R0)
    for _ in range(20):
        x = _near_axis_path(rng, w, 3)
        _, lj = orc.yield_map(0, 1, x)
        h = 1e-5 * np.linalg.norm(x[1])
        J = np.zeros((3, 3))
        for j in range(3):
            xp, xm = x.copy(), x.copy()
            xp[1, j] += h
            xm[1, j] -= h
            J[:, j] = (orc.yield_map(0, 1, xp)[0][1] - orc.yield_map(0, 1, xm)[0][1]) / (2 * h)
        assert abs(math.log(abs(np.linalg.det(J))) - (lj - end_term)) < 1e-7


def test_end_point_area_factor_by_differences(sc):
    w, orc = sc
    eta0, _ = _geom(w)
    rng = np.random.default_rng(5)
    for _ in range(20):
        x = _near_axis_path(rng, w, 2)
        nu = (x[-1] - eta0) / R0
        a = np.cross(nu, rng.normal(size=3))
        a /= np.linalg.norm(a)
        b = np.cross(nu, a)
        h = 1e-6

        def end(d):
            m = nu + d
            y = x.copy()
            y[-1] = eta0 + R0 * m / np.linalg.norm(m)
            return orc.yield_map(0, 1, y)[0][-1]

        da = (end(h * a) - end(-h * a)) / (2 * h * R0)
        db = (end(h * b) - end(-h * b)) / (2 * h * R0)
        ratio = np.linalg.norm(np.cross(da, db))
        _, lj = orc.yield_map(0, 1, x)
        assert abs(math.log(ratio) - lj) < 1e-6
        assert abs(lj - 2 * math.log(R1 / R0)) < 1e-12


def test_axis_becomes_arc_through_sensor1(sc):
    w, orc = sc
    eta0, eta1 = _geom(w)
    D0 = np.linalg.norm(eta0)
    k0 = eta0 / D0
    b0 = D0 - R0
    edir = w["t_emit_dir"][0]
    end = eta0 - R0 * k0

    def img(omega):
        x = np.array([[0.0, 0.0, 0.0], omega * b0 * k0, end])
        return orc.yield_map(0, 1, x)[0][1]

    # tangent at the source along the emission axis
    p = img(1e-7)
    assert np.linalg.norm(p / np.linalg.norm(p) - edir) < 1e-6
    # the arc is a circle through the source: find its radius from three points
    P = np.array([img(0.25), img(0.5), img(0.75)])
    a, b, c = np.linalg.norm(P[1] - P[2]), np.linalg.norm(P[0] - P[2]), np.linalg.norm(P[0] - P[1])
    s = 0.5 * (a + b + c)
    rc = a * b * c / (4 * math.sqrt(s * (s - a) * (s - b) * (s - c)))
    O = np.array([0.0, 0.0, 0.0])
    # the source lies on the same circle: distance from the circumcentre
    A = np.array([P[1] - P[0], P[2] - P[0]])
    nrm = np.cross(A[0], A[1])
    M = np.array([A[0], A[1], nrm])
    rhs = np.array([0.5 * (P[1] @ P[1] - P[0] @ P[0]), 0.5 * (P[2] @ P[2] - P[0] @ P[0]), nrm @ P[0]])
    cen = np.linalg.solve(M, rhs)
    assert abs(np.linalg.norm(cen - O) - rc) < 1e-8 * rc
    assert abs(np.linalg.norm(cen - eta1) - rc) < 1e-8 * rc  # sensor 1's centre on the circle
    # the image of the axis end (omega = 1) lies one radius of arc before sensor 1's centre
    q = img(1.0)
    chord = np.linalg.norm(q - eta1)
    assert abs(chord - 2 * rc * math.sin(R1 / (2 * rc))) < 1e-9 * rc


def test_direct_sector_change_of_variables(sc):
    w, orc = sc
    eta0, _ = _geom(w)
    rng = np.random.default_rng(6)
    N = 60_000
    u = rng.normal(size=(N, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q0 = np.zeros(N)
    q1 = np.zeros(N)
    for i in range(N):
        x = np.array([[0.0, 0.0, 0.0], eta0 + R0 * u[i]])
        q0[i] = math.exp(orc.logp(0, x))
        y, lj = orc.yield_map(0, 1, x)
        q1[i] = math.exp(orc.logp(1, y) + lj)
    area = 4 * math.pi * R0 * R0
    for q, t in ((q0, 0), (q1, 1)):
        Z, se = area * q.mean(), area * q.std() / math.sqrt(N)
        ref = orc.anchor_I2(t)
        print(f"target {t}: Monte Carlo {Z:.6e} +- {se / Z:.2%}, quadrature {ref:.6e}")
        assert se / Z < 0.02
        assert abs(Z - ref) < 4 * se


def test_bridge_sides_are_reciprocal(sc):
    w, orc = sc
    rng = np.random.default_rng(7)
    for _ in range(30):
        x = _near_axis_path(rng, w, int(rng.integers(2, 8)))
        r0 = orc.yield_log_ratio(0, 1, 0, x)
        if not np.isfinite(r0):
            continue
        y, _ = orc.yield_map(0, 1, x)
        r1 = orc.yield_log_ratio(0, 1, 1, y)
        assert abs(r0 + r1) < 1e-8 * max(1.0, abs(r0))
