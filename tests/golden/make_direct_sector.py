"""Writes direct_sector.txt: the textbook direct-sector integral by adaptive
quadrature (scipy), for the cases pinned in the oracle tests."""
import os

import numpy as np
from scipy.integrate import quad

CASES = [(10.0, 0.165, 0.0), (10.0, 0.165, 0.01), (10.0, 0.165, 0.05), (2.0, 0.165, 0.05),
         (50.0, 0.165, 0.09), (1.0, 0.3, 0.2)]


def i2(D, R, c):
    th = np.arcsin(R / D)
    f = lambda t: 0.5 * np.sin(t) * np.exp(-c * (D * np.cos(t) - np.sqrt(max(0.0, R * R - (D * np.sin(t)) ** 2))))
    return quad(f, 0.0, th, epsabs=0.0, epsrel=1e-13, limit=200)[0]


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "direct_sector.txt")
    head = [l for l in open(path) if l.startswith("#")]
    with open(path, "w") as f:
        f.writelines(head)
        for D, R, c in CASES:
            f.write(f"{D:.6g} {R:.6g} {c:.6g} {i2(D, R, c):.15e}\n")
