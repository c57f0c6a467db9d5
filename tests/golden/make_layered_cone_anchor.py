"""Writes layered_cone_anchor.txt: the oracle's single-scatter anchor I_3
(nested product Gauss rules over the emission cone, the ray and the sensor
cap) for cone-source targets of the 100-layer workload, at three
resolutions, so that the convergence of the quadrature is on record next to
the value the device anchor is compared with.  Calls only the oracle."""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

# targets (pair indices of the 100-layer, 1000-pair workload, seed 3) with
# n0 = 3 among the nearest, whose anchor the device is compared on
TARGETS = [877, 364, 321]
RULES = [(24, 24, 16, 10, 10), (40, 40, 24, 12, 12), (56, 56, 32, 16, 16)]


def one(t):
    from oracle import oracle as O
    from paper_1811_04156_amd import workloads as W
    w = W.layered_pairs(seed=3, pairs=1000, chains=1000, cap=512)
    orc = O.Oracle(w)
    return t, int(w["t_n0"][t]), [orc.anchor_I3(t, *r) for r in RULES]


if __name__ == "__main__":
    with ProcessPoolExecutor(len(TARGETS)) as ex:
        rows = list(ex.map(one, TARGETS))
    with open(os.path.join(HERE, "layered_cone_anchor.txt"), "w") as f:
        f.write("# Single-scatter anchor I_3 of cone-source targets of the 100-layer workload (10 m layers,\n")
        f.write("# lambda_s ~ logU[10,60] m, lambda_a ~ logU[40,250] m, g = 0.9; 20 deg cones; seed 3),\n")
        f.write("# by the oracle's nested product Gauss rules (App. \"Intermediate vertex\", \"Final vertex\"):\n")
        f.write("# resolutions " + "; ".join("x".join(map(str, r)) for r in RULES) + "\n")
        f.write("# target n0 I3_low I3_mid I3_high\n")
        for t, n0, v in rows:
            f.write(f"{t} {n0} " + " ".join(f"{x:.15e}" for x in v) + "\n")
