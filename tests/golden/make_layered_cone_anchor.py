"""Writes layered_cone_anchor.txt: the oracle's single-scatter anchor I_3
(nested product Gauss rules over the emission cone, the ray and the sensor
cap) for cone-source targets of the 100-layer workload, at three
resolutions, so that the convergence of the quadrature is on record next to
the value the device anchor is compared with; and
layered_cone_anchor_sample.txt: the same at the two lower resolutions for a
seeded random sample of that workload's targets with n0 = 3, which puts a
number on the anchor error across the batch; and layered_cone_anchor_rim.txt:
two finer resolutions for the sampled targets whose sensor lies within a few
degrees outside the emission cone's rim, where the two lower ones disagree;
and layered_cone_anchor_devres.txt: the oracle's rule at the resolution the
device's anchor uses (32 x 32 directions, 64 x 64 within 10 degrees outside
a cone's rim; 32 radial nodes per layer piece; 8 x 8 cap nodes), to which the
device's value is held closely.  Calls only the oracle.

    python make_layered_cone_anchor.py [fixed|sample|rim|devres]   (default: all)"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

# targets (pair indices of the 100-layer, 1000-pair workload, seed 3) with
# n0 = 3 among the nearest, whose anchor the device is compared on
TARGETS = [877, 364, 321]
RULES = [(24, 24, 16, 10, 10), (40, 40, 24, 12, 12), (56, 56, 32, 16, 16)]
SAMPLE_SEED, SAMPLE_SIZE = 11, 40
# sampled targets with the sensor 0.95 and 3.1 degrees outside the cone's rim
RIM_TARGETS = [484, 269]
RIM_RULES = [(56, 56, 32, 16, 16), (64, 64, 48, 12, 12)]
# the device's resolution: two targets far from a rim (sensors 173 and 79
# degrees off the cone's axis), then three within 10 degrees outside it (0.95,
# 3.1 and 7.9 degrees)
DEVRES = [(128, (32, 32, 32, 8, 8)), (392, (32, 32, 32, 8, 8)),
          (484, (64, 64, 32, 8, 8)), (269, (64, 64, 32, 8, 8)), (877, (64, 64, 32, 8, 8))]


def _workload():
    from paper_1811_04156_amd import workloads as W
    return W.layered_pairs(seed=3, pairs=1000, chains=1000, cap=512)


def one(t, rules=RULES):
    from oracle import oracle as O
    w = _workload()
    orc = O.Oracle(w)
    return t, int(w["t_n0"][t]), [orc.anchor_I3(t, *r) for r in rules]


def one_low_mid(t):
    return one(t, RULES[:2])


def one_rim(tr):
    t, r = tr
    return t, one(t, [r])[2][0]


def sample_targets():
    """SAMPLE_SIZE targets drawn without replacement (seeded) from those with
    n0 = 3, the fixed ones left out."""
    import numpy as np
    n0 = np.asarray(_workload()["t_n0"])
    pool = [t for t in np.flatnonzero(n0 == 3).tolist() if t not in TARGETS]
    rng = np.random.default_rng(SAMPLE_SEED)
    return sorted(int(t) for t in rng.choice(pool, SAMPLE_SIZE, replace=False))


def write_sample():
    ts = sample_targets()
    with ProcessPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        rows = list(ex.map(one_low_mid, ts))
    with open(os.path.join(HERE, "layered_cone_anchor_sample.txt"), "w") as f:
        f.write("# Single-scatter anchor I_3 of a seeded random sample (seed %d, %d targets) of the n0 = 3\n"
                % (SAMPLE_SEED, SAMPLE_SIZE))
        f.write("# targets of the 100-layer, 1000-pair workload (seed 3), by the oracle's nested product\n")
        f.write("# Gauss rules at resolutions " + "; ".join("x".join(map(str, r)) for r in RULES[:2]) + "\n")
        f.write("# target n0 I3_low I3_mid\n")
        for t, n0, v in rows:
            f.write(f"{t} {n0} " + " ".join(f"{x:.15e}" for x in v) + "\n")



def write_fixed():
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


def write_rim():
    jobs = [(t, r) for t in RIM_TARGETS for r in RIM_RULES]
    with ProcessPoolExecutor(len(jobs)) as ex:
        vals = list(ex.map(one_rim, jobs))
    with open(os.path.join(HERE, "layered_cone_anchor_rim.txt"), "w") as f:
        f.write("# Single-scatter anchor I_3 of sampled targets of the 100-layer, 1000-pair workload (seed 3)\n")
        f.write("# whose sensor lies just outside the emission cone's rim, by the oracle's nested product\n")
        f.write("# Gauss rules at resolutions " + "; ".join("x".join(map(str, r)) for r in RIM_RULES) + "\n")
        f.write("# target I3_fine1 I3_fine2\n")
        for t in RIM_TARGETS:
            f.write(f"{t} " + " ".join(f"{v:.15e}" for tt, v in vals if tt == t) + "\n")


def write_devres():
    with ProcessPoolExecutor(len(DEVRES)) as ex:
        vals = list(ex.map(one_rim, DEVRES))
    with open(os.path.join(HERE, "layered_cone_anchor_devres.txt"), "w") as f:
        f.write("# Single-scatter anchor I_3 of targets of the 100-layer, 1000-pair workload (seed 3) by the\n")
        f.write("# oracle's nested product Gauss rules at the device anchor's resolution\n")
        f.write("# target n_polar n_azimuth n_radial n_cap_v n_cap_psi I3\n")
        for (t, r), (_, v) in zip(DEVRES, vals):
            f.write(f"{t} " + " ".join(map(str, r)) + f" {v:.15e}\n")


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("fixed", "all"):
        write_fixed()
    if which in ("sample", "all"):
        write_sample()
    if which in ("rim", "all"):
        write_rim()
    if which in ("devres", "all"):
        write_devres()
