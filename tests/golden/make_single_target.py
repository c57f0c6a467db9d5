"""Writes single_target.txt: the oracle's analog tracer on one isotropic
source and a sensor of radius 0.165 m at 6 m in a homogeneous medium
(scattering length 3 m, absorption length 60 m, g = 0.9): detected intensity
per photon and its split by scatter count (0 .. 6, then >= 7), each as
(mean, standard error).  The reference of the samplers' long-run
intensity and sector occupancy.  Calls only the oracle."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

NPHOT = 600_000_000
ESC = 300.0

if __name__ == "__main__":
    from oracle import oracle as O
    from paper_1811_04156_amd import workloads as W
    w = W.single_target(6.0, 0.165, 3.0, 60.0, 0.9, chains=1, cap=64)
    r = O.Oracle(w).trace_full(0, NPHOT, seed=2024, esc=ESC)
    with open(os.path.join(HERE, "single_target.txt"), "w") as f:
        f.write("# Analog tracer (oracle): isotropic source, sensor R = 0.165 m at 6 m, lambda_s = 3 m, lambda_a = 60 m,\n")
        f.write(f"# g = 0.9 (pure HG); {NPHOT} photons, escape radius {ESC} m.\n")
        f.write("# I se_I, then 8 pairs: detected weight per photon after k = 0..6 and >= 7 scatterings (mean, se)\n")
        f.write(f"{r['I'][0]:.10e} {r['I'][1]:.10e} " + " ".join(f"{m:.10e} {s:.10e}" for m, s in r["bucket"]) + "\n")
