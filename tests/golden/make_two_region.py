"""Writes two_region.txt: the oracle's analog tracer on the paper's two-region
scenario (Sec. "Implementation", Fig. setup: regions split by the y-z plane
with scattering b0 = 0.3 and b1 per m, absorption 0.01 per m, vMF source with
kappa = 38, the simplified-Liu / Henyey-Greenstein mixture with mean cosine
0.95 and f_SL = 0.45, the paper's sensor response) with the sensor positions
scaled by 0.1 (sensors at 12 m and 12.7 m) so that analog tracing reaches a
few tenths of a percent.  Per b1 and sensor: the detected intensity and the
detected weight in path-length bins of 1 m (47 bins from 0, then overflow),
each as (mean, standard error) per photon.  Calls only the oracle."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

SCALE = 0.1
B1 = [0.1, 0.3]
NPHOT = 250_000_000
ESC = 200.0
LBIN = 1.0

if __name__ == "__main__":
    from oracle import oracle as O
    from paper_1811_04156_amd import workloads as W
    rows = []
    for b1 in B1:
        w = W.two_region(b1=b1, scale=SCALE, chains_per_sensor=1, cap=16)
        orc = O.Oracle(w)
        for t in (0, 1):
            r = orc.trace_full(t, NPHOT, seed=1000 + t + int(100 * b1), esc=ESC, lbin=LBIN)
            rows.append((b1, t, r["I"], r["lhist"]))
            print(b1, t, r["I"], flush=True)
    with open(os.path.join(HERE, "two_region.txt"), "w") as f:
        f.write("# Analog tracer (oracle) on the two-region scenario with sensor positions scaled by "
                f"{SCALE}: b0 = 0.3 /m, a = 0.01 /m,\n")
        f.write(f"# {NPHOT} photons per sensor, escape radius {ESC} m, path-length bins of {LBIN} m from 0 "
                "(47 bins, then overflow).\n")
        f.write("# b1 sensor I se_I  then 48 pairs (weight per photon in the bin, its se)\n")
        for b1, t, I, lh in rows:
            f.write(f"{b1} {t} {I[0]:.10e} {I[1]:.10e} " + " ".join(f"{m:.10e} {s:.10e}" for m, s in lh) + "\n")
