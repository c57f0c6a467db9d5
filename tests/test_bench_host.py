"""Host logic of bench.py (CPU): the evaluated-proposal count, the algorithmic
FLOP count behind roofline.frac, the median relative error, the proposal
tuner's candidates, the recorded HBM traffic and its source digest, and the
one-GPU rule of the command line."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _stats(rows):
    """Per-chain statistics rows from (counted, sum n, perturb, birth, death,
    jumps without an evaluation) tuples."""
    st = np.zeros((len(rows), 16))
    for i, (cnt, sn, pp, pb, pd, ne) in enumerate(rows):
        st[i, 0], st[i, 5], st[i, 6], st[i, 7], st[i, 8], st[i, 15] = cnt, sn, pp, pb, pd, ne
    return st


def test_evaluated_counts_only_proposals_with_a_density_change():
    st = _stats([(100, 600, 60, 20, 20, 3), (50, 200, 30, 10, 10, 0)])
    assert bench.evaluated(st) == 147.0


def test_flop_per_launch_follows_the_per_proposal_counts():
    st = _stats([(100, 600, 60, 20, 20, 3), (100, 800, 60, 20, 20, 1)])
    flop, nbar = bench.flop_per_launch(st, 3, 5)
    assert nbar == pytest.approx(7.0)
    jumps = 80 - 4
    ref = 120 * bench.FLOP_PERTURB + jumps * (bench.FLOP_JUMP_BASE + bench.FLOP_JUMP_PER_VERTEX * 7.0)
    assert flop == pytest.approx(ref)


def test_median_relative_error_skips_targets_without_an_estimate():
    I = np.array([1.0, 2.0, np.nan, 4.0, 0.0])
    se = np.array([0.01, 0.04, 0.1, 0.12, 0.1])
    r, k = bench.median_r(I, se)
    assert k == 3 and r == pytest.approx(0.02)


def test_proposal_candidates():
    w = dict(sigma=1.0, kappa_end=5.0, cycle_len=5, n_perturb=3, mala_h=0.05)
    plain = bench.proposal_candidates(w, "plain")
    assert plain[0] == w  # the workload's own proposal first
    assert {c["n_perturb"] for c in plain} == {2, 3, 4}
    # the plain grid crosses the same mixes with every step size as the Langevin one
    assert {(c["sigma"], c["n_perturb"]) for c in plain} >= {(s, k) for s in (0.5, 8.0, 16.0) for k in (2, 3, 4)}
    assert all(0 < c["n_perturb"] < c["cycle_len"] for c in plain)  # every mix keeps both move classes
    assert len({tuple(sorted(c.items())) for c in plain}) == len(plain)  # no candidate twice
    lang = bench.proposal_candidates(w, "langevin")
    assert {c["mala_h"] for c in lang} >= {0.02, 0.05, 0.1, 0.2, 0.5, 1.0}
    # sigma does not enter the Langevin step: its grid is step size x mix
    assert {c["sigma"] for c in lang} == {1.0}
    assert {(c["mala_h"], c["n_perturb"]) for c in lang} >= {(h, k) for h in (0.02, 1.0) for k in (2, 3, 4)}
    assert len({tuple(sorted(c.items())) for c in lang}) == len(lang)
    tree = bench.proposal_candidates(dict(w, mala_h=0.3), "tree")
    assert {c["mala_h"] for c in tree} >= {0.1, 0.3, 1.0}


def test_recorded_traffic_follows_the_kernel_sources(monkeypatch, tmp_path):
    text = open(os.path.join(ROOT, bench.TRAFFIC_PROFILE)).read()
    if "kernel_source_sha256: " + bench.kernel_digest() not in text:
        pytest.skip("the kernel sources changed since the traffic counters were recorded")
    v = bench.recorded_traffic()
    assert v is not None and v > 0
    # any change to a kernel source invalidates the record
    extra = tmp_path / "extra.h"
    extra.write_text("// a changed source\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", bench.KERNEL_SOURCES + [str(extra)])
    assert bench.recorded_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


class _FakeTuner:
    """Stands in for a Sampler: scores are fixed per candidate and trial length."""

    def __init__(self, short, long):
        self.short, self.long, self.calls = short, long, []

    def tune_proposal(self, cands, trial, run=None):
        self.calls.append((len(cands), trial))
        tab = self.short if trial == 100 else self.long
        sc = np.array([tab[c["id"]] for c in cands])
        return int(np.argmax(sc)), sc


def test_two_stage_tuner_takes_the_best_finalist_of_the_longer_trials():
    cands = [{"id": i} for i in range(6)]
    # the short trials rank 4 > 1 > 2; the longer ones put 2 first
    short = [1.0, 5.0, 4.0, 0.5, 6.0, 3.0]
    long = [9.0, 2.0, 3.0, 9.0, 1.0, 9.0]
    f = _FakeTuner(short, long)
    best, sc1, fin = bench.tune_two_stage(f, cands, 100)
    assert fin == [4, 1, 2] and best == 2
    assert f.calls == [(6, 100), (3, 1600)]
    assert list(sc1) == short
    # fewer candidates than finalists: all of them go through
    f = _FakeTuner(short, long)
    best, _, fin = bench.tune_two_stage(f, cands[:2], 100)
    assert sorted(fin) == [0, 1] and best == 0
