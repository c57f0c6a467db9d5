"""Shared helpers of the GPU parity tests: workloads, random paths and the
lock-step replay of device steps on the oracle."""
import math

import numpy as np

from paper_1811_04156_amd import workloads as W

EPS32 = 2.0 ** -24  # unit roundoff of FP32
# Safety factor of the a-priori FP32 error bound of one proposal's log A (see
# fp32_logA_bound): about 100 FP32 operations per log-density change, each
# adding at most one rounding, condition numbers from the gradient.
K_BOUND = 32.0
BASE_BOUND = 1e-4  # rounding of the sum of about 20 local terms of magnitude <= 10


def mixed_workload(cap=48, chains=256, seed=5):
    """Layered medium (12 layers of 6 m, simplified-Liu mixture in every third
    layer, g from 0.8 to 0.95), 8 pairs: isotropic, vMF and cone sources, both
    detection kinds."""
    w = W.layered_pairs(seed=seed, pairs=8, chains=chains, cap=cap, n_layers=12, dz=6.0, dmin=5.0, dmax=30.0,
                        emit_kind=W.EMIT_ISO)
    kind = np.array([0, 1, 2, 0, 1, 2, 0, 0], np.int32)
    param = np.array([0, 3.0, math.radians(60), 0, 8.0, math.radians(75), 0, 0])
    det = np.array([0, 1, 0, 1, 0, 1, 0, 1], np.int32)
    src, sen, rad, ax = w["t_src"], w["t_sensor"], w["t_radius"], w["t_emit_dir"]
    n_init, init = W._cone_start(src, sen, rad, ax, np.where(kind == 2, param, np.pi))
    w.update(W._targets(w["t_medium"], src, sen, rad, kind, ax, param, n_init, init, det,
                        np.tile([0.0, -1.0, 0.0], (8, 1))))
    w["f_sl"] = np.where(np.arange(12) % 3 == 0, 0.45, 0.0)
    w["g"] = np.linspace(0.8, 0.95, 12)
    return w


def random_paths(orc, w, rng, nmax):
    """Random ragged paths with finite density (n in [2, nmax])."""
    C = len(w["c_target"])
    cap = int(w["cap"])
    n = np.zeros(C, np.int32)
    V = np.zeros((C, cap, 3))
    for c in range(C):
        t = int(w["c_target"][c])
        eta = w["t_sensor"][t] - w["t_src"][t]
        R = w["t_radius"][t]
        ax = w["t_emit_dir"][t]
        for _ in range(200):
            k = int(rng.integers(2, nmax + 1))
            v = np.zeros((k, 3))
            if k > 2:
                d = ax * rng.uniform(1, 4) + rng.normal(size=3) * 0.3
                v[1] = d
                for i in range(2, k - 1):
                    v[i] = v[i - 1] + (eta - v[i - 1]) / (k - i) + rng.normal(size=3) * 1.5
            dd = v[k - 2] - eta
            dd /= np.linalg.norm(dd)
            e = dd + 0.4 * rng.normal(size=3)
            e /= np.linalg.norm(e)
            if e @ dd < 0.3:
                e = dd
            v[k - 1] = eta + R * e
            if np.isfinite(orc.logp(t, v)):
                break
        n[c] = k
        V[c, :k] = v
    return n, V


def _window(move, idx, n):
    """Vertices of the current path x and of the proposal y that enter the
    device's local evaluation of log A."""
    if move in (0, 1, 6):  # single-vertex perturbation of vertex idx
        w = [k for k in range(idx - 2, idx + 3) if 1 <= k <= n - 1]
        return w, w
    if move == 2:  # birth on segment idx: y has n + 1 vertices, the new one at idx + 1
        return ([k for k in range(idx - 1, idx + 3) if 1 <= k <= n - 1],
                [k for k in range(idx - 1, idx + 4) if 1 <= k <= n])
    if move == 3:  # death of vertex idx: y has n - 1 vertices
        return ([k for k in range(idx - 2, idx + 3) if 1 <= k <= n - 1],
                [k for k in range(idx - 2, idx + 2) if 1 <= k <= n - 2])
    return list(range(1, n)), list(range(1, n))  # joint move of every interior vertex


def fp32_logA_bound(orc, t, x, y, move, idx):
    """A-priori bound of the FP32 error of one proposal's log A, computed from
    the oracle's FP64 state (never from the device's result):
    BASE_BOUND + K_BOUND * eps32 * sum over the vertices v that the local
    evaluation reads of |d log p / d v|_1 (|v|_1 + 1 m).  Coordinates of
    magnitude |v| carry FP32 rounding eps32 |v|, and every difference,
    direction and length the evaluation forms from them inherits it; the
    gradient turns that into log p, including the ill-conditioned short
    segments next to a vertex (where |d log p / d v| ~ 2 / length)."""
    n = len(x)
    wx, wy = _window(move, idx, n)
    gx = orc.grad(t, x, params=False)
    b = sum(np.abs(gx[k]).sum() * (np.abs(x[k]).sum() + 1.0) for k in wx)
    if y is not None and np.isfinite(orc.logp(t, y)):
        gy = orc.grad(t, y, params=False)
        b += sum(np.abs(gy[k]).sum() * (np.abs(y[k]).sum() + 1.0) for k in wy)
    return BASE_BOUND + K_BOUND * EPS32 * b


def lockstep(rj, w, steps, burn=50, block=0, v_lds=0):
    """Runs `steps` single device steps (FP32) and replays each on the oracle
    from the device's own pre-step state with the same random stream.
    Returns a dict of counts and the per-record FP32 error ratios."""
    import torch
    from oracle import oracle as O
    orc = O.Oracle(w)
    s = rj.Sampler(w, precision="f32")
    s.run(burn, block=block, v_lds=v_lds)
    out = dict(total=0, agree=0, compared=0, near=0, seg_mismatch=0, births=0, ratio=[], dA=[], n_max=0,
               records=0)
    for _ in range(steps):
        n0, V0 = s.get_state()
        step = s.step
        tr, _ = s.run(1, trace=True, block=block, v_lds=v_lds)
        g = tr.cpu().numpy()[:, 0]
        n1, V1 = s.get_state()
        assert s.status.sum().item() == 0
        out["n_max"] = max(out["n_max"], int(n0.max()))
        for c in range(len(n0)):
            t = int(w["c_target"][c])
            x = V0[c, : n0[c]]
            n, v, rec, y = orc.step(w, c, t, int(n0[c]), x, step, proposal=True)
            out["records"] += 1
            assert g[c, 0] == rec[0], (c, step, g[c], rec)
            assert abs(g[c, 4] - rec[4]) <= 4 * EPS32 * abs(rec[4]) + 1e-7
            if rec[0] == 2:
                out["births"] += 1
            if g[c, 2] != rec[2]:
                assert rec[0] == 2, (c, step, g[c], rec)  # only the birth segment choice can differ
                out["seg_mismatch"] += 1
                continue
            assert np.isfinite(g[c, 3]) == np.isfinite(rec[3]), (c, step, g[c], rec)
            bound = BASE_BOUND
            if np.isfinite(rec[3]):
                bound = fp32_logA_bound(orc, t, x, y, int(rec[0]), int(rec[2]))
                d = abs(g[c, 3] - rec[3])
                out["compared"] += 1
                out["dA"].append(d)
                out["ratio"].append(d / bound)
            margin = bound + 1e-5
            if abs(rec[3] - rec[4]) > margin or not np.isfinite(rec[3]):
                out["total"] += 1
                same = g[c, 1] == rec[1]
                out["agree"] += same
                if same:
                    # the accepted path is the FP32 rounding of the oracle's proposal
                    assert n1[c] == n
                    assert np.allclose(V1[c, :n], v, atol=2e-4, rtol=1e-5), (c, step)
            else:
                out["near"] += 1
    out["ratio"] = np.array(out["ratio"])
    out["dA"] = np.array(out["dA"])
    torch.cuda.synchronize()
    return out
