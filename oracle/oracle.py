"""ctypes binding of the FP64 CPU oracle (``oracle/rjoracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product library never
imports this module.  It takes the plain arrays of
``paper_1811_04156_amd.workloads`` and nothing from the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rjoracle.cpp")
LIB = os.path.join(HERE, "librjoracle.so")

NSTAT = 16
MOVE_NAMES = ["interior", "end", "birth", "death", "mala", "null", "local_mala"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (host only)."""
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", LIB, SRC, "-lpthread"]
        subprocess.run(cmd, check=True)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        d, i, u32, u64, i64, p = C.c_double, C.c_int, C.c_uint32, C.c_uint64, C.c_int64, C.c_void_p
        sig = {
            "orc_philox": (None, [p, p, p]),
            "orc_step_draws": (None, [u64, u32, u64, p]),
            "orc_unif": (d, [u32]),
            "orc_p_hg": (d, [d, d]), "orc_p_sl": (d, [d, d]), "orc_sigma_sr": (d, [d, d, d]),
            "orc_q_s": (d, [d, d]), "orc_q_t": (d, [d]), "orc_jac_bisph": (d, [d, d, d]),
            "orc_kappa_eq": (d, [d]), "orc_sample_cos_s": (d, [d, d]),
            "orc_bisph": (None, [p, p, d, d, d, p]), "orc_bisph_inv": (None, [p, p, p, p]),
            "orc_onb": (None, [p, p, p]),
            "orc_create": (p, [i, p, p, p, p, p, p, p, p, i, p, p, p, p, p, p, p, p, p, p, p, i]),
            "orc_destroy": (None, [p]),
            "orc_logp": (d, [p, i, i, p]),
            "orc_tau": (d, [p, i, p, p, i]),
            "orc_beta": (d, [p, i, p, p]),
            "orc_grad": (None, [p, i, i, p, p, p, p, p]),
            "orc_step": (None, [p, p, p, u32, i, p, p, p, p, p]),
            "orc_propose": (d, [p, p, p, i, i, i, p, i, p, p, p, p]),
            "orc_run": (None, [p, p, p, i, p, p, p, p, p, p, i]),
            "orc_anchor_I2": (d, [p, i, i, i]),
            "orc_anchor_I3": (d, [p, i, i, i, i, i, i]),
            "orc_trace": (None, [p, i, u64, i64, d, d, i, p]),
            "orc_trace_tallies": (i, []),
            "orc_yield_map": (d, [p, i, i, i, i, p, p]),
            "orc_yield_log_ratio": (d, [p, i, i, i, i, p]),
            "orc_tree_coords": (d, [i, p, p, p, p]),
            "orc_tree_path": (d, [i, p, p, p, p, p, p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------------------
# scalar helpers (closed forms of the paper)
# ---------------------------------------------------------------------------
def tree_coords(verts):
    """Tree coordinates (zeta, t, phi), each (n,) by vertex index, of a path
    and log |d path / d coordinates|."""
    v = _f64(verts).reshape(-1, 3)
    n = len(v)
    z, t, ph = np.zeros(n), np.zeros(n), np.zeros(n)
    lj = lib().orc_tree_coords(n, _ptr(v), _ptr(z), _ptr(t), _ptr(ph))
    return z, t, ph, lj


def tree_path(f0, fend, zeta, t, phi):
    """The path with end points f0, fend and interior tree coordinates; returns
    (path (n, 3), log-Jacobian)."""
    z, tt, ph = _f64(zeta), _f64(t), _f64(phi)
    n = len(z)
    out = np.zeros((n, 3))
    lj = lib().orc_tree_path(n, _ptr(_f64(f0)), _ptr(_f64(fend)), _ptr(z), _ptr(tt), _ptr(ph), _ptr(out))
    return out, lj


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def step_draws(seed, chain, step):
    out = np.zeros(8, np.uint32)
    lib().orc_step_draws(seed, chain, step, _ptr(out))
    return out


def unif(x):
    return lib().orc_unif(int(x))


def p_hg(mu, G):
    return lib().orc_p_hg(mu, G)


def p_sl(mu, G):
    return lib().orc_p_sl(mu, G)


def sigma_sr(mu, G, fsl):
    return lib().orc_sigma_sr(mu, G, fsl)


def q_s(s, beta):
    return lib().orc_q_s(s, beta)


def q_t(t):
    return lib().orc_q_t(t)


def jac_bisph(s, t, gam):
    return lib().orc_jac_bisph(s, t, gam)


def kappa_eq(G):
    return lib().orc_kappa_eq(G)


def sample_cos_s(u, beta):
    return lib().orc_sample_cos_s(u, beta)


def bisph(A, B, s, t, phi):
    out = np.zeros(3)
    lib().orc_bisph(_ptr(_f64(A)), _ptr(_f64(B)), s, t, phi, _ptr(out))
    return out


def bisph_inv(A, B, f):
    out = np.zeros(3)
    lib().orc_bisph_inv(_ptr(_f64(A)), _ptr(_f64(B)), _ptr(_f64(f)), _ptr(out))
    return out


def onb(n):
    a, b = np.zeros(3), np.zeros(3)
    lib().orc_onb(_ptr(_f64(n)), _ptr(a), _ptr(b))
    return a, b


def birth_thresh(frac):
    return int(min(max(round(frac * 2.0**32), 0), 2**32 - 1))


# ---------------------------------------------------------------------------
# workload context
# ---------------------------------------------------------------------------
class Oracle:
    """FP64 oracle bound to one workload (media + targets)."""

    def __init__(self, w, logw=None):
        self.w = w
        self.cap = int(w["cap"])
        self._keep = [
            _f64(w["m_axis"]), _i32(w["m_layer_off"]), _i32(w["m_layer_cnt"]), _f64(w["edges"]),
            _f64(w["lam_s"]), _f64(w["lam_a"]), _f64(w["g"]), _f64(w["f_sl"]),
            _i32(w["t_medium"]), _f64(w["t_src"]), _f64(w["t_sensor"]), _f64(w["t_radius"]),
            _i32(w["t_emit_kind"]), _f64(w["t_emit_dir"]), _f64(w["t_emit_param"]),
            _i32(w["t_det_kind"]), _f64(w["t_det_dir"]), _i32(w["t_n0"]),
            None if logw is None else _f64(logw),
        ]
        k = self._keep
        self.h = lib().orc_create(
            len(w["m_layer_cnt"]), _ptr(k[0]), _ptr(k[1]), _ptr(k[2]), _ptr(k[3]), _ptr(k[4]),
            _ptr(k[5]), _ptr(k[6]), _ptr(k[7]), len(w["t_src"]), _ptr(k[8]), _ptr(k[9]),
            _ptr(k[10]), _ptr(k[11]), _ptr(k[12]), _ptr(k[13]), _ptr(k[14]), _ptr(k[15]),
            _ptr(k[16]), _ptr(k[17]), _ptr(k[18]), self.cap)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    # -- density ----------------------------------------------------------
    def logp(self, t, verts):
        v = _f64(verts).reshape(-1, 3)
        return lib().orc_logp(self.h, int(t), len(v), _ptr(v))

    def tau(self, t, P, Q, which):
        return lib().orc_tau(self.h, int(t), _ptr(_f64(P)), _ptr(_f64(Q)), 0 if which == "a" else 1)

    def beta(self, t, A, B):
        return lib().orc_beta(self.h, int(t), _ptr(_f64(A)), _ptr(_f64(B)))

    def grad(self, t, verts, params=True):
        v = _f64(verts).reshape(-1, 3)
        gv = np.zeros_like(v)
        med = int(self.w["t_medium"][t])
        L = int(self.w["m_layer_cnt"][med])
        ds, da, dg = np.zeros(L), np.zeros(L), np.zeros(L)
        lib().orc_grad(self.h, int(t), len(v), _ptr(v), _ptr(gv), _ptr(ds) if params else None,
                       _ptr(da), _ptr(dg))
        return (gv, ds, da, dg) if params else gv

    # -- sampler ----------------------------------------------------------
    def _params(self, run, step0, steps):
        ip = np.array([run["seed"], step0, run["burn_in"], steps, run["cycle_len"], run["n_perturb"],
                       birth_thresh(run["birth_frac"]), run.get("sampler", 0)], np.uint64)
        dp = np.array([run["sigma"], run["kappa_end"], run.get("mala_h", 0.05)], np.float64)
        return ip, dp

    def step(self, run, chain, t, n, verts, step, proposal=False):
        """One step of one chain; returns (n, verts, record) and, if asked,
        the proposed path (None when the step made no proposal)."""
        ip, dp = self._params(run, step, 1)
        v = np.zeros((self.cap, 3))
        v[:n] = np.asarray(verts)[:n]
        nn = C.c_int(int(n))
        rec = np.zeros(5)
        npr = C.c_int(0)
        pr = np.zeros((self.cap + 1, 3)) if proposal else None
        lib().orc_step(self.h, _ptr(ip), _ptr(dp), int(chain), int(t), C.byref(nn), _ptr(v), _ptr(rec),
                       C.byref(npr), _ptr(pr))
        out = (nn.value, v[: nn.value].copy(), rec)
        if proposal:
            return out + ((pr[: npr.value].copy() if npr.value else None),)
        return out

    def propose(self, run, t, verts, kind, idx, u):
        """One proposal from continuous draws u (see orc_propose): returns
        (proposed path or None, log A, move code)."""
        ip, dp = self._params(run, 0, 1)
        v = _f64(verts).reshape(-1, 3)
        uu = _f64(u)
        y = np.zeros((len(v) + 1, 3))
        ny, mv = C.c_int(0), C.c_int(0)
        la = lib().orc_propose(self.h, _ptr(ip), _ptr(dp), int(t), int(kind), len(v), _ptr(v), int(idx), _ptr(uu),
                               C.byref(ny), _ptr(y), C.byref(mv))
        return (y[: ny.value].copy() if ny.value else None), la, mv.value

    def run(self, run, state, steps, step0=0, trace=False, threads=None, chain_ids=None):
        """Advance every chain of ``state`` (dict with target, n, verts (C, cap, 3)) by
        ``steps`` steps in place; returns per-chain stats (C, 16) and the optional
        trace (C, steps, 5)."""
        Cn = len(state["target"])
        ip, dp = self._params(run, step0, steps)
        tgt = _i32(state["target"])
        n = _i32(state["n"])
        v = _f64(state["verts"])
        ids = _i32(np.arange(Cn) if chain_ids is None else chain_ids)
        stats = np.zeros((Cn, NSTAT))
        tr = np.zeros((Cn, steps, 5)) if trace else None
        th = threads or max(1, min(os.cpu_count() or 1, Cn))
        lib().orc_run(self.h, _ptr(ip), _ptr(dp), Cn, _ptr(ids), _ptr(tgt), _ptr(n), _ptr(v), _ptr(stats),
                      _ptr(tr), int(th))
        state["n"], state["verts"] = n, v
        return stats, tr

    # -- relative light yield ------------------------------------------------
    def yield_map(self, t0, t1, verts, inverse=False):
        """The light-yield map T (or its inverse) of a path between targets t0
        and t1; returns (mapped path, log |det dT/dx| at the sensor-0 path)."""
        v = _f64(verts).reshape(-1, 3)
        out = np.zeros_like(v)
        lj = lib().orc_yield_map(self.h, int(t0), int(t1), 1 if inverse else 0, len(v), _ptr(v), _ptr(out))
        return out, lj

    def yield_log_ratio(self, t0, t1, side, verts):
        """Bridge log-ratio of one path: log q1/q0 (side 0, a sensor-0 path)
        or log q0/q1 at T^-1(y) (side 1, a sensor-1 path)."""
        v = _f64(verts).reshape(-1, 3)
        return lib().orc_yield_log_ratio(self.h, int(t0), int(t1), int(side), len(v), _ptr(v))

    # -- anchors and tracer -------------------------------------------------
    def anchor_I2(self, t, nv=48, npsi=48):
        return lib().orc_anchor_I2(self.h, int(t), nv, npsi)

    def anchor_I3(self, t, nth=24, nps=24, nr=48, nv=12, npsi=12):
        return lib().orc_anchor_I3(self.h, int(t), nth, nps, nr, nv, npsi)

    def trace(self, t, nphot, seed=12345, esc=None, threads=None):
        """Analog tracer: (mean, se) of the detected weight per photon and the
        per-scatter-count split (8, 2)."""
        r = self.trace_full(t, nphot, seed, esc, threads)
        return r["I"][0], r["I"][1], r["bucket"]

    def trace_full(self, t, nphot, seed=12345, esc=None, threads=None, lbin=0.0):
        """Analog tracer, every tally as (mean, se) per photon:
        I (2,) detected weight; bucket (8, 2) weight by scatter count (last: >= 7);
        bucket_L (8, 2) weight x path length by scatter count; wL (2,) weight x
        path length; wN (2,) weight x scatter count; lhist (48, 2) weight by
        path-length bin of width lbin (last bin: overflow)."""
        K = lib().orc_trace_tallies()
        out = np.zeros(2 * K)
        if esc is None:
            esc = 2000.0
        th = threads or (os.cpu_count() or 1)
        lib().orc_trace(self.h, int(t), seed, int(nphot), float(esc), float(lbin), int(th), _ptr(out))
        o = out.reshape(K, 2)
        return dict(I=o[0], bucket=o[1:9], bucket_L=o[9:17], wL=o[17], wN=o[18], lhist=o[19:])


def initial_state(w, chains=None):
    """Chains started from their target's starting path (float64, cap slots)."""
    tgt = np.asarray(w["c_target"] if chains is None else w["c_target"][:chains], np.int32)
    cap = int(w["cap"])
    Cn = len(tgt)
    v = np.zeros((Cn, cap, 3))
    n = np.asarray(w["t_init_n"])[tgt].astype(np.int32)
    v[:, :3] = np.asarray(w["t_init"])[tgt]
    return dict(target=tgt, n=n, verts=v)


def intensity(w, stats, anchors, groups=16):
    """Anchored tilted-sector estimate per target from per-chain statistics:
    I = I_{n0} * sum(1/w(n)) / sum(1[n = n0]/w(n0)), delete-one-group
    jackknife over ``groups`` chain groups of each target."""
    T = len(w["t_src"])
    tgt = np.asarray(w["c_target"][: len(stats)])
    I = np.full(T, np.nan)
    se = np.full(T, np.nan)
    for t in range(T):
        idx = np.nonzero(tgt == t)[0]
        if len(idx) == 0:
            continue
        g = np.arange(len(idx)) % groups
        A = np.array([stats[idx[g == k], 1].sum() for k in range(groups)])
        B = np.array([stats[idx[g == k], 2].sum() for k in range(groups)])
        if B.sum() <= 0:
            continue
        I[t] = anchors[t] * A.sum() / B.sum()
        G = min(groups, len(idx))
        jk = np.array([anchors[t] * (A.sum() - A[k]) / (B.sum() - B[k]) for k in range(G) if B.sum() > B[k]])
        if len(jk) == G:
            se[t] = np.sqrt((G - 1) / G * np.sum((jk - jk.mean()) ** 2))
    return I, se
