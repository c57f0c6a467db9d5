"""ctypes binding of librjpath.so (argument marshalling only).

Every numeric step runs in the HIP kernels behind the C ABI declared in
``include/rjpath.h``; PyTorch provides device memory and the stream.  If the
library is missing the import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librjpath.so")

RJPATH_OK, RJPATH_EINVAL, RJPATH_ENOMEM, RJPATH_EHIP, RJPATH_ENODATA, RJPATH_ENOTSUP = 0, -1, -2, -3, -4, -5
F32, F64 = 0, 1
PLAIN, MALA, LMALA, TREE = 0, 1, 2, 3
NSTAT = 16
TRACE_WORDS = 5

_p = C.c_void_p


class MediumDesc(C.Structure):
    _fields_ = [("n_media", C.c_int32), ("axis", _p), ("layer_off", _p), ("layer_cnt", _p), ("edges", _p),
                ("lam_s", _p), ("lam_a", _p), ("g", _p), ("f_sl", _p)]


class Targets(C.Structure):
    _fields_ = [("n_targets", C.c_int32), ("medium", _p), ("src", _p), ("sensor", _p), ("radius", _p),
                ("emit_kind", _p), ("emit_dir", _p), ("emit_param", _p), ("det_kind", _p), ("det_dir", _p),
                ("n0", _p), ("logw", _p)]


class Chains(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("cap", C.c_int32), ("precision", C.c_int32), ("target", _p), ("n", _p),
                ("verts", _p), ("logp", _p), ("status", _p), ("stats", _p), ("work", _p)]


class RunParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("step0", C.c_uint64), ("burn_in", C.c_int64), ("steps", C.c_int32),
                ("cycle_len", C.c_int32), ("n_perturb", C.c_int32), ("birth_thresh", C.c_uint32),
                ("sigma", C.c_double), ("kappa_end", C.c_double), ("sampler", C.c_int32), ("mala_h", C.c_double),
                ("block_chains", C.c_int32), ("v_lds", C.c_int32), ("chunk", C.c_int32), ("trace", _p),
                ("hist", _p), ("step_counter", _p)]


class Proposal(C.Structure):
    _fields_ = [("sigma", C.c_double), ("kappa_end", C.c_double), ("mala_h", C.c_double), ("cycle_len", C.c_int32),
                ("n_perturb", C.c_int32)]


EXPORTS = ["rjpath_last_error", "rjpath_version", "rjpath_init_medium", "rjpath_free_medium", "rjpath_run_chains",
           "rjpath_anchor", "rjpath_intensity", "rjpath_grad", "rjpath_autotune", "rjpath_tune_tilt", "rjpath_dlogi_dtheta",
           "rjpath_intensity_noalloc", "rjpath_yield_accumulate", "rjpath_yield", "rjpath_length_hist",
           "rjpath_tune_proposal", "rjpath_score_length", "rjpath_dlength_dtheta"]

_lib = None


class RJPathError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rjpath error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Loads librjpath.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1811_04156_amd/build.py (no CPU fallback)")
    L = C.CDLL(path)
    L.rjpath_last_error.restype = C.c_char_p
    L.rjpath_version.restype = C.c_char_p
    L.rjpath_init_medium.argtypes = [C.POINTER(_p), C.POINTER(MediumDesc), _p]
    L.rjpath_free_medium.argtypes = [_p]
    L.rjpath_run_chains.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), C.POINTER(RunParams), _p]
    L.rjpath_anchor.argtypes = [_p, C.POINTER(Targets), _p, _p]
    L.rjpath_intensity.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), C.c_int32, _p, _p, _p, _p, _p, _p]
    L.rjpath_grad.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), _p, _p, _p, _p]
    L.rjpath_autotune.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), C.POINTER(RunParams), C.c_int32,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32), _p]
    L.rjpath_tune_tilt.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), C.POINTER(RunParams), C.c_int32, _p,
                                   C.c_double, C.c_double, _p]
    L.rjpath_dlogi_dtheta.argtypes = [_p, C.POINTER(Targets), _p, _p, _p]
    L.rjpath_intensity_noalloc.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), C.c_int32, _p, _p, _p, _p, _p,
                                           _p]
    L.rjpath_yield_accumulate.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), C.c_int32, _p, _p, C.c_int32,
                                          _p, _p, _p]
    L.rjpath_yield.argtypes = [C.c_int32, C.c_int32, _p, _p, _p, _p]
    L.rjpath_length_hist.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), C.c_int32, C.c_double, C.c_double,
                                     _p, _p]
    L.rjpath_tune_proposal.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), C.POINTER(RunParams), C.c_int32,
                                       C.POINTER(Proposal), C.c_int32, C.c_int32, _p, C.POINTER(C.c_int32), _p]
    L.rjpath_score_length.argtypes = [_p, C.POINTER(Targets), C.POINTER(Chains), _p, _p]
    L.rjpath_dlength_dtheta.argtypes = [_p, C.POINTER(Targets), _p, _p, _p, _p, _p]
    for f in EXPORTS[2:]:
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _check(code, allow=()):
    if code != RJPATH_OK and code not in allow:
        raise RJPathError(code, load().rjpath_last_error().decode())
    return code


def _np_ptr(a):
    return a.ctypes.data_as(_p) if a is not None else None


def _tp(t):
    return _p(t.data_ptr()) if t is not None else None


def birth_thresh(frac):
    return int(min(max(round(frac * 2.0**32), 1), 2**32 - 1))


class Medium:
    """Owns an rjpath_medium handle built from a workload's media arrays."""

    def __init__(self, w, stream=None):
        L = load()
        self._arr = [np.ascontiguousarray(w[k], dtype=np.float64) for k in ("m_axis",)] + \
            [np.ascontiguousarray(w[k], dtype=np.int32) for k in ("m_layer_off", "m_layer_cnt")] + \
            [np.ascontiguousarray(w[k], dtype=np.float64) for k in ("edges", "lam_s", "lam_a", "g", "f_sl")]
        a = self._arr
        d = MediumDesc(len(w["m_layer_cnt"]), *[_np_ptr(x) for x in a])
        h = _p()
        _check(L.rjpath_init_medium(C.byref(h), C.byref(d), stream))
        self.h = h
        self.L_total = int(np.sum(w["m_layer_cnt"]))

    def close(self):
        if getattr(self, "h", None):
            load().rjpath_free_medium(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sampler:
    """Device state of one batched run: targets, chains, statistics.

    All tensors live on ``device``; the launch, the statistics and the
    estimators run in librjpath's kernels."""

    def __init__(self, w, device="cuda", precision=None, logw=None, chains=None, stream=None, medium=None):
        load()
        self.w = w
        self.dev = torch.device(device)
        prec = precision or w.get("precision", "f32")
        self.prec = F64 if prec in ("f64", F64) else F32
        self.rdt = torch.float64 if self.prec == F64 else torch.float32
        self.cap = int(w["cap"])
        self.stream = stream
        self.medium = medium or Medium(w, self._stream_ptr())
        d = self.dev
        f64 = lambda k: torch.as_tensor(np.ascontiguousarray(w[k], np.float64), device=d)
        i32 = lambda k: torch.as_tensor(np.ascontiguousarray(w[k], np.int32), device=d)
        self.t = dict(medium=i32("t_medium"), src=f64("t_src"), sensor=f64("t_sensor"), radius=f64("t_radius"),
                      emit_kind=i32("t_emit_kind"), emit_dir=f64("t_emit_dir"), emit_param=f64("t_emit_param"),
                      det_kind=i32("t_det_kind"), det_dir=f64("t_det_dir"), n0=i32("t_n0"))
        self.T = len(w["t_src"])
        self.logw = None
        if logw is not None:
            self.set_logw(logw)
        tgt = np.asarray(w["c_target"] if chains is None else w["c_target"][:chains], np.int32)
        self.C = len(tgt)
        self.target = torch.as_tensor(tgt, device=d)
        self.n = torch.as_tensor(np.asarray(w["t_init_n"])[tgt].astype(np.int32), device=d)
        self.verts = torch.zeros((self.cap, self.C, 4), dtype=self.rdt, device=d)
        init = torch.as_tensor(np.asarray(w["t_init"]), dtype=self.rdt, device=d)  # (T, 3, 3)
        self.verts[:3, :, :3] = init[self.target.long()].permute(1, 0, 2)
        self.logp = torch.zeros(self.C, dtype=torch.float64, device=d)
        self.status = torch.zeros(self.C, dtype=torch.int32, device=d)
        self.stats = torch.zeros((self.C, NSTAT), dtype=torch.float64, device=d)
        self.work = None
        self.step = 0

    def _stream_ptr(self):
        if self.stream is not None:
            return _p(self.stream.cuda_stream)
        if torch.cuda.is_available():
            return _p(torch.cuda.current_stream().cuda_stream)
        return None

    def set_logw(self, logw):
        lw = torch.as_tensor(np.ascontiguousarray(logw, np.float64), device=self.dev).reshape(self.T, self.cap + 1)
        self.logw = lw.contiguous()

    def set_state(self, n, verts_xyz):
        """n (C,), verts (C, k, 3) with k <= cap (relative to each source)."""
        n = torch.as_tensor(np.asarray(n, np.int32), device=self.dev)
        v = torch.as_tensor(np.asarray(verts_xyz), dtype=self.rdt, device=self.dev)
        self.n.copy_(n)
        self.verts.zero_()
        self.verts[: v.shape[1], :, :3] = v.permute(1, 0, 2)

    def get_state(self):
        n = self.n.cpu().numpy()
        v = self.verts[..., :3].permute(1, 0, 2).cpu().numpy().astype(np.float64)
        return n, v

    # -- C structs ----------------------------------------------------------
    def _targets(self):
        t = self.t
        return Targets(self.T, _tp(t["medium"]), _tp(t["src"]), _tp(t["sensor"]), _tp(t["radius"]),
                       _tp(t["emit_kind"]), _tp(t["emit_dir"]), _tp(t["emit_param"]), _tp(t["det_kind"]),
                       _tp(t["det_dir"]), _tp(t["n0"]), _tp(self.logw))

    def _chains(self):
        return Chains(self.C, self.cap, self.prec, _tp(self.target), _tp(self.n), _tp(self.verts), _tp(self.logp),
                      _tp(self.status), _tp(self.stats), _tp(self.work))

    def _params(self, steps, run=None, trace=None, hist=None, block=0, v_lds=0, chunk=0, step0=None, counter=None):
        r = dict(self.w)
        r.update(run or {})
        if int(r.get("sampler", 0)) in (MALA, TREE) and self.work is None:
            self.work = torch.zeros_like(self.verts)
        return RunParams(int(r["seed"]), int(self.step if step0 is None else step0), int(r["burn_in"]), int(steps),
                         int(r["cycle_len"]), int(r["n_perturb"]), birth_thresh(r["birth_frac"]), float(r["sigma"]),
                         float(r["kappa_end"]), int(r.get("sampler", 0)), float(r.get("mala_h", 0.05)), int(block),
                         int(v_lds), int(chunk), _tp(trace), _tp(hist), _tp(counter))

    def _capture(self, fn):
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                fn(_p(side.cuda_stream))
        torch.cuda.current_stream().wait_stream(side)
        return g

    def capture_run(self, steps, run=None, block=0, v_lds=0):
        """Captures `steps` sampler steps of every chain in a CUDA/HIP graph
        whose every replay advances the chains by `steps` steps (the step
        index lives in a device counter).  Replay with replay_run()."""
        self.counter = torch.tensor([self.step], dtype=torch.int64, device=self.dev)
        p = self._params(steps, run, None, None, block, v_lds, 0, counter=self.counter)
        tg, ch = self._targets(), self._chains()

        def body(sp):
            _check(load().rjpath_run_chains(self.medium.h, C.byref(tg), C.byref(ch), C.byref(p), sp))

        g = self._capture(body)
        self._graph_steps = steps
        return g

    def capture_stats(self, score=True, intensity=True, groups=16):
        """Captures the per-chunk statistics of the hot path in a graph: the
        score pass adding into self.score_acc (rjpath_grad) and the intensity
        estimator into device tensors (rjpath_intensity_noalloc, with the
        anchors computed once beforehand).  Returns the dict of output tensors
        (I, se, ess, rhat) that every replay rewrites."""
        self.score_acc = torch.zeros((self.T, 1 + 3 * self.medium.L_total), dtype=torch.float64, device=self.dev)
        anc = torch.as_tensor(self.anchor(), dtype=torch.float64, device=self.dev)
        out = {k: torch.empty(self.T, dtype=torch.float64, device=self.dev) for k in ("I", "se", "ess", "rhat")}
        tg, ch = self._targets(), self._chains()

        def body(sp):
            if score:
                _check(load().rjpath_grad(self.medium.h, C.byref(tg), C.byref(ch), None, None, _tp(self.score_acc),
                                          sp))
            if intensity:
                _check(load().rjpath_intensity_noalloc(self.medium.h, C.byref(tg), C.byref(ch), int(groups), _tp(anc),
                                                       _tp(out["I"]), _tp(out["se"]), _tp(out["ess"]),
                                                       _tp(out["rhat"]), sp))

        self._keep_graph_args = (tg, ch, anc)
        return self._capture(body), out

    def capture(self, steps, run=None, score=True, block=0, v_lds=0):
        """Captures one chunk of the hot path (`steps` sampler steps, then the
        score pass) in one graph whose every replay advances the chains by
        `steps` steps.  Returns (graph, score tensor accumulated by each replay)."""
        self.counter = torch.tensor([self.step], dtype=torch.int64, device=self.dev)
        self.score_acc = torch.zeros((self.T, 1 + 3 * self.medium.L_total), dtype=torch.float64, device=self.dev)
        p = self._params(steps, run, None, None, block, v_lds, 0, counter=self.counter)
        tg, ch = self._targets(), self._chains()

        def body(sp):
            _check(load().rjpath_run_chains(self.medium.h, C.byref(tg), C.byref(ch), C.byref(p), sp))
            if score:
                _check(load().rjpath_grad(self.medium.h, C.byref(tg), C.byref(ch), None, None, _tp(self.score_acc),
                                          sp))

        g = self._capture(body)
        self._graph_steps = steps
        return g, self.score_acc

    def replay(self, g, times=1):
        """Replays a graph from capture() / capture_run() (advancing the step index)."""
        for _ in range(times):
            g.replay()
        self.step += times * self._graph_steps

    # -- calls --------------------------------------------------------------
    def run(self, steps, run=None, trace=False, hist=False, block=0, v_lds=0, chunk=0):
        """Advances all chains by ``steps`` steps; returns the trace tensor
        (C, steps, 5) and/or the sector histogram (T, cap+1) when asked."""
        tr = torch.zeros((self.C, steps, TRACE_WORDS), dtype=torch.float64, device=self.dev) if trace else None
        hs = torch.zeros((self.T, self.cap + 1), dtype=torch.int32, device=self.dev) if hist else None
        p = self._params(steps, run, tr, hs, block, v_lds, chunk)
        tg, ch = self._targets(), self._chains()
        _check(load().rjpath_run_chains(self.medium.h, C.byref(tg), C.byref(ch), C.byref(p), self._stream_ptr()))
        self.step += steps
        return tr, hs

    def autotune(self, steps, run=None):
        p = self._params(steps, run)
        tg, ch = self._targets(), self._chains()
        b, v = C.c_int32(), C.c_int32()
        _check(load().rjpath_autotune(self.medium.h, C.byref(tg), C.byref(ch), C.byref(p), int(steps), C.byref(b),
                                      C.byref(v), self._stream_ptr()))
        self.step += steps
        return b.value, v.value

    def tune_proposal(self, candidates, trial_steps, groups=16, run=None):
        """rjpath_tune_proposal over candidate dicts with keys sigma,
        kappa_end, mala_h, cycle_len, n_perturb (missing keys: the workload's
        values).  Returns (best index, scores); the chains advance by
        2 * len(candidates) * trial_steps steps."""
        r = dict(self.w)
        r.update(run or {})
        arr = (Proposal * len(candidates))()
        for i, c in enumerate(candidates):
            arr[i] = Proposal(float(c.get("sigma", r["sigma"])), float(c.get("kappa_end", r["kappa_end"])),
                              float(c.get("mala_h", r.get("mala_h", 0.05))), int(c.get("cycle_len", r["cycle_len"])),
                              int(c.get("n_perturb", r["n_perturb"])))
        p = self._params(trial_steps, run)
        tg, ch = self._targets(), self._chains()
        sc = np.zeros(len(candidates))
        b = C.c_int32()
        _check(load().rjpath_tune_proposal(self.medium.h, C.byref(tg), C.byref(ch), C.byref(p), len(candidates), arr,
                                           int(trial_steps), int(groups), _np_ptr(sc), C.byref(b),
                                           self._stream_ptr()))
        self.step += 2 * len(candidates) * trial_steps
        return b.value, sc

    def tune_tilt(self, rounds=4, steps=400, max_logw=40.0, floor_push=3.0, run=None):
        """Sector-tilt tuning in librjpath (rjpath_tune_tilt): `rounds` pilot
        rounds of `steps` steps, the tilt table updated on the device after
        each; the chains advance, their statistics are left untouched."""
        if self.logw is None:
            self.logw = torch.zeros((self.T, self.cap + 1), dtype=torch.float64, device=self.dev)
        hist = torch.zeros((self.T, self.cap + 1), dtype=torch.int32, device=self.dev)
        p = self._params(steps, run)
        tg, ch = self._targets(), self._chains()
        _check(load().rjpath_tune_tilt(self.medium.h, C.byref(tg), C.byref(ch), C.byref(p), int(rounds), _tp(hist),
                                       float(max_logw), float(floor_push), self._stream_ptr()))
        self.step += rounds * steps
        return self.logw, hist

    def dlogI(self, score):
        """d log I / d theta (T, L_total, 3) on the device from accumulated
        score sums (rjpath_dlogi_dtheta)."""
        out = torch.empty((self.T, 3 * self.medium.L_total), dtype=torch.float64, device=self.dev)
        tg = self._targets()
        _check(load().rjpath_dlogi_dtheta(self.medium.h, C.byref(tg), _tp(score), _tp(out), self._stream_ptr()))
        return out.reshape(self.T, self.medium.L_total, 3)

    def anchor(self, refresh=False):
        """Anchor-sector integrals (T,), computed once and cached."""
        if refresh or getattr(self, "_anchor", None) is None:
            a = np.zeros(self.T)
            tg = self._targets()
            _check(load().rjpath_anchor(self.medium.h, C.byref(tg), _np_ptr(a), self._stream_ptr()))
            self._anchor = a
        return self._anchor

    def intensity(self, groups=16):
        T = self.T
        an = self.anchor()
        I, se, ess, rh = (np.zeros(T) for _ in range(4))
        tg, ch = self._targets(), self._chains()
        code = load().rjpath_intensity(self.medium.h, C.byref(tg), C.byref(ch), int(groups), _np_ptr(an),
                                       _np_ptr(I), _np_ptr(se), _np_ptr(ess), _np_ptr(rh), self._stream_ptr())
        _check(code, allow=(RJPATH_ENODATA,))
        return dict(I=I, se=se, ess=ess, rhat=rh, anchor=an, code=code)

    def intensity_noalloc(self, groups=16, anchor=None):
        """rjpath_intensity_noalloc: the estimator with every buffer in the
        library's static device array; returns device tensors (I, se, ess,
        rhat).  anchor: None (computed on the device) or a (T,) device tensor."""
        out = [torch.empty(self.T, dtype=torch.float64, device=self.dev) for _ in range(4)]
        tg, ch = self._targets(), self._chains()
        _check(load().rjpath_intensity_noalloc(self.medium.h, C.byref(tg), C.byref(ch), int(groups), _tp(anchor),
                                               *[_tp(x) for x in out], self._stream_ptr()))
        return dict(zip(("I", "se", "ess", "rhat"), out))

    def grad(self, logp=True, dv=False, score=False):
        """log p (C,), d log p / d vertices (layout of verts) and the score
        sums (T, 1 + 3 L_total); `score` may be an existing device tensor of
        that shape, which the call adds to."""
        lp = torch.full((self.C,), float("nan"), dtype=torch.float64, device=self.dev) if logp else None
        g = torch.zeros_like(self.verts) if dv else None
        if isinstance(score, torch.Tensor):
            sc = score
        else:
            sc = torch.zeros((self.T, 1 + 3 * self.medium.L_total), dtype=torch.float64, device=self.dev) \
                if score else None
        tg, ch = self._targets(), self._chains()
        _check(load().rjpath_grad(self.medium.h, C.byref(tg), C.byref(ch), _tp(lp), _tp(g), _tp(sc),
                                  self._stream_ptr()))
        return lp, g, sc

    # -- snapshot estimators --------------------------------------------------
    def yield_pairs(self, pairs):
        """Device tables of rjpath_yield_accumulate for a list of (t0, t1)
        sensor pairs: (pairs (2P,), role (T,), P)."""
        pr = np.asarray(pairs, np.int32).reshape(-1, 2)
        role = np.full(self.T, -1, np.int32)
        for k, (a, b) in enumerate(pr):
            if role[a] >= 0 or role[b] >= 0 or a == b:
                raise ValueError("each target may belong to one pair only")
            role[a], role[b] = 2 * k, 2 * k + 1
        return (torch.as_tensor(pr.reshape(-1), device=self.dev), torch.as_tensor(role, device=self.dev), len(pr))

    def yield_accumulate(self, tables, acc=None, groups=16, logr=False):
        """Adds one bridge sample per chain (rjpath_yield_accumulate); returns
        (acc, per-chain log r or None)."""
        pr, role, P = tables
        if acc is None:
            acc = torch.zeros((P, 2, groups, 2), dtype=torch.float64, device=self.dev)
        lr = torch.empty(self.C, dtype=torch.float64, device=self.dev) if logr else None
        tg, ch = self._targets(), self._chains()
        _check(load().rjpath_yield_accumulate(self.medium.h, C.byref(tg), C.byref(ch), int(P), _tp(pr), _tp(role),
                                              int(groups), _tp(acc), _tp(lr), self._stream_ptr()))
        return acc, lr

    def light_yield(self, acc):
        """B = I_1 / I_0 and its standard error per pair (rjpath_yield)."""
        P, _, groups, _ = acc.shape
        B, se = np.zeros(P), np.zeros(P)
        code = load().rjpath_yield(int(P), int(groups), _tp(acc), _np_ptr(B), _np_ptr(se), self._stream_ptr())
        _check(code, allow=(RJPATH_ENODATA,))
        return B, se

    def length_hist(self, bins, l0, width, hist=None):
        """Adds the current paths' lengths into per-target histograms
        (rjpath_length_hist); returns the (T, bins + 1) tensor, whose last
        column is the normaliser."""
        if hist is None:
            hist = torch.zeros((self.T, bins + 1), dtype=torch.float64, device=self.dev)
        tg, ch = self._targets(), self._chains()
        _check(load().rjpath_length_hist(self.medium.h, C.byref(tg), C.byref(ch), int(bins), float(l0), float(width),
                                         _tp(hist), self._stream_ptr()))
        return hist

    def score_length(self, score_L=None):
        """Adds the length-weighted score sums of the current paths
        (rjpath_score_length) into score_L (T, 1 + 3 L_total)."""
        if score_L is None:
            score_L = torch.zeros((self.T, 1 + 3 * self.medium.L_total), dtype=torch.float64, device=self.dev)
        tg, ch = self._targets(), self._chains()
        _check(load().rjpath_score_length(self.medium.h, C.byref(tg), C.byref(ch), _tp(score_L), self._stream_ptr()))
        return score_L

    def dlength(self, score, score_L):
        """Mean path length (T,) and its gradient (T, L_total, 3) from the two
        score sums (rjpath_dlength_dtheta)."""
        m = torch.empty(self.T, dtype=torch.float64, device=self.dev)
        dm = torch.empty((self.T, 3 * self.medium.L_total), dtype=torch.float64, device=self.dev)
        tg = self._targets()
        _check(load().rjpath_dlength_dtheta(self.medium.h, C.byref(tg), _tp(score), _tp(score_L), _tp(m), _tp(dm),
                                            self._stream_ptr()))
        return m, dm.reshape(self.T, self.medium.L_total, 3)
