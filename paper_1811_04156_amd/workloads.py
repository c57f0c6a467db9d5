"""Seeded synthetic inputs for the photon-path sampler.

This module only draws geometry and medium parameters (numpy ``default_rng``)
and lays them out as plain arrays.  It holds none of the method's arithmetic:
no densities, attenuation, proposals or estimators.  Both the FP64 oracle and
the HIP path read the same arrays produced here.

Array conventions (all float64 unless noted):

media (M media, L layers in total)
    m_axis      (M, 3)   unit layer axis of each medium
    m_layer_off (M,)     int32, index of the medium's first layer
    m_layer_cnt (M,)     int32, number of layers of the medium
    edges       (L + M,) layer edges along the axis; medium m owns
                         edges[m_layer_off[m] + m : ... + m_layer_cnt[m] + 1];
                         the first and last layer extend to -inf / +inf
    lam_s, lam_a, g, f_sl (L,)  scattering length, absorption length (m),
                         mean scattering cosine, simplified-Liu fraction
targets (T targets; one target = one source/sensor pair)
    t_medium (T,) int32; t_src (T, 3) absolute source position;
    t_sensor (T, 3) absolute sensor centre; t_radius (T,);
    t_emit_kind (T,) int32: 0 isotropic, 1 von Mises-Fisher, 2 uniform cone;
    t_emit_dir (T, 3); t_emit_param (T,): kappa (vMF) or half-angle in rad (cone);
    t_det_kind (T,) int32: 0 uniform detection, 1 the paper's angular response;
    t_det_dir (T, 3)
    t_init_n (T,) int32 and t_init (T, 3, 3): a starting path with at most
    three vertices, relative to the source (vertex 0 is the source itself).
    t_n0 (T,) int32: anchor sector, 2 when every direction from the source
    into the sensor lies inside the emission support, else 3.
chains
    c_target (C,) int32

The workloads follow the paper's synthetic setting (Sec. "Implementation":
point source, spherical sensors of 0.15-0.165 m, homogeneous or layered
scattering/absorbing bulk, Henyey-Greenstein scattering).
"""
from __future__ import annotations

import numpy as np

EMIT_ISO, EMIT_VMF, EMIT_CONE = 0, 1, 2
DET_UNIFORM, DET_PAPER = 0, 1

DEFAULT_RUN = dict(seed=0, steps=10_000, burn_in=1_000, cycle_len=5, n_perturb=3,
                   birth_frac=0.5, sigma=1.0, kappa_end=20.0, sampler=0, mala_h=0.05)


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _rand_dirs(rng, k):
    v = rng.normal(size=(k, 3))
    return _unit(v)


def _straight_start(src, sensor, radius):
    """Two-vertex starting path: source -> sensor point facing the source."""
    d = sensor - src
    dist = np.linalg.norm(d, axis=-1, keepdims=True)
    end = d - radius[:, None] * d / dist
    init = np.zeros((len(src), 3, 3))
    init[:, 1] = end
    return np.full(len(src), 2, np.int32), init


def _cone_start(src, sensor, radius, axis, half_angle):
    """Starting path for cone sources (paper: seed from one traced path).

    If the sensor centre is inside the emission cone the straight path is
    used; otherwise one scattering vertex is placed on the cone axis at half
    the source-sensor distance and the end point is the sensor point facing
    that vertex.
    """
    n, init = _straight_start(src, sensor, radius)
    d = sensor - src
    dist = np.linalg.norm(d, axis=-1)
    inside = np.einsum("ij,ij->i", d / dist[:, None], axis) > np.cos(half_angle)
    v1 = axis * (0.5 * dist)[:, None]
    to = d - v1
    tl = np.linalg.norm(to, axis=-1, keepdims=True)
    end = v1 + to - radius[:, None] * to / tl
    for i in np.nonzero(~inside)[0]:
        n[i] = 3
        init[i, 1] = v1[i]
        init[i, 2] = end[i]
    return n, init


def _homog_media(lam_s, lam_a, g):
    M = len(lam_s)
    return dict(
        m_axis=np.tile([0.0, 0.0, 1.0], (M, 1)),
        m_layer_off=np.arange(M, dtype=np.int32),
        m_layer_cnt=np.ones(M, np.int32),
        edges=np.tile([0.0, 1.0], M).astype(np.float64),
        lam_s=np.asarray(lam_s, np.float64), lam_a=np.asarray(lam_a, np.float64),
        g=np.asarray(g, np.float64), f_sl=np.zeros(M),
    )


def _layered_medium(lam_s, lam_a, g, z0, dz):
    L = len(lam_s)
    return dict(
        m_axis=np.array([[0.0, 0.0, 1.0]]),
        m_layer_off=np.array([0], np.int32),
        m_layer_cnt=np.array([L], np.int32),
        edges=z0 + dz * np.arange(L + 1, dtype=np.float64),
        lam_s=np.asarray(lam_s, np.float64), lam_a=np.asarray(lam_a, np.float64),
        g=np.asarray(g, np.float64), f_sl=np.zeros(L),
    )


def _targets(medium, src, sensor, radius, emit_kind, emit_dir, emit_param,
             init_n, init, det_kind=None, det_dir=None):
    T = len(src)
    src_a, sen_a = np.asarray(src, np.float64), np.asarray(sensor, np.float64)
    d = sen_a - src_a
    dist = np.linalg.norm(d, axis=-1)
    n0 = np.full(T, 2, np.int32)
    for i in range(T):
        if int(emit_kind[i]) == EMIT_CONE:
            ang = np.arccos(np.clip(np.dot(d[i] / dist[i], emit_dir[i]), -1, 1))
            if ang + np.arcsin(min(1.0, radius[i] / dist[i])) > emit_param[i]:
                n0[i] = 3
    return dict(t_n0=n0,
        t_medium=np.asarray(medium, np.int32),
        t_src=np.asarray(src, np.float64), t_sensor=np.asarray(sensor, np.float64),
        t_radius=np.asarray(radius, np.float64),
        t_emit_kind=np.asarray(emit_kind, np.int32),
        t_emit_dir=np.asarray(emit_dir, np.float64),
        t_emit_param=np.asarray(emit_param, np.float64),
        t_det_kind=np.zeros(T, np.int32) if det_kind is None else np.asarray(det_kind, np.int32),
        t_det_dir=np.tile([0.0, -1.0, 0.0], (T, 1)) if det_dir is None else np.asarray(det_dir, np.float64),
        t_init_n=np.asarray(init_n, np.int32), t_init=np.asarray(init, np.float64),
    )


def single_target(distance=10.0, radius=0.165, lam_s=25.0, lam_a=100.0, g=0.9,
                  chains=64, cap=64, direction=(0.0, 0.0, 1.0), emit_kind=EMIT_ISO,
                  emit_param=0.0, emit_dir=(0.0, 0.0, 1.0), det_kind=DET_UNIFORM,
                  det_dir=(0.0, -1.0, 0.0), f_sl=0.0, **run):
    """One source/sensor pair in an infinite homogeneous medium."""
    media = _homog_media([lam_s], [lam_a], [g])
    media["f_sl"] = np.array([f_sl], np.float64)
    src = np.zeros((1, 3))
    sensor = np.asarray(direction, np.float64)[None] / np.linalg.norm(direction) * distance
    r = np.array([radius])
    n, init = _straight_start(src, sensor, r)
    tg = _targets([0], src, sensor, r, [emit_kind], [emit_dir], [emit_param], n, init,
                  [det_kind], [det_dir])
    w = dict(name="single", cap=int(cap), **media, **tg,
             c_target=np.zeros(chains, np.int32))
    w.update(DEFAULT_RUN)
    w.update(run)
    return w


def reference_target(**over):
    """Plain RJMCMC, FP64: isotropic point source, homogeneous medium
    (scattering length 25 m, absorption length 100 m, g = 0.9), one sensor of
    radius 0.165 m at 10 m, 64 chains x 1e4 steps, cap 64, mix 60/20/20,
    sigma = 1 m, Philox seed 0."""
    w = single_target(10.0, 0.165, 25.0, 100.0, 0.9, chains=64, cap=64, seed=0)
    w["name"] = "reference_target"
    w["precision"] = "f64"
    w.update(over)
    return w


def homogeneous_groups(seed=1, groups=256, per_group=256, steps=10_000, cap=256, **over):
    """Batched plain RJMCMC, FP32 evaluation: 256 chain-groups of 256 chains;
    per group a homogeneous medium (scattering length log-U[10,50] m,
    absorption length log-U[50,200] m, g ~ U[0.8,0.95]) and a sensor of
    radius 0.165 m at a distance ~ U[5,100] m in a uniform direction."""
    rng = np.random.default_rng(seed)
    lam_s = np.exp(rng.uniform(np.log(10.0), np.log(50.0), groups))
    lam_a = np.exp(rng.uniform(np.log(50.0), np.log(200.0), groups))
    g = rng.uniform(0.8, 0.95, groups)
    dist = rng.uniform(5.0, 100.0, groups)
    dirs = _rand_dirs(rng, groups)
    media = _homog_media(lam_s, lam_a, g)
    src = np.zeros((groups, 3))
    sensor = dirs * dist[:, None]
    r = np.full(groups, 0.165)
    n, init = _straight_start(src, sensor, r)
    tg = _targets(np.arange(groups), src, sensor, r, np.zeros(groups, np.int32), np.tile([0, 0, 1.0], (groups, 1)),
                  np.zeros(groups), n, init)
    w = dict(name="homogeneous_groups", cap=int(cap), **media, **tg,
             c_target=np.repeat(np.arange(groups, dtype=np.int32), per_group))
    w.update(DEFAULT_RUN)
    w.update(seed=seed, steps=steps, burn_in=steps // 10, precision="f32")
    w.update(over)
    return w


def layered_pairs(seed=3, pairs=1000, chains=1 << 20, cap=512, steps=10_000,
                  n_layers=100, dz=10.0, half_angle_deg=20.0, dmin=10.0, dmax=150.0,
                  emit_kind=EMIT_CONE, **over):
    """Layered medium with ragged source/sensor pairs: n_layers horizontal
    layers of dz metres (scattering length log-U[10,60] m, absorption length
    log-U[40,250] m, g = 0.9); each pair has a cone source (20 deg half-angle,
    horizontal axis, uniform azimuth) at a uniform depth and a sensor at a
    distance ~ U[dmin,dmax] in a uniform direction, kept inside the stack.
    Chains are assigned to pairs in contiguous runs: chain c belongs to pair
    floor(c * pairs / chains) (1048 or 1049 chains per pair at 2^20 chains),
    so a block of chains covers one or two targets."""
    rng = np.random.default_rng(seed)
    lam_s = np.exp(rng.uniform(np.log(10.0), np.log(60.0), n_layers))
    lam_a = np.exp(rng.uniform(np.log(40.0), np.log(250.0), n_layers))
    g = np.full(n_layers, 0.9)
    top = n_layers * dz
    media = _layered_medium(lam_s, lam_a, g, 0.0, dz)
    src = np.zeros((pairs, 3))
    sensor = np.zeros((pairs, 3))
    axis = np.zeros((pairs, 3))
    for i in range(pairs):
        src[i, 2] = rng.uniform(0.0, top)
        az = rng.uniform(0.0, 2 * np.pi)
        axis[i] = [np.cos(az), np.sin(az), 0.0]
        while True:
            d = _rand_dirs(rng, 1)[0] * rng.uniform(dmin, dmax)
            if 0.0 <= src[i, 2] + d[2] <= top:
                break
        sensor[i] = src[i] + d
    r = np.full(pairs, 0.165)
    half = np.deg2rad(half_angle_deg)
    if emit_kind == EMIT_CONE:
        n, init = _cone_start(src, sensor, r, axis, np.full(pairs, half))
        param = np.full(pairs, half)
    else:
        n, init = _straight_start(src, sensor, r)
        param = np.zeros(pairs)
    tg = _targets(np.zeros(pairs), src, sensor, r, np.full(pairs, emit_kind), axis,
                  param, n, init)
    w = dict(name="layered", cap=int(cap), **media, **tg,
             c_target=(np.arange(chains, dtype=np.int64) * pairs // chains).astype(np.int32))
    w.update(DEFAULT_RUN)
    w.update(seed=seed, steps=steps, burn_in=steps // 10, precision="f32")
    w.update(over)
    return w


def layered_batch(**over):
    """Layered medium, ragged batch: 100 layers of 10 m, 1000 cone-source
    pairs at 10-150 m, 2^20 chains, cap 512."""
    w = layered_pairs(seed=3, pairs=1000, chains=1 << 20, cap=512)
    w["name"] = "layered_batch"
    w.update(over)
    return w


def layered_batch_langevin(**over):
    """The layered batch's medium and geometry with 262,144 chains and the
    gradient-informed (MALA) sampler."""
    w = layered_pairs(seed=3, pairs=1000, chains=262_144, cap=512)
    w.update(name="layered_batch_langevin", sampler=1)
    w.update(over)
    return w


def two_region(b1=0.3, b0=0.3, a=0.01, scale=1.0, radius=0.15, chains_per_sensor=64, cap=512, kappa=38.0,
               steps=10_000, seed=11):
    """The paper's synthetic test (Sec. "Implementation", Fig. setup): the
    bulk split by the y-z plane into a region x < 0 with scattering b0 and a
    region x >= 0 with scattering b1 (absorption a everywhere; m^-1), the
    simplified-Liu / Henyey-Greenstein mixture with mean cosine 0.95 and
    f_SL = 0.45, a von Mises-Fisher source (kappa = 38 along z) at the origin,
    and two sensors of radius 0.15 m at (0, 0, 120) and (60, 7, 104) m with the
    paper's angular response about (0, -1, 0).  `radius` may also give the two
    radii.  `scale` multiplies the sensor positions only (0.05 gives a variant short enough for the analog tracer).
    Target 0 is sensor 0, target 1 sensor 1; chains in two contiguous runs."""
    media = dict(m_axis=np.array([[1.0, 0.0, 0.0]]), m_layer_off=np.array([0], np.int32),
                 m_layer_cnt=np.array([2], np.int32), edges=np.array([-1.0, 0.0, 1.0]),
                 lam_s=np.array([1.0 / b0, 1.0 / b1]), lam_a=np.array([1.0 / a, 1.0 / a]),
                 g=np.array([0.95, 0.95]), f_sl=np.array([0.45, 0.45]))
    src = np.zeros((2, 3))
    sen = np.array([[0.0, 0.0, 120.0], [60.0, 7.0, 104.0]]) * scale
    r = np.broadcast_to(np.asarray(radius, np.float64), (2,)).copy()
    n, init = _straight_start(src, sen, r)
    tg = _targets(np.zeros(2), src, sen, r, np.full(2, EMIT_VMF), np.tile([0.0, 0.0, 1.0], (2, 1)),
                  np.full(2, kappa), n, init, np.full(2, DET_PAPER), np.tile([0.0, -1.0, 0.0], (2, 1)))
    w = dict(name="two_region", cap=int(cap), **media, **tg,
             c_target=np.repeat(np.arange(2, dtype=np.int32), chains_per_sensor))
    w.update(DEFAULT_RUN)
    w.update(seed=seed, steps=steps, burn_in=steps // 10, precision="f32")
    return w


def array_strings(rows=2, per_row=5, spacing=125.0, sensors=60, dz=17.0, zc=500.0):
    """Horizontal (x, y) positions of vertical strings on a triangular lattice
    (rows offset by half a spacing) and the sensor depths along each string."""
    xy = np.array([[c * spacing + (r % 2) * spacing / 2, r * spacing * np.sqrt(3) / 2]
                   for r in range(rows) for c in range(per_row)])
    z = zc + dz * (np.arange(sensors) - (sensors - 1) / 2)
    return xy, z


def string_calibration(seed=5, n_sources=50, reach=200.0, chains_per_target=512, cap=512, steps=4000, n_layers=100,
            dz=10.0, sources=None, max_targets=None):
    """Calibration-shaped batch: 10 vertical strings (two rows of five, 125 m
    apart on a triangular lattice) of 60 sensors at 17 m spacing (radius
    0.165 m) in the 100-layer medium; isotropic flasher sources at the
    positions of n_sources sensors drawn with the seed; one target per other
    sensor within `reach` of a source; chains_per_target chains per target in
    contiguous runs.  The per-layer scattering and absorption lengths drawn
    here (as for the ragged layered batch) are the ground truth of the
    calibration fit.  `sources` (indices into the sensor list) and
    `max_targets` cut the batch down for tests."""
    rng = np.random.default_rng(seed)
    lam_s = np.exp(rng.uniform(np.log(10.0), np.log(60.0), n_layers))
    lam_a = np.exp(rng.uniform(np.log(40.0), np.log(250.0), n_layers))
    g = np.full(n_layers, 0.9)
    media = _layered_medium(lam_s, lam_a, g, 0.0, dz)
    xy, z = array_strings()
    pos = np.array([[x, y, zz] for x, y in xy for zz in z])  # (600, 3), string-major
    src_idx = np.sort(rng.choice(len(pos), n_sources, replace=False)) if sources is None else np.asarray(sources)
    src, sen = [], []
    for i in src_idx:
        d = np.linalg.norm(pos - pos[i], axis=1)
        for k in np.nonzero((d <= reach) & (d > 0))[0]:
            src.append(pos[i])
            sen.append(pos[k])
    src, sen = np.array(src), np.array(sen)
    if max_targets is not None:
        keep = np.argsort(np.linalg.norm(sen - src, axis=1), kind="stable")[:max_targets]
        src, sen = src[keep], sen[keep]
    T = len(src)
    r = np.full(T, 0.165)
    n, init = _straight_start(src, sen, r)
    tg = _targets(np.zeros(T), src, sen, r, np.zeros(T, np.int32), np.tile([0, 0, 1.0], (T, 1)), np.zeros(T),
                  n, init)
    w = dict(name="string_calibration", cap=int(cap), **media, **tg,
             c_target=np.repeat(np.arange(T, dtype=np.int32), chains_per_target), t_source_sensor=src_idx)
    w.update(DEFAULT_RUN)
    w.update(seed=seed, steps=steps, burn_in=steps // 10, precision="f32")
    return w


def subset_chains(w, chains):
    """Same workload with the chain list cut to the first ``chains`` entries."""
    w = dict(w)
    w["c_target"] = np.asarray(w["c_target"][:chains], np.int32)
    return w


def n_targets(w):
    return len(w["t_src"])
