// rj_api.hip -- the C ABI of librjpath: argument checks, the medium tables,
// launch selection and tuning, and the FP64 host finalisation of the
// intensity estimator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "rj_internal.h"
#include "rj_kernels.h"

using namespace rj;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(RJPATH_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, what);     \
    } while (0)

const double PI = 3.14159265358979323846;

// coth(k) - 1/k = g, solved by bisection in FP64.
double kappa_eq(double g) {
    if (g <= 0) return 0.0;
    double lo = 1e-9, hi = 1e6;
    for (int i = 0; i < 300; ++i) {
        double m = 0.5 * (lo + hi);
        double f = 1.0 / std::tanh(m) - 1.0 / m;
        (f < g ? lo : hi) = m;
    }
    return 0.5 * (lo + hi);
}

// n-point Gauss-Legendre rule mapped to [0, 1] (Newton iteration on P_n).
void gl01(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(PI * (i + 0.75) / (n + 0.5)), pp = 1;
        for (int it = 0; it < 200; ++it) {
            double p1 = 1, p2 = 0;
            for (int k = 1; k <= n; ++k) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * k - 1) * z * p2 - (k - 1.0) * p3) / k;
            }
            pp = n * (z * p1 - p2) / (z * z - 1);
            double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-15) break;
        }
        x[i] = 0.5 * (1 - z);
        w[i] = 1.0 / ((1 - z * z) * pp * pp);
    }
}

struct TuneKey {
    int cap, prec, sampler;
    bool operator<(const TuneKey& o) const { return std::tie(cap, prec, sampler) < std::tie(o.cap, o.prec, o.sampler); }
};

} // namespace

struct rjpath_medium {
    int n_media = 0, L_total = 0, n_edges = 0;
    bool layered = false; // some medium has more than one layer
    bool has_sl = false;  // some layer has f_SL > 0
    MedInfo* d_info = nullptr;
    double* d_edge = nullptr;
    double* d_pre = nullptr;
    float* d_lay32 = nullptr;
    double* d_lay64 = nullptr;
    double* d_gl = nullptr; // x (120) then w (120): rules of 8, 16, 32, 64 points
    // intensity workspace
    double* d_ws = nullptr;
    size_t ws_bytes = 0;
    std::map<TuneKey, std::pair<int, int>> tuned;
};

extern "C" {

const char* rjpath_last_error(void) { return g_err.c_str(); }

const char* rjpath_version(void) { return "rjpath 0.1 gfx950"; }

int rjpath_init_medium(rjpath_medium** out, const rjpath_medium_desc* d, void* stream) {
    if (!out || !d) return fail(RJPATH_EINVAL, "null argument");
    *out = nullptr;
    if (d->n_media < 1) return fail(RJPATH_EINVAL, "n_media must be >= 1");
    if (!d->axis || !d->layer_off || !d->layer_cnt || !d->edges || !d->lam_s || !d->lam_a || !d->g || !d->f_sl)
        return fail(RJPATH_EINVAL, "null medium array");
    const int M = d->n_media;
    int L = 0;
    std::vector<MedInfo> info(M);
    for (int m = 0; m < M; ++m) {
        int off = d->layer_off[m], cnt = d->layer_cnt[m];
        if (cnt < 1) return fail(RJPATH_EINVAL, "medium " + std::to_string(m) + " has no layer");
        if (off != L) return fail(RJPATH_EINVAL, "layer_off must be the running sum of layer_cnt");
        L += cnt;
        const double* ax = d->axis + 3 * m;
        double an = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
        if (!(std::fabs(an - 1.0) < 1e-9)) return fail(RJPATH_EINVAL, "medium axis must be a unit vector");
        const double* e = d->edges + off + m;
        bool uni = true;
        for (int l = 0; l < cnt; ++l) {
            if (!(e[l + 1] > e[l])) return fail(RJPATH_EINVAL, "edges must be strictly increasing");
        }
        double h = (e[cnt] - e[0]) / cnt;
        for (int l = 0; l <= cnt; ++l)
            if (std::fabs(e[l] - (e[0] + l * h)) > 1e-9 * std::max(1.0, std::fabs(e[l]))) uni = false;
        info[m] = MedInfo{off, cnt, uni ? 1 : 0, 0, ax[0], ax[1], ax[2], e[0], 1.0 / h};
    }
    std::vector<double> lay(L * LY_NW), edge(L + M), pre(2 * (L + M));
    for (int l = 0; l < L; ++l) {
        double ls = d->lam_s[l], la = d->lam_a[l], g = d->g[l], f = d->f_sl[l];
        if (!(ls > 0) || !(la > 0)) return fail(RJPATH_EINVAL, "scattering and absorption lengths must be > 0");
        if (!(std::fabs(g) < 1)) return fail(RJPATH_EINVAL, "|g| must be < 1");
        if (!(f >= 0 && f <= 1)) return fail(RJPATH_EINVAL, "f_sl must lie in [0, 1]");
        if (f > 0 && !(g > 0)) return fail(RJPATH_EINVAL, "the simplified-Liu term needs g > 0");
        double a = std::isinf(la) ? 0.0 : 1.0 / la, b = std::isinf(ls) ? 0.0 : 1.0 / ls;
        double* y = &lay[l * LY_NW];
        y[LY_A] = a;
        y[LY_B] = b;
        y[LY_C] = a + b;
        y[LY_LOGB] = b > 0 ? std::log(b) : -INFINITY;
        y[LY_G] = g;
        y[LY_HGN] = std::log((1 - g * g) / (4 * PI));
        y[LY_HG1] = (1 - g) * (1 - g);
        y[LY_KEQ] = kappa_eq(g);
        y[LY_FSL] = f;
        y[LY_SLN] = g > 0 ? std::log((1 + g) / (1 - g) / (4 * PI)) : 0.0;
        y[LY_SLA] = g > 0 ? 2 * g / (1 - g) : 0.0;
        y[LY_NW - 1] = 0.0;
    }
    for (int m = 0; m < M; ++m) {
        int off = info[m].off, cnt = info[m].cnt;
        const double* e = d->edges + off + m;
        double pc = 0, pb = 0;
        for (int l = 0; l <= cnt; ++l) {
            edge[off + m + l] = e[l];
            pre[2 * (off + m + l)] = pc;
            pre[2 * (off + m + l) + 1] = pb;
            if (l < cnt) {
                pc += lay[(off + l) * LY_NW + LY_C] * (e[l + 1] - e[l]);
                pb += lay[(off + l) * LY_NW + LY_B] * (e[l + 1] - e[l]);
            }
        }
    }
    std::vector<float> lay32(lay.begin(), lay.end());
    std::vector<double> gl(240);
    int o = 0;
    for (int n : {8, 16, 32, 64}) {
        gl01(n, &gl[o], &gl[120 + o]);
        o += n;
    }
    rjpath_medium* h = new rjpath_medium;
    h->n_media = M;
    h->L_total = L;
    h->n_edges = L + M;
    for (int mi = 0; mi < M; ++mi) h->layered |= info[mi].cnt > 1;
    for (int l = 0; l < L; ++l) h->has_sl |= lay[l * LY_NW + LY_FSL] > 0;
    hipStream_t s = (hipStream_t)stream;
    auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up((void**)&h->d_info, info.data(), sizeof(MedInfo) * M);
    if (e == hipSuccess) e = up((void**)&h->d_edge, edge.data(), sizeof(double) * edge.size());
    if (e == hipSuccess) e = up((void**)&h->d_pre, pre.data(), sizeof(double) * pre.size());
    if (e == hipSuccess) e = up((void**)&h->d_lay32, lay32.data(), sizeof(float) * lay32.size());
    if (e == hipSuccess) e = up((void**)&h->d_lay64, lay.data(), sizeof(double) * lay.size());
    if (e == hipSuccess) e = up((void**)&h->d_gl, gl.data(), sizeof(double) * gl.size());
    if (e == hipSuccess) e = set_run_lds_limit();
    if (e != hipSuccess) {
        rjpath_free_medium(h);
        return hip_fail(e, "rjpath_init_medium");
    }
    *out = h;
    return RJPATH_OK;
}

int rjpath_free_medium(rjpath_medium* h) {
    if (!h) return RJPATH_OK;
    hipFree(h->d_info);
    hipFree(h->d_edge);
    hipFree(h->d_pre);
    hipFree(h->d_lay32);
    hipFree(h->d_lay64);
    hipFree(h->d_gl);
    hipFree(h->d_ws);
    delete h;
    return RJPATH_OK;
}

} // extern "C"

namespace {

int check_targets(const rjpath_medium* m, const rjpath_targets* t) {
    if (!m || !t) return fail(RJPATH_EINVAL, "null handle or targets");
    if (t->n_targets < 1) return fail(RJPATH_EINVAL, "n_targets must be >= 1");
    if (!t->medium || !t->src || !t->sensor || !t->radius || !t->emit_kind || !t->emit_dir || !t->emit_param ||
        !t->det_kind || !t->det_dir || !t->n0)
        return fail(RJPATH_EINVAL, "null target array");
    return RJPATH_OK;
}

int grow_ws(rjpath_medium* m, size_t need) {
    if (need <= m->ws_bytes) return RJPATH_OK;
    if (m->d_ws) HIPCHK(hipFree(m->d_ws), "hipFree");
    m->d_ws = nullptr;
    m->ws_bytes = 0;
    if (hipMalloc((void**)&m->d_ws, need) != hipSuccess) return fail(RJPATH_ENOMEM, "workspace allocation");
    m->ws_bytes = need;
    return RJPATH_OK;
}

int check_common(const rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c) {
    int r = check_targets(m, t);
    if (r) return r;
    if (!c) return fail(RJPATH_EINVAL, "null chains");
    if (c->n_chains < 1) return fail(RJPATH_EINVAL, "n_chains must be >= 1");
    if (c->cap < 2 || c->cap > 4096) return fail(RJPATH_EINVAL, "cap must lie in [2, 4096]");
    if (c->precision != RJPATH_F32 && c->precision != RJPATH_F64) return fail(RJPATH_EINVAL, "bad precision");
    if (!c->target || !c->n || !c->verts || !c->logp || !c->status || !c->stats)
        return fail(RJPATH_EINVAL, "null chain array");
    return RJPATH_OK;
}

KArgs make_args(const rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c) {
    KArgs a{};
    if (!c) {
        static const rjpath_chains none{};
        c = &none;
    }
    a.C = c->n_chains;
    a.cap = c->cap;
    a.prec = c->precision;
    a.target = c->target;
    a.n = c->n;
    a.verts = c->verts;
    a.logp = c->logp;
    a.status = c->status;
    a.stats = c->stats;
    a.work = c->work;
    a.T = t->n_targets;
    a.medium = t->medium;
    a.src = t->src;
    a.sensor = t->sensor;
    a.radius = t->radius;
    a.ek = t->emit_kind;
    a.edir = t->emit_dir;
    a.eparam = t->emit_param;
    a.dk = t->det_kind;
    a.ddir = t->det_dir;
    a.n0 = t->n0;
    a.logw = t->logw;
    a.n_media = m->n_media;
    a.minfo = m->d_info;
    a.edge = m->d_edge;
    a.pre = m->d_pre;
    a.lay = c->precision == RJPATH_F64 ? (const void*)m->d_lay64 : (const void*)m->d_lay32;
    a.lay64 = m->d_lay64;
    a.L_total = m->L_total;
    a.n_edges = m->n_edges;
    a.layered = m->layered;
    a.has_sl = m->has_sl;
    a.tab_bytes = 0;
    if (m->layered && c->precision == RJPATH_F32) {
        // layer table, edges padded to an even count, prefix pairs (the run kernel's LDS layout)
        size_t lay = ((size_t)m->L_total * LY_NW * (c->precision == RJPATH_F64 ? 8 : 4) + 15) & ~(size_t)15;
        size_t bytes = lay + 8 * (((size_t)m->n_edges + 1) & ~(size_t)1) + 16 * (size_t)m->n_edges;
        if (bytes <= 48 * 1024) a.tab_bytes = bytes;
    }
    return a;
}

size_t vtx_bytes(int prec) { return prec == RJPATH_F64 ? 32 : 16; }

const size_t LDS_MAX = 160 * 1024;

// LDS left for the per-lane vertex slots once the media tables are staged
size_t slot_budget(const rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c) {
    return LDS_MAX - make_args(m, t, c).tab_bytes;
}

// Compute units of the current device (the occupancy rule below needs them).
int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

// Default launch configuration.  One wave per SIMD issues at most about one
// instruction per two issue slots of its SIMD, and a second resident wave
// nearly doubles the SIMD's throughput (measured on gfx950).  So:
//  - fewer chains than two waves per SIMD: one 64-chain wave per block with
//    32 slots per lane (16 in FP64), the fastest configuration measured for
//    one wave per SIMD;
//  - otherwise (FP32): 256-chain blocks with as many slots as let two blocks
//    (eight waves) share a CU's LDS, so that two waves are resident per SIMD
//    (the step kernel's register use allows two).
void default_launch(const rjpath_chains* c, size_t tab_bytes, int& block, int& V) {
    const int cap = c->cap;
    block = 64;
    V = std::min(cap, c->precision == RJPATH_F64 ? 16 : 32);
    const long long two_waves = 2LL * 4 * device_cus() * 64;
    if (c->precision == RJPATH_F32 && (long long)c->n_chains >= two_waves) {
        const size_t per_block = LDS_MAX / 2;
        if (per_block > tab_bytes) {
            const long long slots = (long long)((per_block - tab_bytes) / (256 * vtx_bytes(RJPATH_F32))) - 2;
            if (slots >= 8) {
                block = 256;
                V = (int)std::min<long long>(std::min(cap, 32), slots);
            }
        }
    }
}

int run_impl(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, const rjpath_run_params* p,
             hipStream_t s, int block, int V) {
    KArgs a = make_args(m, t, c);
    a.V = V;
    a.seed = p->seed;
    a.burn_in = p->burn_in;
    a.cycle_len = p->cycle_len;
    a.n_perturb = p->n_perturb;
    a.bthresh = p->birth_thresh;
    a.sigma = p->sigma;
    a.kappa_end = p->kappa_end;
    a.mala_h = p->mala_h;
    a.sampler = p->sampler;
    a.trace = p->trace;
    a.trace_steps = p->steps;
    a.hist = p->hist;
    a.step_dev = p->step_counter;
    int chunk = p->chunk > 0 ? p->chunk : p->steps;
    for (int done = 0; done < p->steps; done += chunk) {
        // with a device counter, step0 carries the offset inside this call
        a.step0 = (p->step_counter ? 0 : p->step0) + (uint64_t)done;
        a.steps = std::min(chunk, p->steps - done);
        a.trace_off = done;
        hipError_t e = launch_run(a, block, s);
        if (e != hipSuccess) return hip_fail(e, "run kernel launch");
    }
    if (p->step_counter) {
        hipError_t e = launch_advance(p->step_counter, (uint64_t)p->steps, s);
        if (e != hipSuccess) return hip_fail(e, "step counter kernel launch");
    }
    return RJPATH_OK;
}

int check_run(const rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, const rjpath_run_params* p) {
    int r = check_common(m, t, c);
    if (r) return r;
    if (!p) return fail(RJPATH_EINVAL, "null run parameters");
    if (p->steps < 0) return fail(RJPATH_EINVAL, "steps must be >= 0");
    if (p->cycle_len < 1 || p->n_perturb < 0 || p->n_perturb > p->cycle_len)
        return fail(RJPATH_EINVAL, "need 1 <= cycle_len and 0 <= n_perturb <= cycle_len");
    if (p->n_perturb < p->cycle_len && (p->birth_thresh == 0u))
        return fail(RJPATH_EINVAL, "birth_thresh must be > 0 when jump steps are scheduled");
    if (!(p->sigma > 0) || !(p->kappa_end > 0)) return fail(RJPATH_EINVAL, "sigma and kappa_end must be > 0");
    if (p->sampler != RJPATH_PLAIN && p->sampler != RJPATH_MALA && p->sampler != RJPATH_LMALA &&
        p->sampler != RJPATH_TREE)
        return fail(RJPATH_EINVAL, "bad sampler");
    if (p->sampler != RJPATH_PLAIN && !(p->mala_h > 0)) return fail(RJPATH_EINVAL, "mala_h must be > 0");
    if ((p->sampler == RJPATH_MALA || p->sampler == RJPATH_TREE) && !c->work)
        return fail(RJPATH_EINVAL, "the joint Langevin and tree samplers need the chains' work buffer");
    if (p->block_chains != 0 && (p->block_chains % 64 != 0 || p->block_chains < 64 || p->block_chains > 256))
        return fail(RJPATH_EINVAL, "block_chains must be 64, 128, 192 or 256");
    if (p->v_lds < 0 || p->v_lds > c->cap) return fail(RJPATH_EINVAL, "v_lds must lie in [0, cap]");
    if (p->chunk < 0) return fail(RJPATH_EINVAL, "chunk must be >= 0");
    if (p->step_counter && p->trace) return fail(RJPATH_EINVAL, "trace needs a host step0 (no step_counter)");
    return RJPATH_OK;
}

} // namespace

extern "C" {

int rjpath_run_chains(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, const rjpath_run_params* p,
                      void* stream) {
    int r = check_run(m, t, c, p);
    if (r) return r;
    if (p->steps == 0) return RJPATH_OK;
    int block, V;
    default_launch(c, make_args(m, t, c).tab_bytes, block, V);
    auto it = m->tuned.find(TuneKey{c->cap, c->precision, p->sampler});
    if (it != m->tuned.end()) {
        block = it->second.first;
        V = it->second.second;
    }
    if (p->block_chains) block = p->block_chains;
    if (p->v_lds) V = p->v_lds;
    const size_t budget = slot_budget(m, t, c);
    // each lane's tile holds V slots plus two padding slots
    if ((size_t)(V + 2) * block * vtx_bytes(c->precision) > budget) {
        if (p->v_lds)
            return fail(RJPATH_EINVAL, "(v_lds + 2) * block_chains vertices exceed the LDS left after the media tables");
        V = (int)(budget / (block * vtx_bytes(c->precision))) - 2;
        if (V < 1) return fail(RJPATH_EINVAL, "no LDS left for vertex slots after the media tables");
    }
    return run_impl(m, t, c, p, (hipStream_t)stream, block, V);
}

int rjpath_autotune(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, const rjpath_run_params* p,
                    int32_t steps, int32_t* best_block, int32_t* best_v, void* stream) {
    int r = check_run(m, t, c, p);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    std::vector<std::pair<int, int>> cand;
    const size_t budget = slot_budget(m, t, c);
    {
        // the default launch is always a candidate
        int db, dv;
        default_launch(c, make_args(m, t, c).tab_bytes, db, dv);
        if ((size_t)(dv + 2) * db * vtx_bytes(c->precision) <= budget) cand.push_back({db, dv});
    }
    for (int b : {64, 256})
        for (int v : {8, 12, 16, 24, 32}) {
            int vv = std::min(v, c->cap);
            if ((size_t)(vv + 2) * b * vtx_bytes(c->precision) > budget) continue;
            if (std::find(cand.begin(), cand.end(), std::make_pair(b, vv)) == cand.end()) cand.push_back({b, vv});
        }
    // two passes, the second in reverse order, so that the drift of the chain
    // state during the trials (paths lengthening after a start) favours no candidate
    const int nc = (int)cand.size();
    int trial = steps / (2 * nc);
    if (trial < 1) return fail(RJPATH_EINVAL, "autotune needs steps >= " + std::to_string(2 * nc));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0), "hipEventCreate");
    HIPCHK(hipEventCreate(&e1), "hipEventCreate");
    rjpath_run_params q = *p;
    q.steps = trial;
    q.trace = nullptr;
    q.hist = nullptr;
    q.chunk = 0;
    std::vector<double> tms(nc, 0.0);
    uint64_t step = p->step0;
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < nc; ++i) {
            const auto& cv = cand[pass == 0 ? i : nc - 1 - i];
            q.step0 = step;
            HIPCHK(hipEventRecord(e0, s), "hipEventRecord");
            int rr = run_impl(m, t, c, &q, s, cv.first, cv.second);
            if (rr) return rr;
            HIPCHK(hipEventRecord(e1, s), "hipEventRecord");
            HIPCHK(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            tms[pass == 0 ? i : nc - 1 - i] += ms;
            step += trial;
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    std::pair<int, int> bc = cand[std::min_element(tms.begin(), tms.end()) - tms.begin()];
    // the remainder of the requested steps with the chosen configuration
    int rest = steps - 2 * trial * nc;
    if (rest > 0) {
        q.step0 = step;
        q.steps = rest;
        int rr = run_impl(m, t, c, &q, s, bc.first, bc.second);
        if (rr) return rr;
    }
    m->tuned[TuneKey{c->cap, c->precision, p->sampler}] = bc;
    if (best_block) *best_block = bc.first;
    if (best_v) *best_v = bc.second;
    return RJPATH_OK;
}

int rjpath_tune_proposal(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, const rjpath_run_params* p,
                         int32_t n_cand, const rjpath_proposal* cand, int32_t trial_steps, int32_t groups,
                         double* score, int32_t* best, void* stream) {
    int r = check_run(m, t, c, p);
    if (r) return r;
    if (n_cand < 1 || !cand) return fail(RJPATH_EINVAL, "need at least one candidate");
    if (trial_steps < 1) return fail(RJPATH_EINVAL, "trial_steps must be >= 1");
    if (groups < 2 || groups > 64) return fail(RJPATH_EINVAL, "groups must lie in [2, 64]");
    if (p->step_counter || p->trace) return fail(RJPATH_EINVAL, "rjpath_tune_proposal takes a host step0 and no trace");
    for (int i = 0; i < n_cand; ++i) {
        rjpath_run_params q = *p;
        q.sigma = cand[i].sigma;
        q.kappa_end = cand[i].kappa_end;
        q.mala_h = cand[i].mala_h;
        q.cycle_len = cand[i].cycle_len;
        q.n_perturb = cand[i].n_perturb;
        r = check_run(m, t, c, &q);
        if (r) return fail(r, "candidate " + std::to_string(i) + ": " + g_err);
    }
    hipStream_t s = (hipStream_t)stream;
    const int T = t->n_targets;
    // the trials' statistics go to a buffer of their own: the caller's are untouched
    double* tstats = nullptr;
    const size_t nst = (size_t)c->n_chains * RJPATH_NSTAT;
    if (hipMalloc((void**)&tstats, sizeof(double) * nst) != hipSuccess)
        return fail(RJPATH_ENOMEM, "trial statistics allocation");
    rjpath_chains cc = *c;
    cc.stats = tstats;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<double> ms(n_cand, 0.0), r2sum(n_cand, 0.0);
    std::vector<double> ones(T, 1.0), I(T), se(T);
    uint64_t step = p->step0;
    auto cleanup = [&]() {
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        hipFree(tstats);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(RJPATH_EHIP, "hipEventCreate");
    }
    // two passes, the second in reverse order, so that slow drift of the
    // chains during the trials favours no candidate
    for (int pass = 0; pass < 2 && r == RJPATH_OK; ++pass)
        for (int j = 0; j < n_cand && r == RJPATH_OK; ++j) {
            const int i = pass == 0 ? j : n_cand - 1 - j;
            rjpath_run_params q = *p;
            q.sigma = cand[i].sigma;
            q.kappa_end = cand[i].kappa_end;
            q.mala_h = cand[i].mala_h;
            q.cycle_len = cand[i].cycle_len;
            q.n_perturb = cand[i].n_perturb;
            q.step0 = step;
            q.burn_in = (int64_t)step; // every trial step is sampled
            q.steps = trial_steps;
            q.hist = nullptr;
            q.chunk = 0;
            hipError_t e = fill_f64(tstats, nst, 0.0, s);
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            if (e != hipSuccess) {
                r = hip_fail(e, "trial setup");
                break;
            }
            r = rjpath_run_chains(m, t, &cc, &q, stream);
            if (r) break;
            e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t_ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&t_ms, e0, e1);
            if (e != hipSuccess) {
                r = hip_fail(e, "trial timing");
                break;
            }
            ms[i] += t_ms;
            step += trial_steps;
            // relative error of each target's estimator ratio over this trial
            // (the anchor cancels in se / I)
            int rr = rjpath_intensity(m, t, &cc, groups, ones.data(), I.data(), se.data(), nullptr, nullptr, stream);
            if (rr != RJPATH_OK && rr != RJPATH_ENODATA) {
                r = rr;
                break;
            }
            std::vector<double> rel;
            for (int k = 0; k < T; ++k)
                if (I[k] > 0 && se[k] > 0) rel.push_back((se[k] / I[k]) * (se[k] / I[k]));
            double med = INFINITY; // a trial without any usable target scores 0
            if (!rel.empty()) {
                std::nth_element(rel.begin(), rel.begin() + rel.size() / 2, rel.end());
                med = rel[rel.size() / 2];
            }
            r2sum[i] += med;
        }
    cleanup();
    if (r) return r;
    int bi = 0;
    double bs = -1;
    for (int i = 0; i < n_cand; ++i) {
        // ESS per second of the median target: 1 / (r^2 x time), both passes together
        const double sc = r2sum[i] > 0 && std::isfinite(r2sum[i]) ? 4.0 / (r2sum[i] * ms[i] * 1e-3) : 0.0;
        if (score) score[i] = sc;
        if (sc > bs) {
            bs = sc;
            bi = i;
        }
    }
    if (best) *best = bi;
    return RJPATH_OK;
}

int rjpath_grad(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, double* logp_out, void* dlogp_dv,
                double* score, void* stream) {
    int r = check_common(m, t, c);
    if (r) return r;
    KArgs a = make_args(m, t, c);
    hipError_t e = launch_grad(a, logp_out, dlogp_dv, score, m->L_total, 0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "grad kernel launch");
    return RJPATH_OK;
}

int rjpath_score_length(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, double* score_L,
                        void* stream) {
    int r = check_common(m, t, c);
    if (r) return r;
    if (!score_L) return fail(RJPATH_EINVAL, "null score_L");
    KArgs a = make_args(m, t, c);
    hipError_t e = launch_grad(a, nullptr, nullptr, score_L, m->L_total, 1, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "grad kernel launch");
    return RJPATH_OK;
}

int rjpath_dlength_dtheta(rjpath_medium* m, const rjpath_targets* t, const double* score, const double* score_L,
                          double* mean_L, double* dmean_L, void* stream) {
    int r = check_targets(m, t);
    if (r) return r;
    if (!score || !score_L || !dmean_L) return fail(RJPATH_EINVAL, "null score, score_L or dmean_L");
    HIPCHK(launch_dlength(t->n_targets, 3 * m->L_total, score, score_L, mean_L, dmean_L, (hipStream_t)stream),
           "dlength kernel launch");
    return RJPATH_OK;
}

int rjpath_tune_tilt(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, const rjpath_run_params* p,
                     int32_t rounds, uint32_t* hist, double max_logw, double floor_push, void* stream) {
    int r = check_run(m, t, c, p);
    if (r) return r;
    if (!t->logw) return fail(RJPATH_EINVAL, "rjpath_tune_tilt needs the targets' logw table (updated in place)");
    if (!hist) return fail(RJPATH_EINVAL, "null histogram workspace");
    if (rounds < 1 || p->steps < 1) return fail(RJPATH_EINVAL, "rounds and steps must be >= 1");
    if (p->step_counter || p->trace) return fail(RJPATH_EINVAL, "rjpath_tune_tilt takes a host step0 and no trace");
    if (!(max_logw >= 0) || !(floor_push >= 0)) return fail(RJPATH_EINVAL, "max_logw and floor_push must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    const size_t nh = (size_t)t->n_targets * (c->cap + 1);
    rjpath_run_params q = *p;
    q.hist = hist;
    q.chunk = 0;
    for (int i = 0; i < rounds; ++i) {
        q.step0 = p->step0 + (uint64_t)i * p->steps;
        // pilot steps leave the chain statistics untouched
        q.burn_in = (int64_t)(q.step0 + p->steps);
        HIPCHK(fill_u32(hist, nh, 0u, s), "fill kernel launch");
        r = rjpath_run_chains(m, t, c, &q, stream);
        if (r) return r;
        HIPCHK(launch_tilt(t->n_targets, c->cap, t->n0, hist, (double*)t->logw, max_logw, floor_push, s),
               "tilt kernel launch");
    }
    return RJPATH_OK;
}

int rjpath_dlogi_dtheta(rjpath_medium* m, const rjpath_targets* t, const double* score, double* dlogI, void* stream) {
    int r = check_targets(m, t);
    if (r) return r;
    if (!score || !dlogI) return fail(RJPATH_EINVAL, "null score or dlogI");
    HIPCHK(launch_dlogi(t->n_targets, 3 * m->L_total, score, dlogI, (hipStream_t)stream), "dlogI kernel launch");
    return RJPATH_OK;
}

int rjpath_anchor(rjpath_medium* m, const rjpath_targets* t, double* anchor, void* stream) {
    if (!anchor) return fail(RJPATH_EINVAL, "null anchor output");
    int r = check_targets(m, t);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    const int T = t->n_targets;
    r = grow_ws(m, sizeof(double) * T);
    if (r) return r;
    KArgs a = make_args(m, t, nullptr);
    HIPCHK(launch_anchor(a, m->d_gl, m->d_gl + 120, 120, m->d_ws, s), "anchor kernel launch");
    HIPCHK(hipMemcpyAsync(anchor, m->d_ws, sizeof(double) * T, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    HIPCHK(hipStreamSynchronize(s), "hipStreamSynchronize");
    return RJPATH_OK;
}

int rjpath_intensity_noalloc(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, int32_t groups,
                             const double* anchor, double* I, double* se, double* ess, double* rhat, void* stream) {
    int r = check_common(m, t, c);
    if (r) return r;
    if (groups < 2 || groups > 64) return fail(RJPATH_EINVAL, "groups must lie in [2, 64]");
    const size_t need = (size_t)t->n_targets * groups * RD_NW + (anchor ? 0 : (size_t)t->n_targets);
    const size_t cap = noalloc_scratch_doubles();
    if (need > cap)
        return fail(RJPATH_EINVAL, "rjpath_intensity_noalloc: n_targets * groups * 6 (+ n_targets without anchors) = " +
                                       std::to_string(need) + " doubles exceeds its static buffer of " +
                                       std::to_string(cap));
    KArgs a = make_args(m, t, c);
    HIPCHK(launch_intensity_noalloc(a, groups, anchor, m->d_gl, I, se, ess, rhat, (hipStream_t)stream),
           "rjpath_intensity_noalloc kernels");
    return RJPATH_OK;
}

int rjpath_yield_accumulate(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, int32_t n_pairs,
                            const int32_t* pairs, const int32_t* role, int32_t groups, double* acc, double* logr,
                            void* stream) {
    int r = check_common(m, t, c);
    if (r) return r;
    if (n_pairs < 1) return fail(RJPATH_EINVAL, "n_pairs must be >= 1");
    if (!pairs || !role || !acc) return fail(RJPATH_EINVAL, "null pairs, role or acc");
    if (groups < 2 || groups > 64) return fail(RJPATH_EINVAL, "groups must lie in [2, 64]");
    KArgs a = make_args(m, t, c);
    HIPCHK(launch_yield(a, n_pairs, pairs, role, groups, acc, logr, (hipStream_t)stream), "yield kernel launch");
    return RJPATH_OK;
}

int rjpath_yield(int32_t n_pairs, int32_t groups, const double* acc, double* B, double* se, void* stream) {
    if (n_pairs < 1) return fail(RJPATH_EINVAL, "n_pairs must be >= 1");
    if (groups < 2 || groups > 64) return fail(RJPATH_EINVAL, "groups must lie in [2, 64]");
    if (!acc) return fail(RJPATH_EINVAL, "null acc");
    hipStream_t s = (hipStream_t)stream;
    const size_t na = (size_t)n_pairs * 2 * groups * 2;
    std::vector<double> h(na);
    HIPCHK(hipMemcpyAsync(h.data(), acc, sizeof(double) * na, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    HIPCHK(hipStreamSynchronize(s), "hipStreamSynchronize");
    bool nodata = false;
    for (int k = 0; k < n_pairs; ++k) {
        // side-wise sums of sqrt(r) / w and 1 / w; the bridge is their ratio of ratios
        auto at = [&](int side, int g, int j) { return h[(((size_t)k * 2 + side) * groups + g) * 2 + j]; };
        double S[2] = {0, 0}, W[2] = {0, 0};
        for (int side = 0; side < 2; ++side)
            for (int g = 0; g < groups; ++g) {
                S[side] += at(side, g, 0);
                W[side] += at(side, g, 1);
            }
        double Bk = NAN, sek = NAN;
        if (W[0] > 0 && W[1] > 0 && S[1] > 0) {
            Bk = (S[0] / W[0]) / (S[1] / W[1]);
            std::vector<double> jk;
            for (int g = 0; g < groups; ++g) {
                if (at(0, g, 1) == 0 && at(1, g, 1) == 0) continue;
                const double w0 = W[0] - at(0, g, 1), w1 = W[1] - at(1, g, 1), s1 = S[1] - at(1, g, 0);
                if (!(w0 > 0) || !(w1 > 0) || !(s1 > 0)) {
                    jk.clear();
                    break;
                }
                jk.push_back(((S[0] - at(0, g, 0)) / w0) / (s1 / w1));
            }
            const int G = (int)jk.size();
            if (G >= 2) {
                double mj = 0, ss = 0;
                for (double v : jk) mj += v;
                mj /= G;
                for (double v : jk) ss += (v - mj) * (v - mj);
                sek = std::sqrt((G - 1.0) / G * ss);
            }
        } else {
            nodata = true;
        }
        if (B) B[k] = Bk;
        if (se) se[k] = sek;
    }
    if (nodata) return fail(RJPATH_ENODATA, "a pair has no samples on one side (or no overlap)");
    return RJPATH_OK;
}

int rjpath_length_hist(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, int32_t bins, double l0,
                       double bin_width, double* hist, void* stream) {
    int r = check_common(m, t, c);
    if (r) return r;
    if (bins < 1 || bins > (1 << 20)) return fail(RJPATH_EINVAL, "bins must lie in [1, 2^20]");
    if (!(bin_width > 0) || !std::isfinite(l0)) return fail(RJPATH_EINVAL, "bin_width must be > 0 and l0 finite");
    if (!hist) return fail(RJPATH_EINVAL, "null hist");
    KArgs a = make_args(m, t, c);
    HIPCHK(launch_lhist(a, bins, l0, bin_width, hist, (hipStream_t)stream), "length histogram kernel launch");
    return RJPATH_OK;
}

int rjpath_intensity(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, int32_t groups,
                     const double* anchor, double* I, double* se, double* ess, double* rhat, void* stream) {
    int r = check_common(m, t, c);
    if (r) return r;
    if (groups < 2 || groups > 64) return fail(RJPATH_EINVAL, "groups must lie in [2, 64]");
    hipStream_t s = (hipStream_t)stream;
    const int T = t->n_targets;
    std::vector<double> anc(T);
    if (anchor) {
        std::copy(anchor, anchor + T, anc.begin());
    } else {
        r = rjpath_anchor(m, t, anc.data(), stream);
        if (r) return r;
    }
    size_t nred = (size_t)T * groups * RD_NW;
    r = grow_ws(m, sizeof(double) * nred);
    if (r) return r;
    double* d_red = m->d_ws;
    KArgs a = make_args(m, t, c);
    HIPCHK(fill_f64(d_red, nred, 0.0, s), "fill kernel launch");
    HIPCHK(launch_reduce(a, groups, d_red, s), "reduce kernel launch");
    std::vector<double> red(nred);
    HIPCHK(hipMemcpyAsync(red.data(), d_red, sizeof(double) * nred, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    HIPCHK(hipStreamSynchronize(s), "hipStreamSynchronize");
    bool nodata = false;
    for (int ti = 0; ti < T; ++ti) {
        const double* rt = &red[(size_t)ti * groups * RD_NW];
        double A = 0, B = 0, chains = 0;
        for (int g = 0; g < groups; ++g) {
            A += rt[g * RD_NW + RD_A];
            B += rt[g * RD_NW + RD_B];
            chains += rt[g * RD_NW + RD_CHAINS];
        }
        double Ii = NAN, sei = NAN, rh = NAN;
        if (chains > 0 && !(B > 0)) nodata = true;
        if (B > 0) {
            Ii = anc[ti] * A / B;
            // delete-one-group jackknife over the non-empty groups
            std::vector<double> jk;
            for (int g = 0; g < groups; ++g) {
                if (rt[g * RD_NW + RD_CHAINS] == 0) continue;
                double Bg = B - rt[g * RD_NW + RD_B];
                if (!(Bg > 0)) {
                    jk.clear();
                    break;
                }
                jk.push_back(anc[ti] * (A - rt[g * RD_NW + RD_A]) / Bg);
            }
            int G = (int)jk.size();
            if (G >= 2) {
                double mj = 0;
                for (double v : jk) mj += v;
                mj /= G;
                double ss = 0;
                for (double v : jk) ss += (v - mj) * (v - mj);
                sei = std::sqrt((G - 1.0) / G * ss);
            }
            // potential scale reduction of the path length across groups
            double W = 0, mb = 0, nb = 0;
            std::vector<double> mg;
            for (int g = 0; g < groups; ++g) {
                double ns = rt[g * RD_NW + RD_SAMPLES];
                if (ns < 2) continue;
                double mu = rt[g * RD_NW + RD_L] / ns;
                W += rt[g * RD_NW + RD_L2] / ns - mu * mu;
                mg.push_back(mu);
                nb += ns;
            }
            if (mg.size() >= 2) {
                int k = (int)mg.size();
                W /= k;
                nb /= k;
                for (double v : mg) mb += v;
                mb /= k;
                double Bv = 0;
                for (double v : mg) Bv += (v - mb) * (v - mb);
                Bv /= (k - 1);
                if (W > 0) rh = std::sqrt(((nb - 1) / nb * W + Bv) / W);
            }
        }
        if (I) I[ti] = Ii;
        if (se) se[ti] = sei;
        if (ess) ess[ti] = (sei > 0) ? (Ii / sei) * (Ii / sei) : NAN;
        if (rhat) rhat[ti] = rh;
    }
    if (nodata) return fail(RJPATH_ENODATA, "a target has no anchor-sector visits");
    return RJPATH_OK;
}

} // extern "C"
