// rj_step.h -- the fused reversible-jump step kernel for gfx950 (templates;
// instantiated per precision and sampler in the rj_run_*.hip units).
//
// One chain per lane.  A block owns a tile of chains for every step of the
// launch.  The first V vertices of each chain live in LDS in a vertex-major,
// lane-minor layout ([slot][lane]: per-lane random slots stay conflict-free),
// the rest stay in the caller's HBM array (same [v][C] layout, read and
// written coalesced at launch start and end).  When every lane of a wave fits
// its LDS slots (a wave vote per step) the step runs a branch-free LDS-only
// instantiation.  Layered media are staged in LDS once per block; a
// homogeneous medium lives in registers.
//
// Every step of a launch is the same move class for all lanes (the move
// schedule depends only on the global step index), so waves diverge only
// inside a class: interior and end-point perturbations share one
// local-density evaluator, births and deaths share one jump evaluator.
//
// Method references: path density (App. "Path probability distribution"),
// jump proposal and bi-spherical map (App. "Jump proposal", "Dimension
// matching transformation"), acceptance (eq. acceptFact read in Green's
// form), end-point move on the sensor and proposal mix (Sec. "Path proposal
// distribution"); the Langevin move follows the Discussion's suggestion of
// gradient-informed moves.
#pragma once

#include <hip/hip_runtime.h>

#include "rj_device.h"
#include "rj_kernels.h"

namespace rj {

enum { MV_INTERIOR = 0, MV_END = 1, MV_BIRTH = 2, MV_DEATH = 3, MV_MALA = 4, MV_NULL = 5, MV_LMALA = 6, MV_TREE = 7 };

// Interior-vertex move of the sampler (RJPATH_PLAIN / _MALA / _LMALA / _TREE).
enum { SAMP_PLAIN = 0, SAMP_JOINT = 1, SAMP_LOCAL = 2, SAMP_TREE = 3 };

// Lane-private path storage: slots below V in LDS, the rest in HBM.  LO: the
// whole path is known to be in LDS.  The LDS side is addressed through an
// address-space-3 pointer to a 4-vector, so that every access is one ds_*
// instruction (never a generic flat access).
template <class R> using L4 = R __attribute__((ext_vector_type(4)));
template <class R> using LdsPtr = __attribute__((address_space(3))) L4<R>*;
template <class R> using LdsScalar = __attribute__((address_space(3))) R*;

template <class R> __device__ __forceinline__ Vtx<R> lds_ld(LdsPtr<R> p) {
    const L4<R> q = *p;
    return Vtx<R>{q.x, q.y, q.z, q.w};
}
template <class R> __device__ __forceinline__ void lds_st(LdsPtr<R> p, const Vtx<R>& x) { *p = L4<R>{x.x, x.y, x.z, x.w}; }

// LDS layout: each wave owns a tile of V + 2 slots of 64 lanes, slot -1 and
// slot V being padding, so that a slot stride is a constant (64 vertices) and
// the LDS-only step can read the neighbours of a vertex (slots -1 .. n + 1,
// n < V) without clamping their indices: the padding or stale slots it then
// reads are only ever discarded.
constexpr int WAVE = 64;
constexpr int SLOT_PAD = 2;

template <class R, bool LO> struct PathRef {
    LdsPtr<R> lds; // this lane's slot 0, stride WAVE
    Vtx<R>* glb;   // this chain's vertex 0, stride C
    int V;
    size_t C;
    __device__ __forceinline__ Vtx<R> ld(int v) const {
        if (LO || v < V) return lds_ld<R>(lds + v * WAVE);
        return glb[(size_t)v * C];
    }
    __device__ __forceinline__ void st(int v, const Vtx<R>& x) const {
        if (LO || v < V) lds_st<R>(lds + v * WAVE, x);
        else glb[(size_t)v * C] = x;
    }
    __device__ __forceinline__ V3<R> p(int v) const { return pos(ld(v)); }
    __device__ __forceinline__ R w(int v) const {
        if (LO || v < V) return ((LdsScalar<R>)(lds + v * WAVE))[3];
        return glb[(size_t)v * C].w;
    }
    __device__ __forceinline__ void stw(int v, R x) const {
        if (LO || v < V) ((LdsScalar<R>)(lds + v * WAVE))[3] = x;
        else glb[(size_t)v * C].w = x;
    }
    // Five vertices at once.  LDS-only: five reads.  Otherwise five LDS
    // reads (the indices that lie in HBM read the padding slot V instead)
    // and, for the lanes whose five reach HBM, one branch that reads all five
    // from HBM and keeps those (no branch per vertex on the address space).
    __device__ __forceinline__ void ld5(int i0, int i1, int i2, int i3, int i4, Vtx<R>& o0, Vtx<R>& o1, Vtx<R>& o2,
                                        Vtx<R>& o3, Vtx<R>& o4) const {
        const int c0 = LO || i0 < V ? i0 : V, c1 = LO || i1 < V ? i1 : V, c2 = LO || i2 < V ? i2 : V;
        const int c3 = LO || i3 < V ? i3 : V, c4 = LO || i4 < V ? i4 : V;
        o0 = lds_ld<R>(lds + c0 * WAVE);
        o1 = lds_ld<R>(lds + c1 * WAVE);
        o2 = lds_ld<R>(lds + c2 * WAVE);
        o3 = lds_ld<R>(lds + c3 * WAVE);
        o4 = lds_ld<R>(lds + c4 * WAVE);
        if (LO) return;
        const int hi = max(max(max(i0, i1), max(i2, i3)), i4);
        if (hi >= V) {
            const L4<R>* const g = (const L4<R>*)glb;
            const L4<R> g0 = g[(size_t)i0 * C], g1 = g[(size_t)i1 * C], g2 = g[(size_t)i2 * C];
            const L4<R> g3 = g[(size_t)i3 * C], g4 = g[(size_t)i4 * C];
            if (i0 >= V) o0 = Vtx<R>{g0.x, g0.y, g0.z, g0.w};
            if (i1 >= V) o1 = Vtx<R>{g1.x, g1.y, g1.z, g1.w};
            if (i2 >= V) o2 = Vtx<R>{g2.x, g2.y, g2.z, g2.w};
            if (i3 >= V) o3 = Vtx<R>{g3.x, g3.y, g3.z, g3.w};
            if (i4 >= V) o4 = Vtx<R>{g4.x, g4.y, g4.z, g4.w};
        }
    }
    // The vertex shifts of an accepted jump, split at the LDS/HBM boundary
    // into loops that touch one memory each (no per-vertex branch on the
    // address space), each reading four vertices before writing them (one
    // latency per four): slots lo..hi move one slot up (from the top) ...
    __device__ __forceinline__ void lds_up(int& v, int lo) const {
        for (; v - 3 >= lo; v -= 4) {
            const L4<R> a = lds[v * WAVE], b = lds[(v - 1) * WAVE], c = lds[(v - 2) * WAVE], d = lds[(v - 3) * WAVE];
            lds[(v + 1) * WAVE] = a;
            lds[v * WAVE] = b;
            lds[(v - 1) * WAVE] = c;
            lds[(v - 2) * WAVE] = d;
        }
        for (; v >= lo; --v) lds[(v + 1) * WAVE] = lds[v * WAVE];
    }
    __device__ __forceinline__ void shift_up(int lo, int hi) const {
        int v = hi;
        if (!LO) {
            L4<R>* const g = (L4<R>*)glb;
            for (; v - 3 >= lo && v - 3 >= V; v -= 4) {
                const L4<R> a = g[(size_t)v * C], b = g[(size_t)(v - 1) * C], c = g[(size_t)(v - 2) * C],
                            d = g[(size_t)(v - 3) * C];
                g[(size_t)(v + 1) * C] = a;
                g[(size_t)v * C] = b;
                g[(size_t)(v - 1) * C] = c;
                g[(size_t)(v - 2) * C] = d;
            }
            for (; v >= lo && v >= V; --v) g[(size_t)(v + 1) * C] = g[(size_t)v * C];
            if (v >= lo && v == V - 1) {
                g[(size_t)V * C] = lds[v * WAVE];
                --v;
            }
        }
        lds_up(v, lo);
    }
    // ... or slots lo+1..hi+1 move one slot down (from the bottom).
    __device__ __forceinline__ void shift_down(int lo, int hi) const {
        int v = lo;
        const int top = LO ? hi : (hi < V - 2 ? hi : V - 2); // the moves that stay in LDS
        for (; v + 3 <= top; v += 4) {
            const L4<R> a = lds[(v + 1) * WAVE], b = lds[(v + 2) * WAVE], c = lds[(v + 3) * WAVE],
                        d = lds[(v + 4) * WAVE];
            lds[v * WAVE] = a;
            lds[(v + 1) * WAVE] = b;
            lds[(v + 2) * WAVE] = c;
            lds[(v + 3) * WAVE] = d;
        }
        for (; v <= top; ++v) lds[v * WAVE] = lds[(v + 1) * WAVE];
        if (!LO) {
            L4<R>* const g = (L4<R>*)glb;
            if (v <= hi && v == V - 1) {
                lds[v * WAVE] = g[(size_t)V * C];
                ++v;
            }
            for (; v + 3 <= hi; v += 4) {
                const L4<R> a = g[(size_t)(v + 1) * C], b = g[(size_t)(v + 2) * C], c = g[(size_t)(v + 3) * C],
                            d = g[(size_t)(v + 4) * C];
                g[(size_t)v * C] = a;
                g[(size_t)(v + 1) * C] = b;
                g[(size_t)(v + 2) * C] = c;
                g[(size_t)(v + 3) * C] = d;
            }
            for (; v <= hi; ++v) g[(size_t)v * C] = g[(size_t)(v + 1) * C];
        }
    }
};

template <class R> struct GlobalPath {
    Vtx<R>* glb;
    size_t C;
    __device__ __forceinline__ Vtx<R> ld(int v) const { return glb[(size_t)v * C]; }
    __device__ __forceinline__ V3<R> p(int v) const { return pos(ld(v)); }
    __device__ __forceinline__ void stw(int, R) const {}
};

// Full log p of the path (FP64 sum of the factors), refreshing the cached
// segment scattering depths; also returns the path length L and, where Sb is
// given, the FP64 sum of the refreshed depths in path order.
template <class R, class P>
__device__ __forceinline__ double full_logp(const Tgt<R>& T, const P& ps, int n, double& L, double* Sb = nullptr) {
    V3<R> f0 = ps.p(0), f1 = ps.p(1);
    LPt<R> lc = lpt(T, f1);
    Seg<R> s = make_seg_lp(T, f0, f1, lpt(T, f0), lc);
    bool zero = !(s.len > (R)0);
    double lp = (double)emit_term(T, s.u) + (double)seg_term(s);
    L = (double)s.len;
    double sb = (double)s.tb;
    ps.stw(0, s.tb);
    V3<R> fc = f1;
    for (int k = 1; k <= n - 2; ++k) {
        V3<R> fn = ps.p(k + 1);
        const LPt<R> lnx = lpt(T, fn);
        Seg<R> s2 = make_seg_lp(T, fc, fn, lc, lnx);
        zero |= !(s2.len > (R)0);
        const LayV<R> ly = lay_at(T, lc.l);
        lp += (double)(ly.logb + turn_term(ly, s.u, s2.u)) + (double)seg_term(s2);
        L += (double)s2.len;
        sb += (double)s2.tb;
        ps.stw(k, s2.tb);
        s = s2;
        fc = fn;
        lc = lnx;
    }
    lp += (double)end_term(T, s.u, fc);
    if (zero) lp = -__builtin_inf();
    if (Sb) *Sb = sb;
    return lp;
}

// q(s) of the bi-spherical proposal with concentration beta, in the two
// forms the jump needs: E = e^{-2 beta}, the normaliser
// log((1 - E) / beta) = log(2 sinh(beta) / beta) - beta, and the inverse CDF
// of cos s written as w = 1 + cos s = -log(u' + (1 - u') E) / beta with
// u' = 1 - u.  For beta >= 1/4 the direct forms lose nothing (1 - E > 0.39);
// below that the expm1 / log1p forms are used.
template <class R> struct QS {
    R beta, E, ibeta, lnorm;
    bool small;
};

template <class R> __device__ __forceinline__ QS<R> make_qs(R beta) {
    QS<R> q;
    q.beta = beta;
    R ab = beta < (R)0 ? -beta : beta;
    q.small = ab < (R)0.25;
    q.E = Mth<R>::exp((R)-2 * beta);
    q.ibeta = Mth<R>::rcp(beta);
    if (!q.small) {
        q.lnorm = Mth<R>::log(((R)1 - q.E) * q.ibeta);
    } else if (ab < (R)1e-6) {
        q.lnorm = (R)0.69314718055994530942 - beta;
    } else {
        q.lnorm = Mth<R>::log(-Mth<R>::expm1((R)-2 * beta) * q.ibeta);
    }
    return q;
}

// 1 + cos s from the uniform u (inverse CDF of q(s))
template <class R> __device__ __forceinline__ R qs_sample(const QS<R>& q, R u) {
    R up = (R)1 - u;
    if (!q.small) return -Mth<R>::log(u + up * q.E) * q.ibeta;
    R ab = q.beta < (R)0 ? -q.beta : q.beta;
    if (ab < (R)1e-6) return (R)2 * up;
    return -Mth<R>::log1p(up * Mth<R>::expm1((R)-2 * q.beta)) * q.ibeta;
}

template <class R>
__device__ __forceinline__ void box_muller3(uint32_t a, uint32_t b, uint32_t c, uint32_t d, V3<R>& xi) {
    R u0 = unif<R>(a), u1 = unif<R>(b), u2 = unif<R>(c), u3 = unif<R>(d);
    R rho1 = Mth<R>::sqrt((R)-2 * Mth<R>::log(u0));
    R rho2 = Mth<R>::sqrt((R)-2 * Mth<R>::log(u2));
    xi = {rho1 * Mth<R>::cos2pi(u1), rho1 * Mth<R>::sin2pi(u1), rho2 * Mth<R>::cos2pi(u3)};
}

// ---------------------------------------------------------------------------
// Score of the path: log p and d log p / d vertex, streamed along the path
// with a three-vertex register window.  emit(k, g) receives the finished
// gradient of vertex k (k = 0 .. n-1, in increasing order).
// ---------------------------------------------------------------------------
// d tau_c / d P and d tau_c / d Q of a segment with the endpoints' layer
// points known: the mean coefficient along the segment, plus the change of
// the layers' shares where it crosses edges.
template <class R>
__device__ __forceinline__ void seg_depth_grad_lp(const Tgt<R>& T, LPt<R> P, LPt<R> Q, const Seg<R>& s, V3<R>& dP,
                                                  V3<R>& dQ) {
    R F = s.tc * Mth<R>::rcp(s.len); // mean total coefficient along the segment
    dP = (-F) * s.u;
    dQ = F * s.u;
    if (T.mcnt > 1 && P.l != Q.l) {
        double cP = (double)T.lay[P.l * LY_NW + LY_C], cQ = (double)T.lay[Q.l * LY_NW + LY_C];
        const double du = (double)Q.u - (double)P.u;
        const double inv = du != 0.0 ? 1.0 / du : 0.0;
        R gP = (R)((double)s.len * ((double)F - cP) * inv);
        R gQ = (R)((double)s.len * (cQ - (double)F) * inv);
        const V3<R> ax = T.axr;
        dP = dP + gP * ax;
        dQ = dQ + gQ * ax;
    }
}

// d log sigma / d mu at a turn, q = |ua - ub|^2
template <class R> __device__ __forceinline__ R dturn_dmu(const LayV<R>& ly, R q) {
    R den = ly.hg1 + ly.g * q;
    R dhg = (R)3 * ly.g * Mth<R>::rcp(den);
    if (ly.fsl == (R)0) return dhg;
    R hg = ly.hgn - (R)1.5 * Mth<R>::log(den);
    R v = (R)1 - (R)0.25 * q; // (1 + mu) / 2
    R sl = ly.sln + ly.sla * Mth<R>::log(v);
    R dsl = ly.sla * Mth<R>::rcp((R)2 * v);
    R m = sl > hg ? sl : hg;
    R es = ly.fsl * Mth<R>::exp(sl - m), eh = ((R)1 - ly.fsl) * Mth<R>::exp(hg - m);
    return (es * dsl + eh * dhg) * Mth<R>::rcp(es + eh);
}

template <class R> __device__ __forceinline__ V3<R> dunit(V3<R> u, R len, V3<R> c) {
    // d (u . c) / d r for u = r / |r|
    R il = Mth<R>::rcp(len);
    return il * (c - dot(u, c) * u);
}

// Role of a vertex in a local density factor (see vtx_term).
enum { VK_EMIT = 0, VK_TURN = 1, VK_END = 2, VK_NONE = 3 };

// d log p / d f_j of an interior vertex j from its five-vertex window, the
// terms the single-vertex evaluator reads: the segments A = f_{j-1} -> f_j and
// B = f_j -> f_{j+1} (attenuation and inverse square), the turn at j, the turn
// at j-1 (or, for j = 1, the emission factor, which depends on the direction
// only for a von Mises-Fisher source), and the turn at j+1 (or the end factor
// log(-u . nu) when f_{j+1} is the end point).  log b(f_j) is constant within
// a layer and contributes nothing.
template <class R>
__device__ __forceinline__ V3<R> vertex_grad(const Tgt<R>& T, int km1, const LayV<R>& lm1, V3<R> um, LPt<R> pm1,
                                             LPt<R> po, LPt<R> pp1, const Seg<R>& A, const Seg<R>& B,
                                             const LayV<R>& lo, int kp1, V3<R> up, V3<R> nu1, const LayV<R>& lp1) {
    V3<R> dPA, dQA, dPB, dQB;
    seg_depth_grad_lp(T, pm1, po, A, dPA, dQA);
    seg_depth_grad_lp(T, po, pp1, B, dPB, dQB);
    V3<R> g = ((R)2 * Mth<R>::rcp(B.len)) * B.u - ((R)2 * Mth<R>::rcp(A.len)) * A.u - dQA - dPB;
    {
        const V3<R> dd = A.u - B.u;
        const R h = dturn_dmu(lo, dot(dd, dd));
        g = g + h * (dunit(A.u, A.len, B.u) - dunit(B.u, B.len, A.u));
    }
    {
        const V3<R> dd = um - A.u;
        const R ht = dturn_dmu(lm1, dot(dd, dd));
        const R he = T.ek == RJPATH_EMIT_VMF ? T.kappa : (R)0;
        const bool turn = km1 == VK_TURN;
        g = g + (turn ? ht : he) * dunit(A.u, A.len, turn ? um : T.ed);
    }
    {
        const V3<R> dd = B.u - up;
        const R ht = dturn_dmu(lp1, dot(dd, dd));
        const R ce = -dot(B.u, nu1);
        const bool turn = kp1 == VK_TURN;
        g = g + (turn ? -ht : Mth<R>::rcp(ce)) * dunit(B.u, B.len, turn ? up : nu1);
    }
    return g;
}

// The streaming score as a walker fed one vertex at a time, so that two
// walks (the current path and a proposal generated from the first walk's
// gradients) can advance in one loop.  step(f_k) consumes vertex k >= 1 and
// returns true with the finished gradient of vertex k-2 when k >= 2;
// finish() adds the end term and returns log p, with the gradients of
// vertices n-2 and n-1.
template <class R> struct ScoreWalker {
    V3<R> gA, gB; // gradients of vertices k-2, k-1 in progress
    V3<R> fprev;
    V3<R> uprev; // direction and length of the previous segment
    R lprev;
    double lp;
    bool zero;
    int k; // next vertex to consume

    __device__ __forceinline__ void init(const Tgt<R>& T, V3<R> f0) {
        const V3<R> z = {(R)0, (R)0, (R)0};
        gA = z;
        gB = z;
        fprev = f0;
        uprev = z;
        lprev = (R)0;
        lp = 0.0;
        zero = false;
        k = 1;
    }

    __device__ __forceinline__ bool step(const Tgt<R>& T, V3<R> fcur, V3<R>& gout) {
        // (the layer point of fprev is looked up again rather than kept: two
        // walks advance together and their registers are scarce)
        const LPt<R> pprev = lpt(T, fprev), pcur = lpt(T, fcur);
        Seg<R> s = make_seg_lp(T, fprev, fcur, pprev, pcur);
        zero |= !(s.len > (R)0);
        lp += (double)seg_term(s);
        V3<R> dP, dQ;
        seg_depth_grad_lp(T, pprev, pcur, s, dP, dQ);
        R il2 = (R)2 * Mth<R>::rcp(s.len);
        gB = gB - dP + il2 * s.u;
        const V3<R> z = {(R)0, (R)0, (R)0};
        V3<R> gC = z - dQ - il2 * s.u; // vertex k
        if (k == 1) {
            lp += (double)emit_term(T, s.u);
            if (T.ek == RJPATH_EMIT_VMF) {
                V3<R> d = T.kappa * dunit(s.u, s.len, T.ed);
                gC = gC + d;
                gB = gB - d;
            }
        } else {
            // turn (and scattering density) at vertex k-1 between sprev and s
            const LayV<R> ly = lay_at(T, pprev.l);
            V3<R> dd = uprev - s.u;
            lp += (double)(ly.logb + turn_term(ly, uprev, s.u));
            R h = dturn_dmu(ly, dot(dd, dd));
            V3<R> da = dunit(uprev, lprev, s.u);
            V3<R> db = dunit(s.u, s.len, uprev);
            gA = gA - h * da;
            gB = gB + h * da - h * db;
            gC = gC + h * db;
        }
        const bool done = k >= 2;
        gout = gA;
        gA = gB;
        gB = gC;
        uprev = s.u;
        lprev = s.len;
        fprev = fcur;
        ++k;
        return done;
    }

    __device__ __forceinline__ double finish(const Tgt<R>& T, V3<R>& g_nm2, V3<R>& g_nm1) {
        // end term on segment n-2 and the end point (gA = vertex n-2, gB = vertex n-1)
        lp += (double)end_term(T, uprev, fprev);
        V3<R> d = from_eta(T, fprev);
        R dn2 = dot(d, d);
        R idn = Mth<R>::rsqrt(dn2);
        V3<R> nu = idn * d;
        R c = -dot(uprev, nu);
        R ic = Mth<R>::rcp(c);
        V3<R> dcr = (R)-1 * dunit(uprev, lprev, nu);
        V3<R> dcd = (R)-1 * dunit(nu, dn2 * idn, uprev);
        gA = gA - ic * dcr;
        gB = gB + ic * dcr + ic * dcd;
        if (T.dk == RJPATH_DET_PAPER) {
            R cr = dot(nu, T.dd);
            R th = tanh((R)2 * cr + (R)0.7);
            gB = gB + ((R)3 - (R)2 * th) * dunit(nu, dn2 * idn, T.dd);
        }
        g_nm2 = gA;
        g_nm1 = gB;
        return zero ? -__builtin_inf() : lp;
    }
};

template <class R, class P, class Emit>
__device__ __forceinline__ double score_stream(const Tgt<R>& T, const P& ps, int n, Emit emit) {
    ScoreWalker<R> w;
    w.init(T, ps.p(0));
    V3<R> g, g2;
    for (int k = 1; k < n; ++k)
        if (w.step(T, ps.p(k), g)) emit(k - 2, g);
    const double lp = w.finish(T, g, g2);
    if (n >= 3) emit(n - 2, g);
    emit(n - 1, g2);
    return lp;
}

// Per-lane constants of the step kernel.
struct StepCtx {
    uint32_t chain, k0, k1;
    int cap;
    uint32_t bthresh;
    double log_pb, log_pd; // log of the birth / death probabilities of a jump step
    double sigma, ikappa, e2k, mala_h;
    int sampler;
    const double* logw;
    uint32_t* hist; // this target's sector histogram (cap + 1 counts) or NULL
};



// log rho(nu) of the paper's angular response (0 for a uniform response)
template <class R> __device__ __forceinline__ R rho_log(const Tgt<R>& T, V3<R> nu) {
    if (T.dk != RJPATH_DET_PAPER) return (R)0;
    R cr = dot(nu, T.dd);
    R z = (R)2 * cr + (R)0.7;
    R az = z < (R)0 ? -z : z;
    // log rho = 3 c - 1 - log cosh(2 c + 0.7), log cosh z = |z| + log1p(e^{-2|z|}) - log 2
    return (R)3 * cr - (R)1 - (az + Mth<R>::log1p(Mth<R>::exp((R)-2 * az)) - (R)0.69314718055994530942);
}

// ---------------------------------------------------------------------------
// One factor of the path density attached to one vertex (App. "Path
// probability distribution"), evaluated branch-free so that lanes of a wave
// whose vertices play different roles do not diverge:
//   VK_EMIT: the source, log eps(ub) of the first direction;
//   VK_TURN: an interior vertex, log b + log sigma_sr(ua . ub);
//   VK_END:  the end point with outward sensor normal nu, log max(0, -ua . nu)
//            (the angular response log rho(nu) is added by the caller where
//            it does not cancel);
//   VK_NONE: no vertex (0).
// CE / CT / CN: whether the kinds END / EMIT / NONE can occur at the call.
// ---------------------------------------------------------------------------
template <class R, bool CE, bool CT, bool CN>
__device__ __forceinline__ R vtx_term(const Tgt<R>& T, int kind, const LayV<R>& ly, V3<R> ua, V3<R> ub, V3<R> nu) {
    V3<R> d = ua - ub;
    const R q = dot(d, d);
    R X = ly.hg1 + ly.g * q; // HG denominator, 1 - mu = |ua - ub|^2 / 2
    R ce = (R)1;
    if (CE) {
        ce = -dot(ua, nu);
        if (kind == VK_END) X = ce;
    }
    const R lx = Mth<R>::log(X);
    R out = ly.logb + ly.hgn - (R)1.5 * lx;
    if (ly.fsl != (R)0) {
        R hg = ly.hgn - (R)1.5 * lx;
        R sl = ly.sln + ly.sla * Mth<R>::log((R)1 - (R)0.25 * q);
        R m = sl > hg ? sl : hg;
        out = ly.logb + m + Mth<R>::log(ly.fsl * Mth<R>::exp(sl - m) + ((R)1 - ly.fsl) * Mth<R>::exp(hg - m));
    }
    if (CE && kind == VK_END) out = ce > (R)0 ? lx : Mth<R>::ninf();
    if (CT && kind == VK_EMIT) out = emit_term(T, ub);
    if (CN && kind == VK_NONE) out = (R)0;
    return out;
}

// The eight random words of one step: Philox4x32-10 blocks 0 and 1 of the
// counter (chain, step).
__device__ __forceinline__ void draw8(const StepCtx& sc, uint64_t step, uint32_t r[8]) {
    uint32_t q0[4] = {sc.chain, (uint32_t)step, (uint32_t)(step >> 32), 0u};
    uint32_t q1[4] = {sc.chain, (uint32_t)step, (uint32_t)(step >> 32), 1u};
    philox4x32_10(q0, sc.k0, sc.k1);
    philox4x32_10(q1, sc.k0, sc.k1);
    r[0] = q0[0]; r[1] = q0[1]; r[2] = q0[2]; r[3] = q0[3];
    r[4] = q1[0]; r[5] = q1[1]; r[6] = q1[2]; r[7] = q1[3];
}

// ---------------------------------------------------------------------------
// Per-lane sampler state and statistics.
// ---------------------------------------------------------------------------
template <class R> struct Lane {
    int n;
    bool live; // the chain steps (a malformed or zero-density chain keeps its state)
    double L;    // path length (running sum; refreshed at launch start)
    double S;    // sum of the cached segment scattering depths (running sum; refreshed at launch start)
    double lp;   // log p (refreshed at launch start and end)
    double invw; // 1 / w(n) of the sector tilt
    double lwm, lw0, lwp; // log w(n - 1), log w(n), log w(n + 1)
    // statistics of this launch.  The sums that depend on n alone are kept
    // lazily: `run` counts the counted steps spent at the current n and is
    // folded in when n changes and at the end of the launch.
    uint32_t run;
    uint32_t hrun; // steps of this launch at the current n not yet added to the sector histogram
    double a1, a2, sl, sl2;
    uint64_t sn;
    uint32_t cnt, c2, ncap, pp, pb, pd, ap, ab, ad, mp, ma;
    uint32_t ne; // jump proposals rejected without a density evaluation (birth at cap, death at n = 2)
};

// 1 / w(n) = e^{-log w(n)} of the sector tilt, a weight of the statistics
// only: FP32 chains take it from the FP32 exponential (relative error
// ~1e-6 at log w = 40, against a 1% target), FP64 chains in FP64.
template <class R> __device__ __forceinline__ double inv_tilt(double lw) {
    if constexpr (sizeof(R) == 4) return (double)Mth<float>::exp(-(float)lw);
    else return exp(-lw);
}

template <class R> __device__ __forceinline__ void fold_run(Lane<R>& ln, int n0, int cap, bool tilt) {
    const uint32_t r = ln.run;
    const bool at0 = ln.n == n0;
    ln.cnt += r;
    ln.c2 += at0 ? r : 0u;
    ln.sn += (uint64_t)r * (uint64_t)ln.n;
    ln.ncap += ln.n == cap ? r : 0u;
    if (tilt) {
        const double a = (double)r * ln.invw;
        ln.a1 += a;
        ln.a2 += at0 ? a : 0.0;
    }
    ln.run = 0;
}

// Adds the steps spent at the current n to the sector histogram.
template <class R> __device__ __forceinline__ void fold_hist(Lane<R>& ln, const StepCtx& sc) {
    if (sc.hist && ln.hrun) atomicAdd(sc.hist + ln.n, ln.hrun);
    ln.hrun = 0;
}


// One step of one lane; returns the move kind, writes log A / accepted / index.
// ---------------------------------------------------------------------------
// Tree-coordinate move of the whole path (App. "Path space coordinate
// system"; Sec. "Path proposal distribution").  Interval (k, l), l - k >= 2,
// places vertex m = (k + l) / 2 by bi-spherical coordinates (zeta, t, phi)
// about the foci f_k, f_l (cos s = tanh zeta), then splits into (k, m) and
// (m, l); the root is (0, n - 1).  The azimuth is measured in a frame handed
// down the tree: the root's is the orthonormal completion of its axis, a
// child's has e3 = the unit normal of the plane of its parent's foci and
// vertex (the parent's frame turned about the parent's axis to the parent
// vertex's azimuth, then rotated onto the child's axis) and e2 = e3 x e1.
// The move draws a von Mises-Fisher step of the end point on the sensor
// (words 4, 5, as the end-point perturbation) and Gaussian steps of variance
// mala_h / n for every (zeta, t, phi) (vertex m: one Philox block with
// counter word 3 = 2 + m), builds the proposal node by node in pre-order (each
// vertex's foci and frame come from vertices placed before it) into the work
// buffer, and accepts with
//   log A = log p(y) - log p(x) + sum_m [log J_m(y) - log J_m(x)],
//   J_m = gamma^3 sech^2(zeta) / (cosh t - tanh zeta)^3.
// The coordinates are formed from unit vectors: with uA, uB the unit vectors
// from f_m to its foci, 1 + cos s = |uA + uB|^2 / 2, 1 - cos s = |uA - uB|^2 / 2
// and sin s = |uA + uB| |uA - uB| / 2, which keep their precision for nearly
// straight (s ~ pi) and nearly folded paths.
// ---------------------------------------------------------------------------
template <class R> struct TreePath {
    // the proposal: vertex 0 from the path, interior vertices from the work
    // buffer, the end point held apart
    GlobalPath<R> work;
    V3<R> y0, yend;
    int n;
    __device__ __forceinline__ V3<R> p(int v) const {
        // (selected per component: a choice between whole vectors would go
        // through the stack)
        const V3<R> g = work.p(v);
        const bool s0 = v == 0, se = v == n - 1;
        return {s0 ? y0.x : (se ? yend.x : g.x), s0 ? y0.y : (se ? yend.y : g.y), s0 ? y0.z : (se ? yend.z : g.z)};
    }
    // the y walk's segment depths are kept in the work buffer (slot v: the
    // segment leaving vertex v) for the copy-back on acceptance
    __device__ __forceinline__ void stw(int v, R x) const { work.glb[(size_t)v * work.C].w = x; }
};

// frame (e2, e3) of interval (k, l) of a path: root -> onb of the axis;
// otherwise from the parent interval (kp, lp) and its vertex fp.  Both are
// formed and one is selected by value (a choice between output references
// would become a dynamically indexed stack slot).
template <class R> struct Frame2 {
    V3<R> e2, e3;
};

template <class R>
__device__ __forceinline__ Frame2<R> tree_frame(bool root, V3<R> e1, V3<R> fkp, V3<R> flp, V3<R> fp) {
    V3<R> r2, r3;
    onb(e1, r2, r3);
    const V3<R> ep = unit_dir(fkp, flp);
    const V3<R> g = fp - fkp;
    const V3<R> c = {ep.y * g.z - ep.z * g.y, ep.z * g.x - ep.x * g.z, ep.x * g.y - ep.y * g.x};
    const V3<R> c3 = Mth<R>::rsqrt(dot(c, c)) * c;
    const V3<R> c2 = {c3.y * e1.z - c3.z * e1.y, c3.z * e1.x - c3.x * e1.z, c3.x * e1.y - c3.y * e1.x};
    Frame2<R> f;
    f.e2 = {root ? r2.x : c2.x, root ? r2.y : c2.y, root ? r2.z : c2.z};
    f.e3 = {root ? r3.x : c3.x, root ? r3.y : c3.y, root ? r3.z : c3.z};
    return f;
}

template <class R, bool LO>
__device__ __forceinline__ void tree_move(const Tgt<R>& T, const PathRef<R, LO>& ps, const GlobalPath<R>& work,
                                          Lane<R>& ln, const StepCtx& sc, uint64_t step, const uint32_t r[8],
                                          R logu, int& accepted, R& logA) {
    const int n = ln.n;
    const V3<R> x0 = ps.p(0), xe = ps.p(n - 1);
    // end point: von Mises-Fisher step about the current sensor normal
    V3<R> yend;
    {
        const R u4 = unif<R>(r[4]), u5 = unif<R>(r[5]);
        const R lg = Mth<R>::log(u4 + ((R)1 - u4) * (R)sc.e2k);
        const V3<R> dd = from_eta(T, xe);
        const V3<R> nu = Mth<R>::rsqrt(dot(dd, dd)) * dd;
        V3<R> e2, e3;
        onb(nu, e2, e3);
        const R omw = -lg * (R)sc.ikappa;
        const R sw = Mth<R>::sqrt(fmax(omw * ((R)2 - omw), (R)0));
        const V3<R> nn = ((R)1 - omw) * nu + sw * (Mth<R>::cos2pi(u5) * e2 + Mth<R>::sin2pi(u5) * e3);
        yend = T.eta + (T.eta_lo + T.rad * nn);
    }
    auto xat = [&](int v) __attribute__((always_inline)) { return ps.p(v); };
    const TreePath<R> yp{work, x0, yend, n};
    auto yat = [&](int v) __attribute__((always_inline)) { return yp.p(v); };
    const R sig = Mth<R>::sqrt((R)sc.mala_h / (R)n);
    double lj = 0.0; // sum of log J(y) - log J(x)
    bool ok = true;
    // Nodes in pre-order (a node before its subtrees, so every vertex's foci
    // and frame are placed before it): node i is found by descending from the
    // root, skipping whole left subtrees by their vertex count.  A lane visits
    // its n - 2 nodes only.
    for (int i = 0; i < n - 2; ++i) {
        {
            int k = 0, l = n - 1, kp = 0, lp = n - 1, left = i;
            bool root = true;
            for (;;) {
                const int mid = (k + l) >> 1;
                if (left == 0) break;
                left -= 1; // the node itself
                kp = k;
                lp = l;
                root = false;
                if (left < mid - k - 1) {
                    l = mid;
                } else {
                    left -= mid - k - 1;
                    k = mid;
                }
            }
            const int m = (k + l) >> 1, pm = (kp + lp) >> 1;
            // current coordinates of x_m
            const V3<R> xk = xat(k), xl = xat(l), xm = xat(m);
            const V3<R> rx = xl - xk;
            const R gx = (R)0.5 * Mth<R>::sqrt(dot(rx, rx));
            const V3<R> e1x = ((R)0.5 * Mth<R>::rcp(gx)) * rx;
            const Frame2<R> fx = tree_frame(root, e1x, xat(kp), xat(lp), xat(pm));
            const V3<R> e2x = fx.e2, e3x = fx.e3;
            const V3<R> va = xk - xm, vb = xl - xm;
            const R dA = Mth<R>::sqrt(dot(va, va)), dB = Mth<R>::sqrt(dot(vb, vb));
            const V3<R> ua = Mth<R>::rcp(dA) * va, ub = Mth<R>::rcp(dB) * vb;
            const V3<R> sp = ua + ub, sm = ua - ub;
            const R np2 = dot(sp, sp), nm2 = dot(sm, sm);
            const R zeta = (R)0.5 * Mth<R>::log(np2 * Mth<R>::rcp(nm2));
            const R tt = Mth<R>::log(dA * Mth<R>::rcp(dB));
            const V3<R> q = xm - (R)0.5 * (xk + xl);
            const R phi = atan2(dot(q, e3x), dot(q, e2x));
            // log J(x): sech zeta = sin s, cosh t - tanh zeta = (dA - dB)^2 / (2 dA dB) + (1 - cos s)
            const R dd = dA - dB;
            const R denx = dd * dd * Mth<R>::rcp((R)2 * dA * dB) + (R)0.5 * nm2;
            lj -= (double)((R)3 * Mth<R>::log(gx) + Mth<R>::log((R)0.25 * np2 * nm2) - (R)3 * Mth<R>::log(denx));
            // proposed coordinates
            uint32_t qd[4] = {sc.chain, (uint32_t)step, (uint32_t)(step >> 32), 2u + (uint32_t)m};
            philox4x32_10(qd, sc.k0, sc.k1);
            V3<R> xi;
            box_muller3<R>(qd[0], qd[1], qd[2], qd[3], xi);
            const R z2 = zeta + sig * xi.x, t2 = tt + sig * xi.y, p2 = phi + sig * xi.z;
            // y_m from its (already placed) foci and frame
            const V3<R> yk = yat(k), yl = yat(l);
            const V3<R> ry = yl - yk;
            const R gy = (R)0.5 * Mth<R>::sqrt(dot(ry, ry));
            const V3<R> e1y = ((R)0.5 * Mth<R>::rcp(gy)) * ry;
            const Frame2<R> fy = tree_frame(root, e1y, yat(kp), yat(lp), yat(pm));
            const V3<R> e2y = fy.e2, e3y = fy.e3;
            // tanh and sech of zeta and cosh t - tanh zeta without cancellation
            const R az = fabs(z2);
            const R ez = Mth<R>::exp((R)-2 * az);
            const R th = copysign(((R)1 - ez) * Mth<R>::rcp((R)1 + ez), z2);
            const R sh = (R)2 * Mth<R>::sqrt(ez) * Mth<R>::rcp((R)1 + ez);
            const R et = Mth<R>::exp(t2), iet = Mth<R>::rcp(et);
            const R sht = (R)0.5 * (et - iet);
            const R s2h = sht * sht * Mth<R>::rcp((R)0.5 * (et + iet) + (R)1); // cosh t - 1 = sinh^2 t / (cosh t + 1)
            const R omt = z2 > (R)0 ? (R)2 * ez * Mth<R>::rcp((R)1 + ez) : (R)1 - th; // 1 - tanh zeta
            const R deny = s2h + omt;
            const V3<R> dir = sht * e1y + sh * (Mth<R>::cos2pi(p2 * (R)0.15915494309189534) * e2y +
                                                Mth<R>::sin2pi(p2 * (R)0.15915494309189534) * e3y);
            const V3<R> ym = (R)0.5 * (yk + yl) + (gy * Mth<R>::rcp(deny)) * dir;
            lj += (double)((R)3 * Mth<R>::log(gy) + (R)2 * Mth<R>::log(sh) - (R)3 * Mth<R>::log(deny));
            ok = ok && isfinite(ym.x) && isfinite(ym.y) && isfinite(ym.z);
            work.glb[(size_t)m * work.C] = Vtx<R>{ym.x, ym.y, ym.z, (R)0};
        }
    }
    double Lx, Ly = 0.0, Sy = 0.0;
    const double lpx = full_logp(T, ps, n, Lx);
    const double lpy = ok ? full_logp(T, yp, n, Ly, &Sy) : -__builtin_inf();
    const double la = lpy - lpx + lj;
    logA = isfinite(lpy) && isfinite(la) ? (R)la : Mth<R>::ninf();
    if (logu < logA) {
        accepted = 1;
        // the proposal with the depths its walk left in the work buffer
        for (int k = 1; k <= n - 2; ++k) ps.st(k, work.ld(k));
        ps.stw(0, work.ld(0).w);
        ps.st(n - 1, Vtx<R>{yend.x, yend.y, yend.z, (R)0});
        ln.L = Ly;
        ln.S = Sy;
    }
}

template <class R, bool LO, int SAMP>
__device__ __forceinline__ void step_body(const Tgt<R>& T, const PathRef<R, LO>& ps, const GlobalPath<R>& work,
                                          Lane<R>& ln, const StepCtx& sc, uint64_t step, bool perturb, bool tree,
                                          int& move, int& idx, int& accepted, R& logA, R& logu) {
    uint32_t r[8];
    draw8(sc, step, r);
    const int n = ln.n;
    // (a chain that is not live rejects every proposal)
    logu = ln.live ? Mth<R>::log(unif<R>(r[1])) : -Mth<R>::ninf();
    move = MV_NULL;
    idx = -1;
    accepted = 0;
    logA = Mth<R>::ninf();
    const V3<R> ex = {(R)1, (R)0, (R)0};
    if constexpr (SAMP == SAMP_TREE) {
        if (tree) {
            move = MV_TREE;
            tree_move<R, LO>(T, ps, work, ln, sc, step, r, logu, accepted, logA);
            return;
        }
    }
    if (perturb) {
        const int j = 1 + pick(r[0], (uint32_t)(n - 1));
        idx = j;
        const bool is_end = (j == n - 1);
        constexpr bool MALA = SAMP == SAMP_JOINT;
        if (MALA && !is_end) {
            // ---------- joint Langevin move of all interior vertices ----------
            move = MV_MALA;
            const R h = (R)sc.mala_h, hh = (R)0.5 * h, sh = Mth<R>::sqrt(h);
            // One loop walks the current path x and the proposal y together:
            // the walk over x finishes the gradient of vertex k, which gives
            // y_k, which the walk over y consumes at once (it finishes the
            // gradient of y_{k-2}).  y goes to the work buffer only for the
            // copy-back on acceptance.
            double half_xi2 = 0.0, rev = 0.0;
            ScoreWalker<R> wx, wy;
            const V3<R> x0 = ps.p(0);
            wx.init(T, x0);
            wy.init(T, x0);
            // y_k, y_{k-1}, y_{k-2} of the last vertex k fed to the y walk, kept
            // as scalars so that the ring stays in registers
            R y0x = x0.x, y0y = x0.y, y0z = x0.z, y1x = x0.x, y1y = x0.y, y1z = x0.z;
            R y2x = x0.x, y2y = x0.y, y2z = x0.z;
            // y_k from the gradient of x at vertex k (interior: Langevin step)
            auto make_y = [&](int k, V3<R> g) __attribute__((always_inline)) {
                V3<R> y = ps.p(k);
                if (k >= 1 && k <= n - 2) {
                    uint32_t q[4] = {sc.chain, (uint32_t)step, (uint32_t)(step >> 32), 2u + (uint32_t)k};
                    philox4x32_10(q, sc.k0, sc.k1);
                    V3<R> xi;
                    box_muller3<R>(q[0], q[1], q[2], q[3], xi);
                    half_xi2 += 0.5 * (double)dot(xi, xi);
                    y = y + hh * g + sh * xi;
                    work.glb[(size_t)k * work.C] = Vtx<R>{y.x, y.y, y.z, (R)0};
                }
                return y;
            };
            // the reverse-proposal term of vertex k from the gradient of y there
            auto rev_term = [&](int k, V3<R> g, V3<R> yk) __attribute__((always_inline)) {
                if (k >= 1 && k <= n - 2) {
                    V3<R> d = ps.p(k) - yk - hh * g;
                    rev += (double)dot(d, d) / (2.0 * (double)h);
                }
            };
            auto feed_y = [&](V3<R> y) __attribute__((always_inline)) {
                y2x = y1x;
                y2y = y1y;
                y2z = y1z;
                y1x = y0x;
                y1y = y0y;
                y1z = y0z;
                y0x = y.x;
                y0y = y.y;
                y0z = y.z;
                const int ky = wy.k;
                V3<R> gy;
                if (wy.step(T, y, gy)) rev_term(ky - 2, gy, V3<R>{y2x, y2y, y2z});
            };
            V3<R> g, g2;
            for (int k = 1; k < n; ++k) {
                if (wx.step(T, ps.p(k), g) && k >= 3) feed_y(make_y(k - 2, g));
            }
            // (vertex 0 never moves; its gradient is not needed)
            const double lpx = wx.finish(T, g, g2);
            if (n >= 3) feed_y(make_y(n - 2, g));
            feed_y(make_y(n - 1, g2));
            const double lpy = wy.finish(T, g, g2);
            if (n >= 3) rev_term(n - 2, g, V3<R>{y1x, y1y, y1z});
            double la = lpy - lpx - rev + half_xi2;
            logA = isfinite(lpy) ? (R)la : Mth<R>::ninf();
            if (logu < logA) {
                accepted = 1;
                for (int k = 1; k <= n - 2; ++k) ps.st(k, work.ld(k));
                full_logp(T, ps, n, ln.L, &ln.S); // refresh the cached depths, L and S
            }
            return;
        }
        // ---------- single-vertex perturbation: the five-vertex window ----------
        const bool hm2 = j >= 2, hp1 = !is_end, hp2 = j <= n - 3;
        // slots j-2 .. j+2 (absent neighbours are replaced by stand-ins below;
        // in LDS their slots are readable as they are, elsewhere the indices
        // are clamped to stay in range)
        Vtx<R> wm2, vm1, vo, wp1, wp2;
        ps.ld5(LO || hm2 ? j - 2 : 0, j - 1, j, LO || hp1 ? j + 1 : 0, LO || hp2 ? j + 2 : 0, wm2, vm1, vo, wp1, wp2);
        const V3<R> gm2 = pos(wm2), fm1 = pos(vm1), fo = pos(vo);
        const V3<R> gp1 = pos(wp1), gp2 = pos(wp2);
        const V3<R> fm2 = hm2 ? gm2 : fm1 - ex;
        const V3<R> fp1 = hp1 ? gp1 : fo + ex;
        const V3<R> fp2 = hp2 ? gp2 : fp1 + ex;
        move = is_end ? MV_END : MV_INTERIOR;
        // layer points of the window vertices, once each; the ones near an
        // edge are settled together with the proposal's (one branch per
        // step), except that the Langevin step needs the old window first
        constexpr bool EARLY = SAMP == SAMP_LOCAL;
        bool q1, q2, q3, q4;
        LPt<R> pm1 = lpt_fast(T, fm1, q1), po = lpt_fast(T, fo, q2), pp1 = lpt_fast(T, fp1, q3);
        if constexpr (EARLY) {
            if (q1 | q2 | q3) {
                lpt_settle(T, fm1, pm1);
                lpt_settle(T, fo, po);
                lpt_settle(T, fp1, pp1);
            }
        }
        Seg<R> Ao, Bo;
        LayV<R> lm1, lo, lp1;
        auto old_window = [&]() __attribute__((always_inline)) {
            Ao = make_seg_lp(T, fm1, fo, pm1, po);
            Bo = make_seg_lp(T, fo, fp1, po, pp1);
            lm1 = lay_at(T, pm1.l);
            lo = lay_at(T, po.l);
            lp1 = lay_at(T, pp1.l);
        };
        if constexpr (EARLY) old_window();
        const V3<R> um = unit_dir(fm2, fm1), up = unit_dir(fp1, fp2), nu1 = unit_dir_eta(T, fp1);
        const int km1 = hm2 ? VK_TURN : VK_EMIT;
        const int kj = is_end ? VK_END : VK_TURN;
        const int kp1 = !hp1 ? VK_NONE : (hp2 ? VK_TURN : VK_END);
        // one log and one sin/cos pair serve both proposals: Box-Muller on
        // words 4..7 for the Gaussian step, and words 4, 5 for the end-point
        // von Mises-Fisher step (inverse CDF of its cosine, uniform azimuth)
        const R u4 = unif<R>(r[4]), u5 = unif<R>(r[5]);
        const R lg = Mth<R>::log(is_end ? u4 + ((R)1 - u4) * (R)sc.e2k : u4);
        const R c5 = Mth<R>::cos2pi(u5), s5 = Mth<R>::sin2pi(u5);
        V3<R> fn, nu, nn;
        R hx = (R)0, half_xi2 = (R)0;
        {
            const R rho1 = Mth<R>::sqrt((R)-2 * lg);
            const R rho2 = Mth<R>::sqrt((R)-2 * Mth<R>::log(unif<R>(r[6])));
            const V3<R> xi = {rho1 * c5, rho1 * s5, rho2 * Mth<R>::cos2pi(unif<R>(r[7]))};
            V3<R> fg;
            if constexpr (SAMP == SAMP_LOCAL) {
                // single-vertex Langevin step with h = mala_h * (shorter adjacent segment)^2
                const V3<R> gx = vertex_grad(T, km1, lm1, um, pm1, po, pp1, Ao, Bo, lo, kp1, up, nu1, lp1);
                const R m = fmin(Ao.len, Bo.len);
                hx = (R)sc.mala_h * m * m;
                half_xi2 = (R)0.5 * dot(xi, xi);
                fg = fo + ((R)0.5 * hx) * gx + Mth<R>::sqrt(hx) * xi;
            } else {
                fg = fo + (R)sc.sigma * xi;
            }
            V3<R> dd = from_eta(T, fo), e2, e3;
            nu = Mth<R>::rsqrt(dot(dd, dd)) * dd; // sensor normal at the current end point
            onb(nu, e2, e3);
            const R omw = -lg * (R)sc.ikappa; // 1 - cos
            const R wv = (R)1 - omw;
            const R sw = Mth<R>::sqrt(fmax(omw * ((R)2 - omw), (R)0));
            nn = wv * nu + sw * (c5 * e2 + s5 * e3); // sensor normal at the proposed end point
            fn = is_end ? T.eta + (T.eta_lo + T.rad * nn) : fg;
        }
        LPt<R> pn = lpt_fast(T, fn, q4);
        if constexpr (EARLY) {
            if (q4) lpt_settle(T, fn, pn);
        } else {
            if (q1 | q2 | q3 | q4) {
                lpt_settle(T, fm1, pm1);
                lpt_settle(T, fo, po);
                lpt_settle(T, fp1, pp1);
                lpt_settle(T, fn, pn);
            }
            old_window();
        }
        const Seg<R> An = make_seg_lp(T, fm1, fn, pm1, pn), Bn = make_seg_lp(T, fn, fp1, pn, pp1);
        const LayV<R> lnw = lay_at(T, pn.l);
        R d = seg_term(An) - seg_term(Ao);
        d += hp1 ? seg_term(Bn) - seg_term(Bo) : (R)0;
        d += vtx_term<R, false, true, false>(T, km1, lm1, um, An.u, nu1) -
             vtx_term<R, false, true, false>(T, km1, lm1, um, Ao.u, nu1);
        d += vtx_term<R, true, false, false>(T, kj, lnw, An.u, Bn.u, nn) -
             vtx_term<R, true, false, false>(T, kj, lo, Ao.u, Bo.u, nu);
        d += vtx_term<R, true, false, true>(T, kp1, lp1, Bn.u, up, nu1) -
             vtx_term<R, true, false, true>(T, kp1, lp1, Bo.u, up, nu1);
        if constexpr (SAMP == SAMP_LOCAL) {
            // log q(x | y) - log q(y | x) of the two Gaussian proposals, each
            // with its own step size (so the normalisations h^{-3/2} enter)
            const V3<R> gy = vertex_grad(T, km1, lm1, um, pm1, pn, pp1, An, Bn, lnw, kp1, up, nu1, lp1);
            const R m = fmin(An.len, Bn.len);
            const R hy = (R)sc.mala_h * m * m;
            const V3<R> b = (fo - fn) - ((R)0.5 * hy) * gy;
            const R lq = (R)1.5 * Mth<R>::log(hx * Mth<R>::rcp(hy)) - dot(b, b) * Mth<R>::rcp((R)2 * hy) + half_xi2;
            d += is_end ? (R)0 : lq;
            move = is_end ? MV_END : MV_LMALA;
        }
        // the angular response changes only when the end point itself moves
        if (T.dk == RJPATH_DET_PAPER && is_end) d += rho_log(T, nn) - rho_log(T, nu);
        logA = d;
        if (logu < logA) {
            accepted = 1;
            ps.st(j, Vtx<R>{fn.x, fn.y, fn.z, hp1 ? Bn.tb : (R)0});
            ps.stw(j - 1, An.tb);
            ln.L += (double)An.len - (double)Ao.len + (hp1 ? (double)Bn.len - (double)Bo.len : 0.0);
            ln.S += ((double)An.tb - (double)vm1.w) + (hp1 ? (double)Bn.tb - (double)vo.w : 0.0);
        }
        return;
    }
    // ---------- birth / death through the bi-spherical map ----------
    const bool birth = r[2] < sc.bthresh;
    move = birth ? MV_BIRTH : MV_DEATH;
    // S = sum of the cached segment depths, kept by the lane as a running sum
    // (summed afresh in path order at every launch start and after whole-path
    // moves).  The segment scan of a birth reads the first WB depths once into
    // registers (loads issued together) and the rest four at a time.
    // (16 cover all but rare long paths of the batched workloads; the FP64
    // and Langevin variants keep 8 so that their registers still allow two
    // resident waves per SIMD where they did)
    constexpr int WB = (sizeof(R) == 4 && SAMP == SAMP_PLAIN) ? 16 : 8;
    const double S = ln.S;
    const bool valid = birth ? (n < sc.cap && S > 0.0) : (n > 2);
    int iA = 0, jv = 1;
    if (valid) {
        if (birth) {
            // segment k with probability tau_b(k) / S: the first k whose
            // cumulative depth exceeds U S, i.e. the number of prefixes that
            // do not (the cumulative sums never decrease)
            const double tgt = (double)unif<double>(r[0]) * S;
            R wv[WB];
#pragma unroll
            for (int v = 0; v < WB; ++v) wv[v] = ps.w(v < n - 1 ? v : 0);
            double cum = 0.0;
            int k = 0;
            // (past the path the cumulative sum stays at S > U S: no count;
            // once it exceeds U S no later prefix counts either)
#pragma unroll
            for (int v = 0; v < WB; ++v) {
                cum += v < n - 1 ? (double)wv[v] : 0.0;
                k += cum <= tgt ? 1 : 0;
            }
            for (int v = WB; v < n - 1 && cum <= tgt; v += 4) {
                R w4[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) w4[i] = ps.w(v + i < n - 1 ? v + i : v);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    cum += v + i < n - 1 ? (double)w4[i] : 0.0;
                    k += cum <= tgt ? 1 : 0;
                }
            }
            k = k < n - 2 ? k : n - 2;
            iA = k;
        } else {
            jv = 1 + pick(r[0], (uint32_t)(n - 2));
            iA = jv - 1;
        }
        idx = birth ? iA : jv;
    }
    const int iB = birth ? iA + 1 : iA + 2;
    const bool hprev = iA >= 1, hnext = iB + 1 <= n - 1;
    V3<R> A, B, gprev, gnext, fj;
    R wA, wj; // cached depths of segments iA and jv (jv's is used by a death)
    if (LO) {
        // slots iA-1 .. iA+3, read as they are (padding makes all readable)
        const Vtx<R> s1 = ps.ld(iA), s2 = ps.ld(iA + 1);
        const V3<R> s0 = ps.p(iA - 1), s3 = ps.p(iA + 2), s4 = ps.p(iA + 3);
        gprev = s0;
        A = pos(s1);
        fj = pos(s2); // jv = iA + 1 for a death (unused by a birth)
        wA = s1.w;
        wj = s2.w;
        B = birth ? pos(s2) : s3;
        gnext = birth ? s3 : s4;
    } else {
        Vtx<R> vA, vj, vB, vp, vn;
        ps.ld5(iA, jv, iB < n ? iB : n - 1, hprev ? iA - 1 : 0, hnext ? iB + 1 : 0, vA, vj, vB, vp, vn);
        A = pos(vA);
        wA = vA.w;
        B = pos(vB);
        gprev = pos(vp);
        gnext = pos(vn);
        fj = pos(vj);
        wj = vj.w;
    }
    const V3<R> fprev = hprev ? gprev : A - ex;
    const V3<R> fnext = hnext ? gnext : B + ex;
    const V3<R> mid = (R)0.5 * (A + B);
    bool q1, q2, q3;
    LPt<R> pA = lpt_fast(T, A, q1), pB = lpt_fast(T, B, q2), pmid = lpt_fast(T, mid, q3);
    if (q1 | q2 | q3) {
        lpt_settle(T, A, pA);
        lpt_settle(T, B, pB);
        lpt_settle(T, mid, pmid);
    }
    const Seg<R> AB = make_seg_lp(T, A, B, pA, pB);
    const LayV<R> lm = lay_at(T, pmid.l);
    const R gam = (R)0.5 * AB.len;
    const R beta = lm.keq + (R)0.5 * (gam * lm.b - (R)1); // centering rule at the midpoint
    const QS<R> qs = make_qs(beta);
    V3<R> fv;
    {
        // the bi-spherical proposal (used by births; deaths take the vertex itself)
        R w = qs_sample(qs, unif<R>(r[4])); // 1 + cos s by the inverse CDF of q(s)
        // t from the logistic q(t): e^t = a/(1-a); sinh t and cosh t - cos s in closed form
        R a5 = unif<R>(r[5]), b5 = (R)1 - a5, ab2 = (R)2 * a5 * b5;
        R ss = Mth<R>::sqrt(fmax(w * ((R)2 - w), (R)0));
        R ph = unif<R>(r[6]);
        V3<R> e2, e3;
        onb(AB.u, e2, e3);
        R sc_ = gam * Mth<R>::rcp((R)1 - ab2 * w);
        V3<R> tr = Mth<R>::cos2pi(ph) * e2 + Mth<R>::sin2pi(ph) * e3;
        const V3<R> fb = mid + sc_ * ((a5 - b5) * AB.u + (ab2 * ss) * tr);
        fv = birth ? fb : fj;
    }
    const LPt<R> pv = lpt(T, fv);
    const Seg<R> sA = make_seg_lp(T, A, fv, pA, pv), sB = make_seg_lp(T, fv, B, pv, pB);
    const V3<R> up = unit_dir(fprev, A), un = unit_dir(B, fnext), nuB = unit_dir_eta(T, B);
    const LayV<R> la = lay_at(T, pA.l), lb = lay_at(T, pB.l), lv = lay_at(T, pv.l);
    const int kA = hprev ? VK_TURN : VK_EMIT, kB = hnext ? VK_TURN : VK_END;
    // (an end point B is the same in x and y: its angular response cancels)
    const R tx = vtx_term<R, false, true, false>(T, kA, la, up, AB.u, nuB) +
                 vtx_term<R, true, false, false>(T, kB, lb, AB.u, un, nuB);
    const R ty = vtx_term<R, false, true, false>(T, kA, la, up, sA.u, nuB) +
                 vtx_term<R, true, false, false>(T, kB, lb, sB.u, un, nuB) +
                 vtx_term<R, false, false, false>(T, VK_TURN, lv, sA.u, sB.u, nuB);
    V3<R> dq = sA.u - sB.u;
    R q = dot(dq, dq);
    // segment factors of y over x times |J| / q(s) q(t) q(phi): the inverse-square
    // factors of the two new segments cancel against J; 1 + cos s = q / 2
    const R LOG2PI = (R)1.83787706640934548356;
    R jac = -sA.tc - sB.tc + AB.tc + (R)2 * Mth<R>::log(sA.len + sB.len) - AB.loglen + qs.lnorm +
            (R)0.5 * beta * q + LOG2PI;
    const int nx = birth ? n : n - 1;
    const double Sx = birth ? S : S - (double)wA - (double)wj + (double)AB.tb;
    R lpup = (R)sc.log_pb + Mth<R>::log(AB.tb) - Mth<R>::log((R)Sx);
    R lpdn = (R)sc.log_pd - Mth<R>::log((R)(nx - 1));
    // logw[nx + 1] - logw[nx] (both differences formed first: a choice between
    // the loads would become a dynamically indexed stack slot)
    const double dlw_b = ln.lwp - ln.lw0, dlw_d = ln.lw0 - ln.lwm;
    R dlw = (sc.logw && valid) ? (R)(birth ? dlw_b : dlw_d) : (R)0;
    R logAb = (ty - tx) + jac + dlw + lpdn - lpup;
    logA = valid ? (birth ? logAb : -logAb) : Mth<R>::ninf();
    if (logu < logA) {
        accepted = 1;
        fold_run(ln, T.n0, sc.cap, sc.logw != nullptr); // the steps spent at the old n
        fold_hist(ln, sc);
        const double dL = (double)sA.len + (double)sB.len - (double)AB.len;
        if (birth) {
            ps.shift_up(iB, n - 1);
            ps.st(iB, Vtx<R>{fv.x, fv.y, fv.z, sB.tb});
            ps.stw(iA, sA.tb);
            ln.L += dL;
            ln.S = (S - (double)wA) + ((double)sA.tb + (double)sB.tb);
            ln.n = n + 1;
            if (sc.logw) {
                ln.lwm = ln.lw0;
                ln.lw0 = ln.lwp;
                ln.lwp = sc.logw[n + 2 <= sc.cap ? n + 2 : sc.cap];
            }
        } else {
            ps.shift_down(jv, n - 2);
            ps.stw(iA, AB.tb);
            ln.L -= dL;
            ln.S = Sx;
            ln.n = n - 1;
            if (sc.logw) {
                ln.lwp = ln.lw0;
                ln.lw0 = ln.lwm;
                ln.lwm = sc.logw[n - 2];
            }
        }
        if (sc.logw) ln.invw = inv_tilt<R>(ln.lw0);
    }
}

// One sampler step of a lane inside the step loop: the move, then the move
// counts, the per-step sums, the optional histogram and trace.
template <class R, bool LO, int SAMP>
__device__ __forceinline__ void one_step(const KArgs& a, const Tgt<R>& T, const PathRef<R, LO>& ps,
                                         const GlobalPath<R>& work, Lane<R>& ln, const StepCtx& sc, uint64_t step0,
                                         int s, int& phase, int c, int t) {
    const uint64_t step = step0 + (uint64_t)s;
    const bool perturb = phase < a.n_perturb;
    int move, idx, accepted;
    R logA, logu;
    const bool counted = (int64_t)step >= a.burn_in;
    // the tree sampler makes the first step of every cycle a tree-coordinate move
    const bool tree = SAMP == SAMP_TREE && phase == 0 && perturb;
    step_body<R, LO, SAMP>(T, ps, work, ln, sc, step, perturb, tree, move, idx, accepted, logA, logu);
    {
        // move counts, branch-free (per-branch updates get merged by the
        // compiler into a dynamically indexed stack slot)
        const uint32_t cu = counted ? 1u : 0u, ca = (uint32_t)accepted;
        const uint32_t ib = cu & (move == MV_BIRTH ? 1u : 0u), id = cu & (move == MV_DEATH ? 1u : 0u);
        const uint32_t ip = cu - ib - id, im = cu & ((move == MV_MALA || move == MV_LMALA || move == MV_TREE) ? 1u : 0u);
        ln.ne += cu & (((move == MV_BIRTH || move == MV_DEATH) && idx < 0) ? 1u : 0u);
        ln.pb += ib;
        ln.pd += id;
        ln.pp += ip;
        ln.mp += im;
        ln.ab += ib & ca;
        ln.ad += id & ca;
        ln.ap += ip & ca;
        ln.ma += im & ca;
    }
    if (counted) {
        ln.run += 1;
        ln.sl += ln.L;
        ln.sl2 += ln.L * ln.L;
    }
    ln.hrun += 1;
    if (a.trace && ln.live) {
        double* tr = a.trace + ((size_t)c * a.trace_steps + a.trace_off + s) * RJPATH_TRACE_WORDS;
        tr[0] = move;
        tr[1] = accepted;
        tr[2] = idx;
        tr[3] = (double)logA;
        tr[4] = (double)logu;
    }
    phase = (phase + 1 == a.cycle_len) ? 0 : phase + 1;
}

// ---------------------------------------------------------------------------
// The step kernel.  MK: MK_HOM (every medium of the launch is homogeneous: the
// layer lookups fold away), MK_LAY (layer tables read from HBM) or MK_LAY_LDS
// (tables staged in LDS).  SL: some layer mixes in the Rayleigh-like term.
// ---------------------------------------------------------------------------
enum { MK_HOM = 0, MK_LAY = 1, MK_LAY_LDS = 2 };

template <class R, int MK, int SAMP, bool SL>
__global__ void __launch_bounds__(256) run_kernel(KArgs a) {
    constexpr bool TAB = MK == MK_LAY_LDS;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, bs = blockDim.x;
    MedTab<R> tab = hbm_tab<R>(a);
    size_t tab_bytes = 0;
    if (TAB) {
        // layer table, then edges, then prefix integrals, each 16-byte aligned
        const size_t nl = (size_t)a.L_total * LY_NW, ne = (size_t)a.n_edges;
        R* lay = (R*)smem;
        double* edge = (double*)(smem + ((nl * sizeof(R) + 15) & ~(size_t)15));
        double* pre = edge + ((ne + 1) & ~(size_t)1);
        for (size_t i = tid; i < nl; i += bs) lay[i] = ((const R*)a.lay)[i];
        for (size_t i = tid; i < ne; i += bs) edge[i] = a.edge[i];
        for (size_t i = tid; i < 2 * ne; i += bs) pre[i] = a.pre[i];
        __syncthreads();
        tab = MedTab<R>{lay, edge, pre};
        tab_bytes = a.tab_bytes;
    }
    const int c = blockIdx.x * bs + tid;
    if (c >= a.C) return;
    const size_t C = (size_t)a.C;
    // this wave's tile, past its leading padding slot
    LdsPtr<R> lslots = (LdsPtr<R>)((L4<R>*)(smem + tab_bytes) + (size_t)(tid / WAVE) * (a.V + SLOT_PAD) * WAVE +
                                   WAVE + tid % WAVE);
    const int t = a.target[c];
    Lane<R> ln{};
    ln.n = a.n[c];
    const int cap = a.cap;
    // malformed chains are flagged and never touched
    if (t < 0 || t >= a.T || ln.n < 2 || ln.n > cap || a.medium[t] < 0 || a.medium[t] >= a.n_media) {
        a.status[c] = 1;
        return;
    }
    Tgt<R> T;
    load_target(a, t, T, tab);
    // compile-time facts of this instantiation (the lookups that test them fold)
    if (MK == MK_HOM) T.mcnt = 1;
    T.sl = SL;
    if (!SL) T.l0.fsl = (R)0;
    PathRef<R, false> ps{lslots, (Vtx<R>*)a.verts + c, a.V, C};
    PathRef<R, true> pl{lslots, (Vtx<R>*)a.verts + c, a.V, C};
    GlobalPath<R> work{a.work ? (Vtx<R>*)a.work + c : nullptr, C};
    // stage the LDS part of the path
    const int nl0 = ln.n < a.V ? ln.n : a.V;
    for (int v = 0; v < nl0; ++v) lds_st<R>(ps.lds + v * WAVE, ps.glb[(size_t)v * C]);

    ln.lp = full_logp(T, ps, ln.n, ln.L, &ln.S);
    const bool healthy = isfinite(ln.lp);
    a.status[c] = healthy ? 0 : 1;

    StepCtx sc;
    sc.chain = (uint32_t)c;
    sc.k0 = (uint32_t)a.seed;
    sc.k1 = (uint32_t)(a.seed >> 32);
    sc.cap = cap;
    sc.bthresh = a.bthresh;
    const double pb = (double)a.bthresh * 0x1p-32;
    sc.log_pb = log(pb);
    sc.log_pd = log1p(-pb);
    sc.sigma = a.sigma;
    sc.ikappa = 1.0 / a.kappa_end;
    sc.e2k = exp(-2.0 * a.kappa_end);
    sc.mala_h = a.mala_h;
    sc.sampler = a.sampler;
    sc.logw = a.logw ? a.logw + (size_t)t * (cap + 1) : nullptr;
    sc.hist = a.hist ? a.hist + (size_t)t * (cap + 1) : nullptr;
    ln.invw = 1.0;
    if (sc.logw) {
        ln.lwm = sc.logw[ln.n - 1];
        ln.lw0 = sc.logw[ln.n];
        ln.lwp = sc.logw[ln.n < cap ? ln.n + 1 : cap];
        ln.invw = inv_tilt<R>(ln.lw0);
    }
    const uint64_t step0 = a.step_dev ? *a.step_dev + a.step0 : a.step0; // step0 is the offset then
    int phase = (int)(step0 % (uint64_t)a.cycle_len);

    ln.live = healthy;
    // Every lane runs every step (a lane that is not live only rejects), so
    // that the step loop is uniform across the wave.  The wave stays in the
    // LDS-only loop while all its paths fit their slots and falls to the
    // general loop (slots beyond V in HBM) while some do not.
    int s = 0;
    while (s < a.steps) {
        for (; s < a.steps && __all(ln.n < a.V); ++s)
            one_step<R, true, SAMP>(a, T, pl, work, ln, sc, step0, s, phase, c, t);
        for (; s < a.steps && !__all(ln.n < a.V); ++s)
            one_step<R, false, SAMP>(a, T, ps, work, ln, sc, step0, s, phase, c, t);
    }

    fold_run(ln, T.n0, cap, sc.logw != nullptr);
    if (healthy) fold_hist(ln, sc);
    // log p of the final path (refreshed once rather than tracked per step)
    if (healthy) ln.lp = full_logp(T, ps, ln.n, ln.L);
    // write back the LDS part, the vertex count, log p and the statistics
    const int nw = ln.n < a.V ? ln.n : a.V;
    for (int v = 0; v < nw; ++v) ps.glb[(size_t)v * C] = lds_ld<R>(ps.lds + v * WAVE);
    a.n[c] = ln.n;
    a.logp[c] = ln.lp;
    if (healthy) {
        double* sp = a.stats + (size_t)c * RJPATH_NSTAT;
        sp[0] += ln.cnt;
        // without a sector tilt 1/w = 1 and the two sums are counts
        sp[1] += sc.logw ? ln.a1 : (double)ln.cnt;
        sp[2] += sc.logw ? ln.a2 : (double)ln.c2;
        sp[3] += ln.sl;
        sp[4] += ln.sl2;
        sp[5] += (double)ln.sn;
        sp[6] += ln.pp;
        sp[7] += ln.pb;
        sp[8] += ln.pd;
        sp[9] += ln.ap;
        sp[10] += ln.ab;
        sp[11] += ln.ad;
        sp[12] += ln.ncap;
        sp[13] += ln.mp;
        sp[14] += ln.ma;
        sp[15] += ln.ne;
    }
}

} // namespace rj
