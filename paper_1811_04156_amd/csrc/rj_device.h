// rj_device.h -- device-side building blocks of the gfx950 path sampler:
// counter-based random numbers, precision traits, layered-medium lookups and
// the factors of the path density (App. "Path probability distribution").
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rj_internal.h"

namespace rj {

// ---------------------------------------------------------------------------
// Precision traits.  FP32 uses the hardware transcendental instructions
// (v_log_f32, v_exp_f32, v_sqrt_f32, v_rsq_f32 and v_sin/v_cos_f32, which take
// their argument in revolutions); FP64 uses the device libm.
// ---------------------------------------------------------------------------
template <class R> struct Mth;

template <> struct Mth<float> {
    // the hardware log2 / exp2 / sqrt without the library's subnormal range
    // scaling: arguments and results of the path density never come near
    // 2^-126 except in degenerate paths whose density is zero anyway
    static __device__ __forceinline__ float log(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
    static __device__ __forceinline__ float exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    // sin / cos of 2 pi u for u in [0, 1)
    static __device__ __forceinline__ float sin2pi(float u) { return __builtin_amdgcn_sinf(u); }
    static __device__ __forceinline__ float cos2pi(float u) { return __builtin_amdgcn_cosf(u); }
    static __device__ __forceinline__ float log1p(float x) { return log1pf(x); }
    static __device__ __forceinline__ float expm1(float x) { return expm1f(x); }
    static __device__ __forceinline__ float ninf() { return -__builtin_inff(); }
};

template <> struct Mth<double> {
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double sin2pi(double u) { return ::sinpi(2.0 * u); }
    static __device__ __forceinline__ double cos2pi(double u) { return ::cospi(2.0 * u); }
    static __device__ __forceinline__ double log1p(double x) { return ::log1p(x); }
    static __device__ __forceinline__ double expm1(double x) { return ::expm1(x); }
    static __device__ __forceinline__ double ninf() { return -__builtin_inf(); }
};

template <class R> struct V3 {
    R x, y, z;
};
template <class R> __device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator*(R s, V3<R> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class R> __device__ __forceinline__ R dot(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// One path vertex as stored: position relative to the source, and w = the
// scattering depth of the segment that leaves the vertex.
template <class R> struct alignas(4 * sizeof(R)) Vtx {
    R x, y, z, w;
};
template <class R> __device__ __forceinline__ V3<R> pos(const Vtx<R>& v) { return {v.x, v.y, v.z}; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): two 32x32->64 products per round via
// v_mad_u64_u32, Weyl key schedule.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform in (0,1) from the top 23 bits: exact in FP32 and FP64 alike.
template <class R> __device__ __forceinline__ R unif(uint32_t x) { return ((R)(x >> 9) + (R)0.5) * (R)0x1p-23; }
// floor(x * m / 2^32)
__device__ __forceinline__ int pick(uint32_t x, uint32_t m) { return (int)__umulhi(x, m); }

// ---------------------------------------------------------------------------
// Layer constants (values, so a homogeneous medium keeps them in registers).
// ---------------------------------------------------------------------------
template <class R> struct LayV {
    R a, b, c, logb, g, hgn, hg1, keq, fsl, sln, sla;
};

template <class R> __device__ __forceinline__ LayV<R> lay_load(const R* p) {
    return LayV<R>{p[LY_A], p[LY_B], p[LY_C], p[LY_LOGB], p[LY_G], p[LY_HGN],
                   p[LY_HG1], p[LY_KEQ], p[LY_FSL], p[LY_SLN], p[LY_SLA]};
}

// ---------------------------------------------------------------------------
// Per-chain view of its target: sensor, emission, detection and medium.
// ---------------------------------------------------------------------------
template <class R> struct Tgt {
    V3<R> eta;    // sensor centre relative to the source (rounded to R)
    V3<R> eta_lo; // its rounding error: eta + eta_lo is the FP64 value
    R rad;        // sensor radius
    int ek;       // emission kind
    V3<R> ed;     // emission axis
    R kappa;      // vMF concentration
    R elog;       // log of the emission normalisation
    R ecos;       // cone: cos(half-angle)
    int dk;       // detection kind
    V3<R> dd;     // detection axis
    int n0;       // anchor sector
    // medium
    int mcnt, uniform;
    bool sl;      // false: no layer of the medium mixes in the Rayleigh-like term
    double ax, ay, az, e0, inv_h, usrc;
    // the FP32 layer lookups: the axis rounded, the source's position in layer
    // units split into its layer lsrc and the fraction fsrc, 1 / h and h
    V3<R> axr;
    R fsrc, ihr, hr;
    int lsrc;
    const MedInfo* mi;   // the medium's axis and spacing (the exact lookups read them here)
    LayV<R> l0;          // layer 0 (the only one of a homogeneous medium)
    const R* lay;        // layer table of this medium (LY_NW per layer), LDS or HBM
    const double* edge;  // edges of this medium (mcnt + 1)
    const double2* pre;  // prefix integrals (c, b) at the edges
};

// p - eta for a point p near the sensor: p - eta_hi is exact there (the two
// are within a factor of two of each other), so the offset from the sensor
// centre keeps its full relative precision although both lie ~100 m from the
// source where the coordinates are kept.
template <class R> __device__ __forceinline__ V3<R> from_eta(const Tgt<R>& T, V3<R> p) {
    return (p - T.eta) - T.eta_lo;
}

template <class R> __device__ __forceinline__ LayV<R> lay_at(const Tgt<R>& T, int l) {
    if (T.mcnt == 1) return T.l0;
    LayV<R> ly = lay_load(T.lay + l * LY_NW);
    if (!T.sl) ly.fsl = (R)0;
    return ly;
}

template <class R> __device__ __forceinline__ double axis_u(const Tgt<R>& T, V3<R> p) {
    return T.usrc + T.ax * (double)p.x + T.ay * (double)p.y + T.az * (double)p.z;
}

// Layer l with edge_l <= u < edge_{l+1}, outer layers unbounded.
template <class R> __device__ __forceinline__ int layer_u(const Tgt<R>& T, double u) {
    int cnt = T.mcnt;
    if (cnt == 1) return 0;
    int l;
    if (T.uniform) {
        double q = floor((u - T.e0) * T.inv_h);
        l = q < 0.0 ? 0 : (q >= (double)(cnt - 1) ? cnt - 1 : (int)q);
        // settle rounding against the stored edges
        if (l > 0 && u < T.edge[l]) --l;
        else if (l + 1 < cnt && u >= T.edge[l + 1]) ++l;
    } else {
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (u >= T.edge[mid]) lo = mid; else hi = mid - 1;
        }
        l = lo;
    }
    return l;
}

template <class R> __device__ __forceinline__ int layer_at(const Tgt<R>& T, V3<R> p) {
    if (T.mcnt == 1) return 0;
    return layer_u(T, axis_u(T, p));
}

// A point's coordinate along the layer axis and its layer index, computed
// once per vertex and step and shared by every factor and segment that
// touches the vertex.  FP64: the absolute coordinate; FP32: the coordinate
// relative to the source (the vertices' own frame, so that it is as precise
// as the vertex itself).
template <class R> struct LPt {
    R u;
    int l;
};

// Layer index of axis coordinate u: for uniformly spaced edges the floor of
// (u - e0) / h, settled against the two stored edges around it without
// branching (the same index as layer_u).
template <class R> __device__ __forceinline__ int layer_idx_s(const Tgt<R>& T, double u, double e0, double inv_h) {
    const int cnt = T.mcnt;
    if (cnt == 1) return 0;
    if (!T.uniform) return layer_u(T, u);
    double q = floor((u - e0) * inv_h);
    q = fmin(fmax(q, 0.0), (double)(cnt - 1));
    const int l = (int)q;
    const double elo = T.edge[l], ehi = T.edge[l + 1];
    const int up = (u >= ehi && l + 1 < cnt) ? 1 : 0;
    const int dn = (u < elo && l > 0) ? 1 : 0;
    return l + up - dn;
}
template <class R> __device__ __forceinline__ int layer_idx(const Tgt<R>& T, double u) {
    return layer_idx_s(T, u, T.e0, T.inv_h);
}

// The exact (FP64) axis coordinate and layer of p, with the medium's axis and
// spacing read from its record (the FP32 step keeps only their FP32 forms).
template <class R> __device__ __forceinline__ double axis_u_m(const Tgt<R>& T, V3<R> p) {
    const MedInfo& m = *T.mi;
    return T.usrc + m.ax * (double)p.x + m.ay * (double)p.y + m.az * (double)p.z;
}

// Axis position of edge k relative to the source (FP32 lookups).
template <class R> __device__ __forceinline__ R edge_rel(const Tgt<R>& T, int k) {
    return T.uniform ? ((R)(k - T.lsrc) - T.fsrc) * T.hr : (R)(T.edge[k] - T.usrc);
}

// Fractional layer coordinates closer than this to an integer, or farther
// than LAYER_REACH layers from the source's, leave the layer to the exact
// lookup: the FP32 layer coordinate is good to 2.5e-5 layers within 64
// layers of the source.
constexpr float LAYER_MARGIN = 0x1p-15f;
constexpr float LAYER_REACH = 64.0f;

// Layer point of p.  FP64: exact.  FP32: u relative to the source in FP32
// and the layer from the fractional layer coordinate; `near` reports the
// points whose layer lpt_settle must decide (near an edge, far from the
// source, or in a medium with unevenly spaced edges).
template <class R> __device__ __forceinline__ LPt<R> lpt_fast(const Tgt<R>& T, V3<R> p, bool& near) {
    near = false;
    if (T.mcnt == 1) return LPt<R>{(R)0, 0};
    if constexpr (sizeof(R) == 8) {
        const double u = axis_u(T, p);
        return LPt<R>{u, layer_idx(T, u)};
    } else {
        const R x = T.axr.x * p.x + T.axr.y * p.y + T.axr.z * p.z;
        const R xi = T.fsrc + x * T.ihr;
        const R fl = floorf(xi), fr = xi - fl;
        const R lf = fminf(fmaxf((R)T.lsrc + fl, (R)0), (R)(T.mcnt - 1));
        near = !T.uniform || fr < (R)LAYER_MARGIN || fr > (R)1 - (R)LAYER_MARGIN || !(fabsf(xi) < (R)LAYER_REACH);
        return LPt<R>{x, (int)lf};
    }
}

// The exact (FP64) layer of p for an FP32 layer point, with u kept inside
// the real edges of that layer, so that the depth pieces of a crossing are
// never negative (no-op in FP64).
template <class R> __device__ __forceinline__ void lpt_settle(const Tgt<R>& T, V3<R> p, LPt<R>& q) {
    if constexpr (sizeof(R) == 4) {
        if (T.mcnt == 1) return;
        const MedInfo& m = *T.mi;
        const int l = layer_idx_s(T, axis_u_m(T, p), m.e0, m.inv_h);
        R x = q.u;
        if (l >= 1) x = fmaxf(x, edge_rel(T, l));
        if (l <= T.mcnt - 2) x = fminf(x, edge_rel(T, l + 1));
        q = LPt<R>{x, l};
    }
}

template <class R> __device__ __forceinline__ LPt<R> lpt(const Tgt<R>& T, V3<R> p) {
    bool near;
    LPt<R> q = lpt_fast(T, p, near);
    if (near) lpt_settle(T, p, q);
    return q;
}

// Optical depths of the segment P -> Q of length len: total c = a + b and
// scattering b; exact piecewise integral along the layer axis (the length
// factor of the depth definition restored).  The crossing case is done in
// FP64 so that short crossings of a layer boundary keep their precision.
template <class R>
__device__ __forceinline__ void seg_depth(const Tgt<R>& T, V3<R> P, V3<R> Q, R len, R& tc, R& tb) {
    if (T.mcnt == 1) {
        tc = T.l0.c * len;
        tb = T.l0.b * len;
        return;
    }
    double uP = axis_u(T, P), uQ = axis_u(T, Q);
    int lP = layer_u(T, uP), lQ = layer_u(T, uQ);
    if (lP == lQ) {
        const R* ly = T.lay + lP * LY_NW;
        tc = ly[LY_C] * len;
        tb = ly[LY_B] * len;
        return;
    }
    double lo = uP, hi = uQ;
    int llo = lP, lhi = lQ;
    if (uP > uQ) {
        lo = uQ; hi = uP; llo = lQ; lhi = lP;
    }
    const R* a = T.lay + llo * LY_NW;
    const R* b = T.lay + lhi * LY_NW;
    double eh = T.edge[llo + 1], el = T.edge[lhi];
    double2 ph = T.pre[llo + 1], pl = T.pre[lhi];
    double Ic = (double)a[LY_C] * (eh - lo) + (pl.x - ph.x) + (double)b[LY_C] * (hi - el);
    double Ib = (double)a[LY_B] * (eh - lo) + (pl.y - ph.y) + (double)b[LY_B] * (hi - el);
    double inv = 1.0 / (hi - lo);
    tc = (R)(Ic * inv) * len;
    tb = (R)(Ib * inv) * len;
}

// seg_depth with the endpoints' layer points already known.
template <class R>
__device__ __forceinline__ void seg_depth_lp(const Tgt<R>& T, LPt<R> P, LPt<R> Q, R len, R& tc, R& tb) {
    if (T.mcnt == 1) {
        tc = T.l0.c * len;
        tb = T.l0.b * len;
        return;
    }
    if constexpr (sizeof(R) == 4) {
        // FP32: the partial layers at both ends from the relative coordinates
        // (each piece as precise as the vertices), the whole layers between
        // from the FP64 prefix integrals
        const bool swap = P.u > Q.u;
        const R lo = swap ? Q.u : P.u, hi = swap ? P.u : Q.u;
        const int llo = swap ? Q.l : P.l, lhi = swap ? P.l : Q.l;
        const R* a = T.lay + llo * LY_NW;
        const R* b = T.lay + lhi * LY_NW;
        const R ac = a[LY_C], ab = a[LY_B], bc = b[LY_C], bb = b[LY_B];
        const double2 ph = T.pre[llo + 1], pl = T.pre[lhi];
        const bool same = P.l == Q.l;
        // mean coefficient = c_hi + (c_lo - c_hi) f + (I_mid - c_hi W) / (hi - lo),
        // f = the share of the low layer, W the width of the whole layers
        // between (0 and I_mid = 0 for neighbouring layers): a thin crossing
        // errs by at most |c_lo - c_hi| of its length
        const R d1 = edge_rel(T, llo + 1) - lo;
        const R W = T.uniform ? (R)(lhi - llo - 1) * T.hr : (R)(T.edge[lhi] - T.edge[llo + 1]);
        const R ir = Mth<R>::rcp(same ? (R)1 : fmaxf(hi - lo, (R)0x1p-100));
        const R f = fminf(d1 * ir, (R)1);
        const R mc = bc + (ac - bc) * f + ((R)(pl.x - ph.x) - bc * W) * ir;
        const R mb = bb + (ab - bb) * f + ((R)(pl.y - ph.y) - bb * W) * ir;
        tc = (same ? ac : mc) * len;
        tb = (same ? ab : mb) * len;
        return;
    }
    // evaluated for every lane and selected (no divergent branch): inside one
    // layer the depth is c * len; across layers the mean coefficient comes
    // from the FP64 prefix integrals between the two axis coordinates
    const bool swap = P.u > Q.u;
    const double lo = swap ? Q.u : P.u, hi = swap ? P.u : Q.u;
    const int llo = swap ? Q.l : P.l, lhi = swap ? P.l : Q.l;
    const R* a = T.lay + llo * LY_NW;
    const R* b = T.lay + lhi * LY_NW;
    const R ac = a[LY_C], ab = a[LY_B];
    const double eh = T.edge[llo + 1], el = T.edge[lhi];
    const double2 ph = T.pre[llo + 1], pl = T.pre[lhi];
    const double Ic = (double)ac * (eh - lo) + (pl.x - ph.x) + (double)b[LY_C] * (hi - el);
    const double Ib = (double)ab * (eh - lo) + (pl.y - ph.y) + (double)b[LY_B] * (hi - el);
    const bool same = P.l == Q.l;
    if constexpr (sizeof(R) == 4) {
        // the quotient is rounded to FP32 anyway: an FP32 reciprocal of the
        // FP64 difference (rounded once) instead of an FP64 division
        const R ir = Mth<R>::rcp((R)(same ? 1.0 : hi - lo));
        tc = same ? ac * len : (R)Ic * ir * len;
        tb = same ? ab * len : (R)Ib * ir * len;
    } else {
        const double inv = 1.0 / (same ? 1.0 : hi - lo);
        tc = same ? ac * len : (R)(Ic * inv) * len;
        tb = same ? ab * len : (R)(Ib * inv) * len;
    }
}

// log of the per-steradian scattering function at a vertex with incoming and
// outgoing unit directions ua, ub; 1 - mu = |ua - ub|^2 / 2 keeps the forward
// peak accurate in FP32.
template <class R> __device__ __forceinline__ R turn_term(const LayV<R>& ly, V3<R> ua, V3<R> ub) {
    V3<R> d = ua - ub;
    R q = dot(d, d); // 2 (1 - mu)
    R hg = ly.hgn - (R)1.5 * Mth<R>::log(ly.hg1 + ly.g * q);
    if (ly.fsl == (R)0) return hg;
    R sl = ly.sln + ly.sla * Mth<R>::log((R)1 - (R)0.25 * q);
    R m = sl > hg ? sl : hg;
    return m + Mth<R>::log(ly.fsl * Mth<R>::exp(sl - m) + ((R)1 - ly.fsl) * Mth<R>::exp(hg - m));
}

// log of the emission density at the first direction u0 (eq. emission_dist
// and the isotropic / cone forms).
template <class R> __device__ __forceinline__ R emit_term(const Tgt<R>& T, V3<R> u0) {
    if (T.ek == RJPATH_EMIT_ISO) return T.elog;
    if (T.ek == RJPATH_EMIT_VMF) {
        V3<R> d = u0 - T.ed;
        return T.elog - (R)0.5 * T.kappa * dot(d, d); // kappa (u.e - 1) + log norm
    }
    return dot(u0, T.ed) >= T.ecos ? T.elog : Mth<R>::ninf();
}

// log of the final factor without its segment terms: log max(0, -u . nu) +
// log rho(nu), with nu the outward normal at the end point fe.
template <class R> __device__ __forceinline__ R end_term(const Tgt<R>& T, V3<R> ul, V3<R> fe) {
    V3<R> d = from_eta(T, fe);
    V3<R> nu = Mth<R>::rsqrt(dot(d, d)) * d;
    R c = -dot(ul, nu);
    if (!(c > (R)0)) return Mth<R>::ninf();
    R t = Mth<R>::log(c);
    if (T.dk == RJPATH_DET_PAPER) {
        R cr = dot(nu, T.dd);
        R z = (R)2 * cr + (R)0.7;
        // log cosh z = |z| + log1p(e^{-2|z|}) - log 2
        R az = z < (R)0 ? -z : z;
        t += (R)3 * cr - (R)1 - (az + Mth<R>::log1p(Mth<R>::exp((R)-2 * az)) - (R)0.69314718055994530942);
    }
    return t;
}

// A straight segment: unit direction, length, log length and depths.
template <class R> struct Seg {
    V3<R> u;
    R len, loglen, tc, tb;
};

template <class R> __device__ __forceinline__ Seg<R> make_seg(const Tgt<R>& T, V3<R> P, V3<R> Q) {
    Seg<R> s;
    V3<R> r = Q - P;
    R l2 = dot(r, r);
    R il = Mth<R>::rsqrt(l2);
    s.u = il * r;
    s.len = l2 * il;
    s.loglen = (R)0.5 * Mth<R>::log(l2);
    seg_depth(T, P, Q, s.len, s.tc, s.tb);
    return s;
}

template <class R>
__device__ __forceinline__ Seg<R> make_seg_lp(const Tgt<R>& T, V3<R> P, V3<R> Q, LPt<R> lP, LPt<R> lQ) {
    Seg<R> s;
    V3<R> r = Q - P;
    R l2 = dot(r, r);
    R il = Mth<R>::rsqrt(l2);
    s.u = il * r;
    s.len = l2 * il;
    s.loglen = (R)0.5 * Mth<R>::log(l2);
    seg_depth_lp(T, lP, lQ, s.len, s.tc, s.tb);
    return s;
}

// -tau_a - tau_b - 2 log |r| of a segment (each segment carries one
// attenuation and one inverse-square factor, p_v and p_f alike).
template <class R> __device__ __forceinline__ R seg_term(const Seg<R>& s) { return -s.tc - (R)2 * s.loglen; }

template <class R> __device__ __forceinline__ V3<R> unit_dir(V3<R> P, V3<R> Q) {
    V3<R> r = Q - P;
    return Mth<R>::rsqrt(dot(r, r)) * r;
}

// unit vector from the sensor centre to Q
template <class R> __device__ __forceinline__ V3<R> unit_dir_eta(const Tgt<R>& T, V3<R> Q) {
    V3<R> r = from_eta(T, Q);
    return Mth<R>::rsqrt(dot(r, r)) * r;
}

// Orthonormal completion of a unit vector (Duff et al., JCGT 2017).
template <class R> __device__ __forceinline__ void onb(V3<R> n, V3<R>& e2, V3<R>& e3) {
    R sgn = copysign((R)1, n.z);
    R a = -Mth<R>::rcp(sgn + n.z);
    R b = n.x * n.y * a;
    e2 = {(R)1 + sgn * n.x * n.x * a, sgn * b, -sgn * n.x};
    e3 = {b, sgn + n.y * n.y * a, -n.y};
}

// Where the media tables are read from during a launch (LDS copy or HBM).
template <class R> struct MedTab {
    const R* lay;
    const double* edge;
    const double* pre;
};

// Loads the view of target t.  `tab` gives the layer tables (the FP64 table
// for the FP64 quadratures regardless of the chains' precision).
template <class R>
__device__ __forceinline__ void load_target(const KArgs& a, int t, Tgt<R>& T, const MedTab<R>& tab) {
    const double* s = a.sensor + 3 * t;
    const double* o = a.src + 3 * t;
    const double ex = s[0] - o[0], ey = s[1] - o[1], ez = s[2] - o[2];
    T.eta = {(R)ex, (R)ey, (R)ez};
    T.eta_lo = {(R)(ex - (double)T.eta.x), (R)(ey - (double)T.eta.y), (R)(ez - (double)T.eta.z)};
    T.rad = (R)a.radius[t];
    T.ek = a.ek[t];
    T.ed = {(R)a.edir[3 * t], (R)a.edir[3 * t + 1], (R)a.edir[3 * t + 2]};
    double ep = a.eparam[t];
    const double PI = 3.14159265358979323846;
    T.kappa = (R)ep;
    T.ecos = (R)0;
    if (T.ek == RJPATH_EMIT_ISO) {
        T.elog = (R)(-log(4.0 * PI));
    } else if (T.ek == RJPATH_EMIT_VMF) {
        // kappa e^{kappa u.e} / (4 pi sinh kappa) = e^{kappa (u.e - 1)} kappa / (2 pi (1 - e^{-2 kappa}))
        T.elog = (R)(log(ep) - log(2.0 * PI) - log1p(-exp(-2.0 * ep)));
    } else {
        double ca = cos(ep);
        T.ecos = (R)ca;
        T.elog = (R)(-log(2.0 * PI * (1.0 - ca)));
    }
    T.dk = a.dk[t];
    T.dd = {(R)a.ddir[3 * t], (R)a.ddir[3 * t + 1], (R)a.ddir[3 * t + 2]};
    T.n0 = a.n0[t];
    const MedInfo mi = a.minfo[a.medium[t]];
    T.mcnt = mi.cnt;
    T.sl = true;
    T.uniform = mi.uniform;
    T.ax = mi.ax;
    T.ay = mi.ay;
    T.az = mi.az;
    T.e0 = mi.e0;
    T.inv_h = mi.inv_h;
    T.usrc = mi.ax * o[0] + mi.ay * o[1] + mi.az * o[2];
    T.mi = a.minfo + a.medium[t];
    T.axr = {(R)mi.ax, (R)mi.ay, (R)mi.az};
    {
        const double xs = (T.usrc - mi.e0) * mi.inv_h;
        const double fl = floor(xs);
        T.lsrc = (int)fmin(fmax(fl, -1e9), 1e9);
        T.fsrc = (R)(xs - fl);
        T.ihr = (R)mi.inv_h;
        T.hr = (R)(1.0 / mi.inv_h);
    }
    T.lay = tab.lay + (size_t)mi.off * LY_NW;
    T.l0 = lay_load(T.lay);
    int eo = mi.off + a.medium[t];
    T.edge = tab.edge + eo;
    T.pre = (const double2*)tab.pre + eo;
}

template <class R> __device__ __forceinline__ MedTab<R> hbm_tab(const KArgs& a) {
    return MedTab<R>{(const R*)a.lay, a.edge, a.pre};
}

} // namespace rj
