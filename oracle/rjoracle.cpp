// rjoracle.cpp -- plain FP64 CPU oracle for reversible-jump MCMC sampling of
// photon paths (Collin, "Using path integrals for the propagation of light in
// a scattering dominated medium", arXiv:1811.04156).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
// reference that the HIP path is checked against.  It is loaded only by the
// tests, by the smoke check and by the CPU-baseline leg of the benchmark; the
// product library never links or calls it, and it shares no code, header or
// table with the HIP sources.
//
// Every quantity is evaluated in double precision, written in the paper's
// factor order and notation.  Where the paper is silent or garbled the
// adopted reading is stated next to the code (readings R1..R17, listed in the
// design notes of the repository).
//
// Parity status of each exported function is stated in its header comment;
// all are pinned by the CPU test-suite against closed forms, quadrature,
// brute force or finite differences.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

const double PI = 3.14159265358979323846;
const double NEG_INF = -std::numeric_limits<double>::infinity();

struct V3 {
    double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 ld3(const double* p) { return {p[0], p[1], p[2]}; }
inline void st3(double* p, V3 v) { p[0] = v.x; p[1] = v.y; p[2] = v.z; }

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator, written from its published
// definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the
// Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t in[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {in[0], in[1], in[2], in[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// Open-interval uniform with 23 random bits: exactly representable in both
// single and double precision, so both implementations see the same value.
inline double unif(uint32_t x) { return ((double)(x >> 9) + 0.5) * 0x1p-23; }
// Unbiased-enough index in [0, m): floor(x * m / 2^32), pure integer.
inline uint32_t pick(uint32_t x, uint32_t m) { return (uint32_t)(((uint64_t)x * m) >> 32); }

// The eight 32-bit draws of one chain at one step: two Philox blocks with
// counter (chain, step low, step high, block) and key (seed low, seed high).
void step_draws(uint64_t seed, uint32_t chain, uint64_t step, uint32_t r[8]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t c0[4] = {chain, (uint32_t)step, (uint32_t)(step >> 32), 0u};
    uint32_t c1[4] = {chain, (uint32_t)step, (uint32_t)(step >> 32), 1u};
    philox4x32_10(c0, key, r);
    philox4x32_10(c1, key, r + 4);
}

// Orthonormal completion of a unit vector (Duff et al., "Building an
// orthonormal basis, revisited", JCGT 2017).
void onb(V3 n, V3* e2, V3* e3) {
    double sgn = std::copysign(1.0, n.z);
    double a = -1.0 / (sgn + n.z);
    double b = n.x * n.y * a;
    *e2 = {1.0 + sgn * n.x * n.x * a, sgn * b, -sgn * n.x};
    *e3 = {b, sgn + n.y * n.y * a, -n.y};
}

// ---------------------------------------------------------------------------
// Medium: absorption a(x) and scattering b(x) (App. "Intermediate vertex").
// A medium is a stack of layers along a unit axis; layer l covers
// [edge[l], edge[l+1]) and the outermost layers extend to -inf / +inf.
// Coefficients are a = 1/absorption length, b = 1/scattering length.
// ---------------------------------------------------------------------------
struct Medium {
    V3 axis;
    int L;
    std::vector<double> edge, a, b, g, fsl;
};

int layer_of(const Medium& m, double u) {
    int l = 0;
    while (l + 1 < m.L && u >= m.edge[l + 1]) ++l;
    return l;
}

// Eq. (b_depth_def) with the segment length restored (reading R1):
// tau_x = |Q-P| * int_0^1 x(P + s (Q-P)) ds, integrated exactly over the
// piecewise-constant layers.  uP, uQ are the layer-axis coordinates.
double depth(const Medium& m, const std::vector<double>& x, double uP, double uQ, double len) {
    if (uP == uQ) return len * x[layer_of(m, uP)];
    double lo = std::min(uP, uQ), hi = std::max(uP, uQ), acc = 0.0;
    for (int l = 0; l < m.L; ++l) {
        double bot = (l == 0) ? -INFINITY : m.edge[l];
        double top = (l == m.L - 1) ? INFINITY : m.edge[l + 1];
        double ov = std::min(hi, top) - std::max(lo, bot);
        if (ov > 0) acc += x[l] * ov;
    }
    return len * acc / (hi - lo);
}

// Length of the segment inside each layer (for parameter derivatives).
void layer_lengths(const Medium& m, double uP, double uQ, double len, std::vector<double>& out) {
    if (uP == uQ) {
        out[layer_of(m, uP)] += len;
        return;
    }
    double lo = std::min(uP, uQ), hi = std::max(uP, uQ);
    for (int l = 0; l < m.L; ++l) {
        double bot = (l == 0) ? -INFINITY : m.edge[l];
        double top = (l == m.L - 1) ? INFINITY : m.edge[l + 1];
        double ov = std::min(hi, top) - std::max(lo, bot);
        if (ov > 0) out[l] += len * ov / (hi - lo);
    }
}

// Angular scattering distribution over cos(theta) (eq. angular_scattering):
// f_SL * p_SL + (1 - f_SL) * p_HG, both with mean cosine Gamma.
double p_hg(double mu, double G) { return 0.5 * (1 - G * G) * std::pow(1 + G * G - 2 * G * mu, -1.5); }
double p_sl(double mu, double G) {
    if (G == 0.0) return 0.5;
    return 0.5 * ((1 + G) / (1 - G)) * std::pow((1 + mu) / 2, 2.0 / (1.0 / G - 1.0));
}
double sigma_mix(double mu, double G, double fsl) { return fsl * p_sl(mu, G) + (1 - fsl) * p_hg(mu, G); }
// Per-steradian phase function, sigma / (2 pi) (reading R3).
double sigma_sr(double mu, double G, double fsl) { return sigma_mix(mu, G, fsl) / (2 * PI); }

// ---------------------------------------------------------------------------
// Targets: point source, spherical sensor (App. "Initial vertex", "Final
// vertex").  Path vertices are stored relative to the source position.
// ---------------------------------------------------------------------------
struct Target {
    V3 src;   // absolute source position
    V3 eta;   // sensor centre relative to the source
    double R; // sensor radius
    int ek;   // emission kind: 0 isotropic, 1 von Mises-Fisher, 2 uniform cone
    V3 edir;
    double eparam; // kappa (vMF) or half-angle (cone)
    int dk;        // detection: 0 uniform, 1 eq. (detection_prob)
    V3 ddir;
    int medium;
    int n0;                  // anchor sector
    std::vector<double> logw; // sector tilt log w(n), n = 0..cap
};

// Eq. (emission_dist) and the isotropic / cone variants (reading R12).
double emission(const Target& t, V3 u) {
    double c = dot(u, t.edir);
    if (t.ek == 0) return 1.0 / (4 * PI);
    if (t.ek == 1) return t.eparam * std::exp(t.eparam * c) / (4 * PI * std::sinh(t.eparam));
    double ca = std::cos(t.eparam);
    return (c >= ca) ? 1.0 / (2 * PI * (1 - ca)) : 0.0;
}

// Eq. (detection_prob); rho = 1 for the uniform sensor (reading R11).
double detection(const Target& t, V3 nu) {
    if (t.dk == 0) return 1.0;
    double c = dot(nu, t.ddir);
    return std::exp(3 * c - 1) / std::cosh(2 * c + 0.7);
}

struct Ctx {
    std::vector<Medium> media;
    std::vector<Target> targets;
    int cap;
};

double axis_coord(const Ctx& cx, const Target& t, V3 f) {
    const Medium& m = cx.media[t.medium];
    return dot(m.axis, t.src + f);
}

// log p of a path f_0..f_{n-1} (relative to the source), the factorised
// density of the appendix ("Path probability distribution"):
//   p = p_i(f0,f1) * prod_{k=1}^{n-2} p_v(f_{k-1},f_k,f_{k+1}) * p_f(f_{n-2},f_{n-1})
// with p_v = b(f_k) e^{-tau(k)} / |r_{k-1}|^2 * sigma_sr(cos theta_k)   (eq. intervtx)
// and  p_f = e^{-tau(last)} max(0, -r_hat . nu) / |r_{n-2}|^2 * rho   (reading R2).
double logp_path(const Ctx& cx, const Target& t, int n, const V3* f) {
    if (n < 2) return NEG_INF;
    const Medium& m = cx.media[t.medium];
    std::vector<V3> uh(n - 1);
    std::vector<double> len(n - 1), tau(n - 1);
    for (int k = 0; k + 1 < n; ++k) {
        V3 r = f[k + 1] - f[k];
        len[k] = norm(r);
        if (!(len[k] > 0)) return NEG_INF;
        uh[k] = (1.0 / len[k]) * r;
        double uP = axis_coord(cx, t, f[k]), uQ = axis_coord(cx, t, f[k + 1]);
        tau[k] = depth(m, m.a, uP, uQ, len[k]) + depth(m, m.b, uP, uQ, len[k]);
    }
    // initial factor
    double pi = emission(t, uh[0]);
    if (!(pi > 0)) return NEG_INF;
    double lp = std::log(pi);
    // intermediate factors
    for (int k = 1; k <= n - 2; ++k) {
        int l = layer_of(m, axis_coord(cx, t, f[k]));
        double bk = m.b[l];
        if (!(bk > 0)) return NEG_INF;
        double mu = dot(uh[k - 1], uh[k]);
        double pv = bk * std::exp(-tau[k - 1]) / (len[k - 1] * len[k - 1]) * sigma_sr(mu, m.g[l], m.fsl[l]);
        lp += std::log(pv);
    }
    // final factor
    V3 d = f[n - 1] - t.eta;
    V3 nu = (1.0 / norm(d)) * d;
    double cphi = std::max(0.0, -dot(uh[n - 2], nu));
    if (!(cphi > 0)) return NEG_INF;
    double pf = std::exp(-tau[n - 2]) * cphi / (len[n - 2] * len[n - 2]) * detection(t, nu);
    lp += std::log(pf);
    return lp;
}

// ---------------------------------------------------------------------------
// Dimension-matching transformation (App. "Dimension matching
// transformation"): bi-spherical coordinates (s, t, phi) about the foci A, B,
// with the origin at their midpoint (reading R5) and t = ln(d_A / d_B) with
// the primary axis pointing from A to B (reading R6).
// ---------------------------------------------------------------------------
V3 bisph(V3 A, V3 B, double s, double t, double phi) {
    V3 r = B - A;
    double gam = 0.5 * norm(r);
    V3 e1 = (1.0 / (2 * gam)) * r, e2, e3;
    onb(e1, &e2, &e3);
    V3 mid = 0.5 * (A + B);
    double den = std::cosh(t) - std::cos(s);
    V3 dir = std::sinh(t) * e1 + std::sin(s) * (std::cos(phi) * e2 + std::sin(phi) * e3);
    return mid + (gam / den) * dir;
}

void bisph_inv(V3 A, V3 B, V3 f, double* s, double* t, double* phi) {
    double dA = norm(f - A), dB = norm(f - B);
    double cs = dot(A - f, B - f) / (dA * dB);
    cs = std::max(-1.0, std::min(1.0, cs));
    *s = std::acos(cs);
    *t = std::log(dA / dB);
    V3 r = B - A;
    V3 e1 = (1.0 / norm(r)) * r, e2, e3;
    onb(e1, &e2, &e3);
    V3 q = f - 0.5 * (A + B);
    V3 tr = q - dot(q, e1) * e1;
    *phi = std::atan2(dot(tr, e3), dot(tr, e2));
    if (*phi < 0) *phi += 2 * PI;
}

double jac_bisph(double s, double t, double gam) { return std::pow(gam / (std::cosh(t) - std::cos(s)), 3) * std::sin(s); }

// q(s) = beta e^{-beta cos s} sin s / (2 sinh beta); uniform-in-cos limit at beta = 0.
double q_s(double s, double beta) {
    if (beta == 0.0) return 0.5 * std::sin(s);
    return beta * std::exp(-beta * std::cos(s)) * std::sin(s) / (2 * std::sinh(beta));
}
double q_t(double t) { return 1.0 / (2 + 2 * std::cosh(t)); }
double q_phi() { return 1.0 / (2 * PI); }

// Inverse CDF of q(s): F(s) = (e^{-beta cos s} - e^{-beta}) / (e^{beta} - e^{-beta}).
double sample_cos_s(double u, double beta) {
    if (beta == 0.0) return 1.0 - 2.0 * u;
    if (std::fabs(beta) < 300.0)
        return -std::log(std::exp(-beta) + u * (std::exp(beta) - std::exp(-beta))) / beta;
    // same inverse CDF with e^{beta} factored out (overflow-free)
    return -1.0 - std::log1p(-(1.0 - u) * -std::expm1(-2 * beta)) / beta;
}

// coth k - 1/k = Gamma (von Mises-Fisher concentration with mean cosine Gamma).
double kappa_eq(double G) {
    if (G <= 0) return 0.0;
    double lo = 1e-12, hi = 1e7;
    for (int i = 0; i < 200; ++i) {
        double mid = 0.5 * (lo + hi);
        double v = 1.0 / std::tanh(mid) - 1.0 / mid;
        if (v < G) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// Centering rule: beta = kappa_eq + (gamma b(f') - 1)/2, with b and Gamma
// evaluated at the midpoint of the chosen segment (reading R7).
double centre_beta(const Ctx& cx, const Target& t, V3 A, V3 B) {
    const Medium& m = cx.media[t.medium];
    int l = layer_of(m, axis_coord(cx, t, 0.5 * (A + B)));
    double gam = 0.5 * norm(B - A);
    return kappa_eq(m.g[l]) + (gam * m.b[l] - 1.0) / 2.0;
}

double seg_taub(const Ctx& cx, const Target& t, V3 P, V3 Q) {
    const Medium& m = cx.media[t.medium];
    return depth(m, m.b, axis_coord(cx, t, P), axis_coord(cx, t, Q), norm(Q - P));
}

// ---------------------------------------------------------------------------
// Run parameters and the reversible-jump step.
// ---------------------------------------------------------------------------
struct Params {
    uint64_t seed;
    uint64_t step0;
    int64_t burn_in;
    int steps;
    int cycle_len, n_perturb;
    uint32_t birth_thresh; // birth iff draw < birth_thresh (birth fraction * 2^32)
    double sigma, kappa_end;
    int sampler; // 0 plain, 1 joint Langevin move of all interior vertices, 2 single-vertex Langevin move,
                 // 3 tree-coordinate move of the whole path (first step of every cycle)
    double mala_h;
};

enum { MV_INTERIOR = 0, MV_END = 1, MV_BIRTH = 2, MV_DEATH = 3, MV_MALA = 4, MV_NULL = 5, MV_LMALA = 6, MV_TREE = 7 };
enum { NSTAT = 16 };

struct StepRec {
    int move, accepted, index;
    double logA, logu;
};

double logw_of(const Target& t, int n) { return t.logw.empty() ? 0.0 : t.logw[n]; }

// Green's acceptance for the birth x (n vertices) -> y (n+1) with the new
// vertex between x_k and x_{k+1} (eq. acceptFact, read as in reading R4):
// A = p(y) w(n+1) P(n+1 -> n) |J| / (p(x) w(n) P(n -> n+1, k) q(s) q(t) q(phi)).
double log_birth_ratio(const Ctx& cx, const Target& t, const Params& P, const std::vector<V3>& x,
                       int k, const std::vector<V3>& y, double s, double tt) {
    int n = (int)x.size();
    double S = 0;
    for (int l = 0; l + 1 < n; ++l) S += seg_taub(cx, t, x[l], x[l + 1]);
    double tk = seg_taub(cx, t, x[k], x[k + 1]);
    double pb = (double)P.birth_thresh * 0x1p-32;
    double p_up = pb * tk / S;                  // p(n -> n+1, k), jump-proposal appendix
    double p_down = (1.0 - pb) / (double)(n + 1 - 2); // p(n+1 -> n, k) = 1/(n+1-2)
    double gam = 0.5 * norm(x[k + 1] - x[k]);
    double beta = centre_beta(cx, t, x[k], x[k + 1]);
    double J = jac_bisph(s, tt, gam);
    double q = q_s(s, beta) * q_t(tt) * q_phi();
    double lpy = logp_path(cx, t, n + 1, y.data());
    double lpx = logp_path(cx, t, n, x.data());
    return (lpy + logw_of(t, n + 1)) - (lpx + logw_of(t, n)) + std::log(p_down) - std::log(p_up) + std::log(J) -
           std::log(q);
}

double path_length(const std::vector<V3>& f) {
    double L = 0;
    for (size_t k = 0; k + 1 < f.size(); ++k) L += norm(f[k + 1] - f[k]);
    return L;
}

// Gradient of log p with respect to the vertices (declared below).
void grad_vertices(const Ctx& cx, const Target& t, int n, const V3* f, V3* g);

// ---------------------------------------------------------------------------
// Proposals as functions of continuous draws.  The sampler below feeds them
// the uniforms of its random words; the tests feed them arbitrary uniforms to
// measure the density of each proposal from its own map (numerical Jacobian
// of draws -> proposed path), independently of the printed J and q.
// ---------------------------------------------------------------------------
struct Prop {
    int move;
    std::vector<V3> y; // proposed path (empty: no proposal, rejected)
    double logA;
};

// Three standard normals from four uniforms (Box-Muller, the fourth normal unused).
V3 box_muller3(const double u[4]) {
    double rho1 = std::sqrt(-2 * std::log(u[0]));
    double rho2 = std::sqrt(-2 * std::log(u[2]));
    return {rho1 * std::cos(2 * PI * u[1]), rho1 * std::sin(2 * PI * u[1]), rho2 * std::cos(2 * PI * u[3])};
}

// Step size of the single-vertex Langevin move at interior vertex j of f:
// mala_h times the squared length of the shorter segment at f_j, so that the
// drift and noise stay a fixed fraction of the local length scale.
double local_h(const Params& P, const std::vector<V3>& f, int j) {
    double la = norm(f[j] - f[j - 1]), lb = norm(f[j + 1] - f[j]);
    double m = std::min(la, lb);
    return P.mala_h * m * m;
}

// Perturbation of vertex j (1 <= j <= n-1) from the uniforms u[0..3]:
//  - interior vertex, plain sampler: Gaussian step sigma * xi (symmetric);
//  - interior vertex, single-vertex Langevin sampler: y_j = f_j + (h/2) g_j + sqrt(h) xi
//    with g_j = d log p / d f_j and h = local_h, accepted with the ratio of the
//    two Gaussian proposal densities (the reverse one at y);
//  - the end point: von Mises-Fisher step on the sensor sphere about its
//    current normal, cos = 1 + log(u0 + (1 - u0) e^{-2 kappa}) / kappa,
//    azimuth 2 pi u1 (symmetric).
Prop propose_perturb(const Ctx& cx, const Target& t, const Params& P, const std::vector<V3>& f, int j,
                     const double u[4]) {
    int n = (int)f.size();
    Prop pr{MV_INTERIOR, f, NEG_INF};
    if (j <= n - 2 && P.sampler == 2) {
        pr.move = MV_LMALA;
        std::vector<V3> gx(n), gy(n);
        grad_vertices(cx, t, n, f.data(), gx.data());
        double hx = local_h(P, f, j);
        V3 xi = box_muller3(u);
        pr.y[j] = f[j] + (0.5 * hx) * gx[j] + std::sqrt(hx) * xi;
        double lpx = logp_path(cx, t, n, f.data()), lpy = logp_path(cx, t, n, pr.y.data());
        if (std::isfinite(lpy)) {
            grad_vertices(cx, t, n, pr.y.data(), gy.data());
            double hy = local_h(P, pr.y, j);
            V3 a = pr.y[j] - f[j] - (0.5 * hx) * gx[j];
            V3 b = f[j] - pr.y[j] - (0.5 * hy) * gy[j];
            // log N(y; x + hx/2 gx, hx) and log N(x; y + hy/2 gy, hy) in 3 dimensions
            double lq_fwd = -1.5 * std::log(hx) - dot(a, a) / (2 * hx);
            double lq_rev = -1.5 * std::log(hy) - dot(b, b) / (2 * hy);
            pr.logA = lpy - lpx + lq_rev - lq_fwd;
        }
        return pr;
    }
    if (j <= n - 2) {
        pr.y[j] = f[j] + P.sigma * box_muller3(u);
    } else {
        pr.move = MV_END;
        V3 d = f[n - 1] - t.eta;
        V3 nu = (1.0 / norm(d)) * d, e2, e3;
        onb(nu, &e2, &e3);
        double k = P.kappa_end;
        double w = 1.0 + std::log(u[0] + (1.0 - u[0]) * std::exp(-2 * k)) / k;
        double phi = 2 * PI * u[1];
        double sw = std::sqrt(std::max(0.0, 1.0 - w * w));
        V3 nn = w * nu + sw * (std::cos(phi) * e2 + std::sin(phi) * e3);
        pr.y[n - 1] = t.eta + t.R * nn;
    }
    pr.logA = logp_path(cx, t, n, pr.y.data()) - logp_path(cx, t, n, f.data());
    return pr;
}

// Metropolis-adjusted Langevin move of all interior vertices jointly:
// y_k = f_k + (h/2) g_k + sqrt(h) xi_k, xi_k from the uniforms U[4(k-1) .. 4(k-1)+3].
Prop propose_mala(const Ctx& cx, const Target& t, const Params& P, const std::vector<V3>& f, const double* U) {
    int n = (int)f.size();
    Prop pr{MV_MALA, f, NEG_INF};
    double h = P.mala_h;
    std::vector<V3> gx(n), gy(n);
    grad_vertices(cx, t, n, f.data(), gx.data());
    for (int k = 1; k <= n - 2; ++k) pr.y[k] = f[k] + (0.5 * h) * gx[k] + std::sqrt(h) * box_muller3(U + 4 * (k - 1));
    double lpx = logp_path(cx, t, n, f.data()), lpy = logp_path(cx, t, n, pr.y.data());
    if (std::isfinite(lpy)) {
        grad_vertices(cx, t, n, pr.y.data(), gy.data());
        double fwd = 0, rev = 0;
        for (int k = 1; k <= n - 2; ++k) {
            V3 a = pr.y[k] - f[k] - (0.5 * h) * gx[k];
            V3 b = f[k] - pr.y[k] - (0.5 * h) * gy[k];
            fwd += dot(a, a);
            rev += dot(b, b);
        }
        pr.logA = lpy - lpx - rev / (2 * h) + fwd / (2 * h);
    }
    return pr;
}

// ---------------------------------------------------------------------------
// Tree coordinates of a path (App. "Path space coordinate system") and the
// global move built on them (Sec. "Path proposal distribution").
// Interval (k, l) with l - k >= 2 places vertex m = floor((k + l) / 2) by
// bi-spherical coordinates about the foci f_k, f_l, with s replaced by
// zeta = artanh(cos s); it then splits into (k, m) and (m, l).  The root is
// (0, n - 1).  The azimuth phi of vertex m is measured in the frame of its
// interval: the root's frame is the orthonormal completion of its axis
// (onb); a child's frame is its parent's frame turned about the parent's
// axis by the parent vertex's phi, then by the rotation that takes the
// parent's axis to the child's.  Vertex m given its ancestors is the
// bi-spherical map of (zeta, t, phi), so the Jacobian of the whole map is the
// product over vertices of gamma^3 sech^2(zeta) / (cosh t - tanh zeta)^3
// (the printed cosh^2 zeta is read as sech^2 zeta: sin s ds = sech^2 zeta dzeta).
// ---------------------------------------------------------------------------
struct TreeNode {
    int k, l, m, parent; // parent: index into the node list (-1: root)
};

std::vector<TreeNode> tree_nodes(int n) {
    std::vector<TreeNode> out;
    std::vector<TreeNode> queue{{0, n - 1, 0, -1}};
    for (size_t q = 0; q < queue.size(); ++q) {
        TreeNode nd = queue[q];
        if (nd.l - nd.k < 2) continue;
        nd.m = (nd.k + nd.l) / 2;
        const int me = (int)out.size();
        out.push_back(nd);
        queue.push_back({nd.k, nd.m, 0, me});
        queue.push_back({nd.m, nd.l, 0, me});
    }
    return out;
}

struct Frame {
    V3 e1, e2, e3;
};

V3 cross3(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// Rodrigues rotation of v about the unit axis a by the angle with cosine c, sine s
V3 rotate_about(V3 v, V3 a, double c, double s) { return c * v + s * cross3(a, v) + ((1 - c) * dot(a, v)) * a; }

Frame child_frame(const Frame& P, double phi_p, V3 e1c) {
    V3 e2r = std::cos(phi_p) * P.e2 + std::sin(phi_p) * P.e3;
    V3 e3r = (-std::sin(phi_p)) * P.e2 + std::cos(phi_p) * P.e3;
    V3 ax = cross3(P.e1, e1c);
    double sn = norm(ax), cs = dot(P.e1, e1c);
    if (!(sn > 0)) return {e1c, e2r, e3r};
    ax = (1.0 / sn) * ax;
    return {e1c, rotate_about(e2r, ax, cs, sn), rotate_about(e3r, ax, cs, sn)};
}

double tree_logjac(double gam, double zeta, double t) {
    return 3 * std::log(gam) + 2 * std::log(1.0 / std::cosh(zeta)) - 3 * std::log(std::cosh(t) - std::tanh(zeta));
}

// Coordinates (zeta, t, phi) of every interior vertex (indexed by vertex) and
// log |d path / d coordinates|.
double tree_coords(const std::vector<V3>& f, std::vector<double>& zeta, std::vector<double>& tt,
                   std::vector<double>& phi) {
    const int n = (int)f.size();
    zeta.assign(n, 0.0);
    tt.assign(n, 0.0);
    phi.assign(n, 0.0);
    std::vector<TreeNode> nodes = tree_nodes(n);
    std::vector<Frame> fr(nodes.size());
    double lj = 0;
    for (size_t i = 0; i < nodes.size(); ++i) {
        const TreeNode& nd = nodes[i];
        V3 A = f[nd.k], B = f[nd.l], x = f[nd.m];
        V3 e1 = (1.0 / norm(B - A)) * (B - A);
        if (nd.parent < 0) {
            fr[i].e1 = e1;
            onb(e1, &fr[i].e2, &fr[i].e3);
        } else {
            fr[i] = child_frame(fr[nd.parent], phi[nodes[nd.parent].m], e1);
        }
        double dA = norm(x - A), dB = norm(x - B);
        double cs = std::max(-1.0, std::min(1.0, dot(A - x, B - x) / (dA * dB)));
        zeta[nd.m] = std::atanh(cs);
        tt[nd.m] = std::log(dA / dB);
        V3 q = x - 0.5 * (A + B);
        phi[nd.m] = std::atan2(dot(q, fr[i].e3), dot(q, fr[i].e2));
        lj += tree_logjac(0.5 * norm(B - A), zeta[nd.m], tt[nd.m]);
    }
    return lj;
}

// The path with end points f0, fend and interior coordinates (zeta, t, phi);
// returns log |d path / d coordinates| through *lj.
std::vector<V3> tree_path(V3 f0, V3 fend, int n, const std::vector<double>& zeta, const std::vector<double>& tt,
                          const std::vector<double>& phi, double* lj) {
    std::vector<V3> f(n);
    f[0] = f0;
    f[n - 1] = fend;
    std::vector<TreeNode> nodes = tree_nodes(n);
    std::vector<Frame> fr(nodes.size());
    *lj = 0;
    for (size_t i = 0; i < nodes.size(); ++i) {
        const TreeNode& nd = nodes[i];
        V3 A = f[nd.k], B = f[nd.l];
        V3 e1 = (1.0 / norm(B - A)) * (B - A);
        if (nd.parent < 0) {
            fr[i].e1 = e1;
            onb(e1, &fr[i].e2, &fr[i].e3);
        } else {
            fr[i] = child_frame(fr[nd.parent], phi[nodes[nd.parent].m], e1);
        }
        const double gam = 0.5 * norm(B - A), z = zeta[nd.m], t = tt[nd.m], p = phi[nd.m];
        V3 dir = std::sinh(t) * e1 + (1.0 / std::cosh(z)) * (std::cos(p) * fr[i].e2 + std::sin(p) * fr[i].e3);
        f[nd.m] = 0.5 * (A + B) + (gam / (std::cosh(t) - std::tanh(z))) * dir;
        *lj += tree_logjac(gam, z, t);
    }
    return f;
}

// The global move: the end point takes a von Mises-Fisher step on the sensor
// (uniforms ue[0..1], as the end-point perturbation), then every interior
// coordinate zeta, t, phi a Gaussian step of variance mala_h / n (three
// normals per vertex k from the uniforms U[4(k-1) .. 4(k-1)+3]); the proposal
// is symmetric in (end point, coordinates), so
// log A = log p(y) - log p(x) + log J(y) - log J(x).
Prop propose_tree(const Ctx& cx, const Target& t, const Params& P, const std::vector<V3>& f, const double ue[2],
                  const double* U) {
    const int n = (int)f.size();
    Prop pr{MV_TREE, f, NEG_INF};
    std::vector<double> z, tt, ph;
    const double ljx = tree_coords(f, z, tt, ph);
    V3 d = f[n - 1] - t.eta;
    V3 nu = (1.0 / norm(d)) * d, e2, e3;
    onb(nu, &e2, &e3);
    const double k = P.kappa_end;
    const double w = 1.0 + std::log(ue[0] + (1.0 - ue[0]) * std::exp(-2 * k)) / k;
    const double sw = std::sqrt(std::max(0.0, 1.0 - w * w));
    const double az = 2 * PI * ue[1];
    V3 yend = t.eta + t.R * (w * nu + sw * (std::cos(az) * e2 + std::sin(az) * e3));
    const double sig = std::sqrt(P.mala_h / n);
    for (int m = 1; m <= n - 2; ++m) {
        V3 xi = box_muller3(U + 4 * (m - 1));
        z[m] += sig * xi.x;
        tt[m] += sig * xi.y;
        ph[m] += sig * xi.z;
    }
    double ljy = 0;
    pr.y = tree_path(f[0], yend, n, z, tt, ph, &ljy);
    const double lpy = logp_path(cx, t, n, pr.y.data());
    if (std::isfinite(lpy) && std::isfinite(ljy)) pr.logA = lpy - logp_path(cx, t, n, f.data()) + ljy - ljx;
    return pr;
}

// Birth of a vertex on segment k of f (n < cap) from the uniforms u[0..2]:
// cos s by the inverse CDF of q(s), t = logit(u1) (logistic q(t)),
// phi = 2 pi u2, new vertex at the bi-spherical point (s, t, phi) of the foci
// f_k, f_{k+1}.
Prop propose_birth(const Ctx& cx, const Target& t, const Params& P, const std::vector<V3>& f, int k,
                   const double u[3]) {
    Prop pr{MV_BIRTH, {}, NEG_INF};
    double beta = centre_beta(cx, t, f[k], f[k + 1]);
    double s = std::acos(std::max(-1.0, std::min(1.0, sample_cos_s(u[0], beta))));
    double tt = std::log(u[1] / (1.0 - u[1]));
    double phi = 2 * PI * u[2];
    V3 fn = bisph(f[k], f[k + 1], s, tt, phi);
    pr.y.assign(f.begin(), f.begin() + k + 1);
    pr.y.push_back(fn);
    pr.y.insert(pr.y.end(), f.begin() + k + 1, f.end());
    pr.logA = log_birth_ratio(cx, t, P, f, k, pr.y, s, tt);
    return pr;
}

// Death of interior vertex j of f (n > 2): the reverse of the birth that
// would create f_j on the segment f_{j-1} f_{j+1} of the shorter path; its
// ratio is the inverse of that birth's (alpha = min(1, 1/A)).
Prop propose_death(const Ctx& cx, const Target& t, const Params& P, const std::vector<V3>& f, int j) {
    Prop pr{MV_DEATH, f, NEG_INF};
    pr.y.erase(pr.y.begin() + j);
    double s, tt, phi;
    bisph_inv(f[j - 1], f[j + 1], f[j], &s, &tt, &phi);
    pr.logA = -log_birth_ratio(cx, t, P, pr.y, j - 1, f, s, tt);
    return pr;
}

// One step of one chain: move selection from the schedule, proposal, Green
// acceptance, update.  The random draws of the step are fixed by (seed,
// chain, step): word 0 chooses the vertex/segment, word 1 is the accept
// uniform, word 2 the birth/death coin, words 4..7 the proposal; the joint
// Langevin move draws one more block per interior vertex k (counter word 3 =
// 2 + k).
StepRec rj_step(const Ctx& cx, const Target& t, const Params& P, uint32_t chain, uint64_t step,
                std::vector<V3>& f, std::vector<V3>* proposal = nullptr) {
    uint32_t r[8];
    step_draws(P.seed, chain, step, r);
    StepRec rec{MV_NULL, 0, -1, NEG_INF, std::log(unif(r[1]))};
    int n = (int)f.size();
    bool perturb = (int)(step % (uint64_t)P.cycle_len) < P.n_perturb;
    const double u4[4] = {unif(r[4]), unif(r[5]), unif(r[6]), unif(r[7])};
    Prop pr{MV_NULL, {}, NEG_INF};
    const bool tree = perturb && P.sampler == 3 && step % (uint64_t)P.cycle_len == 0;
    if (tree) {
        rec.index = -1;
        uint32_t key[2] = {(uint32_t)P.seed, (uint32_t)(P.seed >> 32)};
        std::vector<double> U(4 * std::max(0, n - 2));
        for (int k = 1; k <= n - 2; ++k) {
            uint32_t c[4] = {chain, (uint32_t)step, (uint32_t)(step >> 32), 2u + (uint32_t)k}, q[4];
            philox4x32_10(c, key, q);
            for (int i = 0; i < 4; ++i) U[4 * (k - 1) + i] = unif(q[i]);
        }
        pr = propose_tree(cx, t, P, f, u4, U.data());
    } else if (perturb) {
        int j = 1 + (int)pick(r[0], (uint32_t)(n - 1));
        rec.index = j;
        if (j <= n - 2 && P.sampler == 1) {
            uint32_t key[2] = {(uint32_t)P.seed, (uint32_t)(P.seed >> 32)};
            std::vector<double> U(4 * (n - 2));
            for (int k = 1; k <= n - 2; ++k) {
                uint32_t c[4] = {chain, (uint32_t)step, (uint32_t)(step >> 32), 2u + (uint32_t)k}, q[4];
                philox4x32_10(c, key, q);
                for (int i = 0; i < 4; ++i) U[4 * (k - 1) + i] = unif(q[i]);
            }
            pr = propose_mala(cx, t, P, f, U.data());
        } else {
            pr = propose_perturb(cx, t, P, f, j, u4);
        }
    } else if (r[2] < P.birth_thresh) {
        rec.move = MV_BIRTH;
        if (n >= cx.cap) return rec; // p(n > cap) = 0 (reading R9)
        double S = 0;
        std::vector<double> tb(n - 1);
        for (int l = 0; l + 1 < n; ++l) S += (tb[l] = seg_taub(cx, t, f[l], f[l + 1]));
        if (!(S > 0)) return rec;
        // segment k chosen with probability tau_b(k) / S (reading R8)
        double target = unif(r[0]) * S, cum = 0;
        int k = n - 2;
        for (int l = 0; l + 1 < n; ++l) {
            cum += tb[l];
            if (cum > target) { k = l; break; }
        }
        rec.index = k;
        pr = propose_birth(cx, t, P, f, k, u4);
    } else {
        rec.move = MV_DEATH;
        if (n <= 2) return rec; // no intermediate vertex to remove (reading R9)
        int j = 1 + (int)pick(r[0], (uint32_t)(n - 2));
        rec.index = j;
        pr = propose_death(cx, t, P, f, j);
    }
    rec.move = pr.move;
    rec.logA = pr.logA;
    if (proposal) *proposal = pr.y;
    if (rec.logu < rec.logA) {
        rec.accepted = 1;
        f = pr.y;
    }
    return rec;
}

void accumulate(const Ctx& cx, const Target& t, const std::vector<V3>& f, const StepRec& rec, double* st) {
    int n = (int)f.size();
    double L = path_length(f);
    st[0] += 1;
    st[1] += std::exp(-logw_of(t, n));
    if (n == t.n0) st[2] += std::exp(-logw_of(t, n));
    st[3] += L;
    st[4] += L * L;
    st[5] += n;
    int cls = (rec.move == MV_INTERIOR || rec.move == MV_END || rec.move == MV_MALA || rec.move == MV_LMALA ||
               rec.move == MV_TREE)
                  ? 0
                  : (rec.move == MV_BIRTH ? 1 : 2);
    st[6 + cls] += 1;
    st[9 + cls] += rec.accepted;
    st[12] += (n == cx.cap);
    // a jump that proposed nothing (birth at the cap, death at n = 2): no density was evaluated
    st[15] += (rec.move == MV_BIRTH || rec.move == MV_DEATH) && rec.index < 0;
    if (rec.move == MV_MALA || rec.move == MV_LMALA || rec.move == MV_TREE) {
        st[13] += 1;
        st[14] += rec.accepted;
    }
}

// ---------------------------------------------------------------------------
// Gradients of log p (score of the path density).
// ---------------------------------------------------------------------------
// d/dP and d/dQ of tau_x along P->Q: tau = len * F(uP, uQ) with F the mean
// coefficient along the axis; dF/duP = (F - x(uP)) / (uQ - uP).
void depth_grad(const Medium& m, const std::vector<double>& x, double uP, double uQ, V3 uh, double len, V3* dP,
                V3* dQ) {
    double F = depth(m, x, uP, uQ, len) / len;
    *dP = (-F) * uh;
    *dQ = F * uh;
    if (uP != uQ && layer_of(m, uP) != layer_of(m, uQ)) {
        double dFdP = (F - x[layer_of(m, uP)]) / (uQ - uP);
        double dFdQ = (x[layer_of(m, uQ)] - F) / (uQ - uP);
        *dP = *dP + (len * dFdP) * m.axis;
        *dQ = *dQ + (len * dFdQ) * m.axis;
    }
}

double dlog_sigma_dmu(double mu, double G, double fsl) {
    double hg = p_hg(mu, G), dhg = hg * 1.5 * 2 * G / (1 + G * G - 2 * G * mu);
    double sl = p_sl(mu, G), dsl = (G == 0.0) ? 0.0 : sl * (2.0 / (1.0 / G - 1.0)) / (1 + mu);
    return (fsl * dsl + (1 - fsl) * dhg) / (fsl * sl + (1 - fsl) * hg);
}

double dlog_sigma_dG(double mu, double G, double fsl) {
    // analytic derivative of the HG part; SL part by its closed form
    double den = 1 + G * G - 2 * G * mu;
    double hg = p_hg(mu, G);
    double dhg = 0.5 * (-2 * G) * std::pow(den, -1.5) + 0.5 * (1 - G * G) * (-1.5) * std::pow(den, -2.5) * (2 * G - 2 * mu);
    double sl = p_sl(mu, G), dsl = 0.0;
    if (fsl != 0.0) {
        double dal = 2.0 / ((1 - G) * (1 - G)); // d/dG of the exponent 2G/(1-G)
        dsl = sl * (2.0 / ((1 + G) * (1 - G)) + dal * std::log((1 + mu) / 2));
    }
    return (fsl * dsl + (1 - fsl) * dhg) / (fsl * sl + (1 - fsl) * hg);
}

// d/d(unit vector) helpers: u = r/len, d(u.c)/dr = (c - (u.c) u)/len
V3 dunit_dot(V3 u, double len, V3 c) { return (1.0 / len) * (c - dot(u, c) * u); }

void grad_vertices(const Ctx& cx, const Target& t, int n, const V3* f, V3* g) {
    const Medium& m = cx.media[t.medium];
    for (int k = 0; k < n; ++k) g[k] = {0, 0, 0};
    std::vector<V3> uh(n - 1);
    std::vector<double> len(n - 1);
    for (int k = 0; k + 1 < n; ++k) {
        V3 r = f[k + 1] - f[k];
        len[k] = norm(r);
        uh[k] = (1.0 / len[k]) * r;
        // -tau_a - tau_b - 2 log len of segment k
        double uP = axis_coord(cx, t, f[k]), uQ = axis_coord(cx, t, f[k + 1]);
        V3 aP, aQ, bP, bQ;
        depth_grad(m, m.a, uP, uQ, uh[k], len[k], &aP, &aQ);
        depth_grad(m, m.b, uP, uQ, uh[k], len[k], &bP, &bQ);
        V3 dl_dQ = uh[k];
        g[k] = g[k] - aP - bP + (2.0 / len[k]) * dl_dQ;
        g[k + 1] = g[k + 1] - aQ - bQ - (2.0 / len[k]) * dl_dQ;
    }
    // emission: log eps(u0); only the vMF form depends on the direction
    if (t.ek == 1) {
        V3 d = t.eparam * dunit_dot(uh[0], len[0], t.edir);
        g[1] = g[1] + d;
        g[0] = g[0] - d;
    }
    // turns
    for (int k = 1; k <= n - 2; ++k) {
        int l = layer_of(m, axis_coord(cx, t, f[k]));
        double mu = dot(uh[k - 1], uh[k]);
        double dl = dlog_sigma_dmu(mu, m.g[l], m.fsl[l]);
        V3 dA = dunit_dot(uh[k - 1], len[k - 1], uh[k]); // d mu / d r_{k-1}
        V3 dB = dunit_dot(uh[k], len[k], uh[k - 1]);     // d mu / d r_k
        g[k - 1] = g[k - 1] - dl * dA;
        g[k] = g[k] + dl * dA - dl * dB;
        g[k + 1] = g[k + 1] + dl * dB;
    }
    // end: log(-u_{n-2} . nu) + log rho(nu), nu = (f_{n-1} - eta)/|.|
    V3 d = f[n - 1] - t.eta;
    double dn = norm(d);
    V3 nu = (1.0 / dn) * d;
    double c = -dot(uh[n - 2], nu);
    V3 dc_dr = (-1.0) * dunit_dot(uh[n - 2], len[n - 2], nu); // d c / d r_{n-2}
    V3 dc_dd = (-1.0) * dunit_dot(nu, dn, uh[n - 2]);         // d c / d (f_{n-1} - eta)
    g[n - 2] = g[n - 2] - (1.0 / c) * dc_dr;
    g[n - 1] = g[n - 1] + (1.0 / c) * dc_dr + (1.0 / c) * dc_dd;
    if (t.dk == 1) {
        double cr = dot(nu, t.ddir);
        double dlr = 3.0 - 2.0 * std::tanh(2 * cr + 0.7);
        g[n - 1] = g[n - 1] + dlr * dunit_dot(nu, dn, t.ddir);
    }
    g[0] = {0, 0, 0}; // the source is fixed
}

// d log p / d (per-layer scattering length, absorption length, Gamma).
void grad_params(const Ctx& cx, const Target& t, int n, const V3* f, double* d_lams, double* d_lama, double* d_g) {
    const Medium& m = cx.media[t.medium];
    std::vector<double> Ltot(m.L, 0.0);
    std::vector<double> nsc(m.L, 0.0), dg(m.L, 0.0);
    for (int k = 0; k + 1 < n; ++k)
        layer_lengths(m, axis_coord(cx, t, f[k]), axis_coord(cx, t, f[k + 1]), norm(f[k + 1] - f[k]), Ltot);
    for (int k = 1; k <= n - 2; ++k) {
        int l = layer_of(m, axis_coord(cx, t, f[k]));
        nsc[l] += 1;
        V3 a = f[k] - f[k - 1], b = f[k + 1] - f[k];
        double mu = dot(a, b) / (norm(a) * norm(b));
        dg[l] += dlog_sigma_dG(mu, m.g[l], m.fsl[l]);
    }
    for (int l = 0; l < m.L; ++l) {
        double dla = -Ltot[l];                                             // d/da
        double dlb = (m.b[l] > 0 ? nsc[l] / m.b[l] : 0.0) - Ltot[l];      // d/db
        d_lama[l] = -m.a[l] * m.a[l] * dla; // a = 1/lambda_a
        d_lams[l] = -m.b[l] * m.b[l] * dlb; // b = 1/lambda_s
        d_g[l] = dg[l];
    }
}

// ---------------------------------------------------------------------------
// Anchor integral of the direct sector (n = 2):
//   I_2 = int over directions u hitting the sensor of eps(u) e^{-tau} rho dOmega,
// equal to the n = 2 path integral since dOmega = cos(Phi) dA / r^2.
// Parametrised by v = sqrt(R^2 - D^2 sin^2 theta)/R in [0,1] (smooth in v) and
// the azimuth psi about the source->sensor axis; Gauss-Legendre in v,
// trapezoid (spectrally accurate, periodic) in psi.
// ---------------------------------------------------------------------------
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0);
    w.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(PI * (i + 0.75) / (n + 0.5)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1, p1 = 0;
            for (int j = 1; j <= n; ++j) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2 * j - 1) * z * p1 - (j - 1) * p2) / j;
            }
            dp = n * (z * p0 - p1) / (z * z - 1);
            double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2 / ((1 - z * z) * dp * dp);
    }
}

// Sensor seen from point P (relative to the target source) with angular
// weight wfun(u): returns int_{dirs hitting the sensor} wfun(u) e^{-tau(P->hit)} rho dOmega.
template <class W>
double cap_integral(const Ctx& cx, const Target& t, V3 P, int nv, int npsi, W wfun) {
    const Medium& m = cx.media[t.medium];
    V3 dvec = t.eta - P;
    double D = norm(dvec), R = t.R;
    if (D <= R) return NAN;
    V3 ax = (1.0 / D) * dvec, e2, e3;
    onb(ax, &e2, &e3);
    std::vector<double> gx, gw;
    gauss_legendre(nv, gx, gw);
    double sum = 0;
    for (int i = 0; i < nv; ++i) {
        double v = 0.5 * (gx[i] + 1), wv = 0.5 * gw[i];
        double s2 = (R * R / (D * D)) * (1 - v * v); // sin^2 theta
        double ct = std::sqrt(1 - s2), st = std::sqrt(s2);
        double len = D * ct - R * v;
        double jac = (R * R / (D * D)) * v / ct; // sin theta dtheta = jac dv
        for (int j = 0; j < npsi; ++j) {
            double psi = 2 * PI * (j + 0.5) / npsi;
            V3 u = ct * ax + st * (std::cos(psi) * e2 + std::sin(psi) * e3);
            V3 hit = P + len * u;
            V3 nu = (1.0 / R) * (hit - t.eta);
            double uP = axis_coord(cx, t, P), uQ = axis_coord(cx, t, hit);
            double tau = depth(m, m.a, uP, uQ, len) + depth(m, m.b, uP, uQ, len);
            sum += wv * (2 * PI / npsi) * jac * wfun(u) * std::exp(-tau) * detection(t, nu);
        }
    }
    return sum;
}

double anchor_I2(const Ctx& cx, const Target& t, int nv, int npsi) {
    return cap_integral(cx, t, V3{0, 0, 0}, nv, npsi, [&](V3 u) { return emission(t, u); });
}

// Single-scatter sector (n = 3):
//   I_3 = int dOmega_0 eps(w0) int_0^inf dr e^{-tau(0 -> r w0)} b(r w0) K(r w0),
//   K(P) = int_{sensor seen from P} sigma_sr(w0 . u) e^{-tau(P -> hit)} rho dOmega,
// since d^3 f1 / |f1|^2 = dr dOmega_0.  Nested product Gauss rules: the outer
// direction over the emission support (cone: polar angle in [0, alpha]; else
// the whole sphere), the distance via r = -log(1 - x)/c_ref, and K by the cap
// rule above.
double anchor_I3(const Ctx& cx, const Target& t, int nth, int nps, int nr, int nv, int npsi) {
    const Medium& m = cx.media[t.medium];
    V3 ax = t.ek == 0 ? V3{0, 0, 1} : t.edir, e2, e3;
    onb(ax, &e2, &e3);
    double cmax = (t.ek == 2) ? std::cos(t.eparam) : -1.0;
    std::vector<double> tx, tw, rx, rw;
    gauss_legendre(nth, tx, tw);
    gauss_legendre(nr, rx, rw);
    const double u0 = axis_coord(cx, t, V3{0, 0, 0});
    double sum = 0;
    for (int i = 0; i < nth; ++i) {
        double c0 = 0.5 * (1 - cmax) * tx[i] + 0.5 * (1 + cmax); // cos polar in [cmax, 1]
        double wc = 0.5 * (1 - cmax) * tw[i];
        double s0 = std::sqrt(std::max(0.0, 1 - c0 * c0));
        for (int j = 0; j < nps; ++j) {
            double ps = 2 * PI * (j + 0.5) / nps;
            V3 w0 = c0 * ax + s0 * (std::cos(ps) * e2 + std::sin(ps) * e3);
            double eps = emission(t, w0);
            if (!(eps > 0)) continue;
            // The radial integrand jumps with b(x) and kinks with tau where the
            // ray crosses a layer edge: integrate piece by piece between the
            // crossings; the last, unbounded piece uses r = r_m - log(1-x)/c_m,
            // which maps its exponential attenuation onto [0, 1).
            double du = dot(m.axis, w0);
            std::vector<double> br{0.0};
            if (du != 0)
                for (int k = 1; k < m.L; ++k) {
                    double rk = (m.edge[k] - u0) / du;
                    if (rk > 0) br.push_back(rk);
                }
            std::sort(br.begin(), br.end());
            for (size_t pc = 0; pc < br.size(); ++pc) {
                double a = br[pc];
                if (depth(m, m.a, u0, u0 + du * a, a) + depth(m, m.b, u0, u0 + du * a, a) > 60) break;
                bool last = pc + 1 == br.size();
                int lpc = layer_of(m, u0 + du * (last ? a + 1.0 : 0.5 * (a + br[pc + 1])));
                double cm = m.a[lpc] + m.b[lpc];
                for (int q = 0; q < nr; ++q) {
                    double x = 0.5 * (rx[q] + 1), wx = 0.5 * rw[q], r, drdx;
                    if (!last) {
                        r = a + (br[pc + 1] - a) * x;
                        drdx = br[pc + 1] - a;
                    } else if (cm > 0) {
                        r = a - std::log1p(-x) / cm;
                        drdx = 1.0 / (cm * (1 - x));
                    } else {
                        double L0 = norm(t.eta);
                        r = a + L0 * x / (1 - x);
                        drdx = L0 / ((1 - x) * (1 - x));
                    }
                    V3 f1 = r * w0;
                    if (norm(t.eta - f1) <= t.R * 1.0000001) continue;
                    int l = layer_of(m, axis_coord(cx, t, f1));
                    double uf = axis_coord(cx, t, f1);
                    double tau = depth(m, m.a, u0, uf, r) + depth(m, m.b, u0, uf, r);
                    double K = cap_integral(cx, t, f1, nv, npsi,
                                            [&](V3 u) { return sigma_sr(dot(w0, u), m.g[l], m.fsl[l]); });
                    sum += wc * (2 * PI / nps) * wx * drdx * eps * std::exp(-tau) * m.b[l] * K;
                }
            }
        }
    }
    return sum;
}

// ---------------------------------------------------------------------------
// Relative light yield (Sec. "Comparison of relative light yield", App.
// "Relative light yield transformation").  The ratio B = I_1 / I_0 of the
// intensities of two sensors that share a source and a medium is estimated
// with the geometric bridge estimator
//   B = E_0[sqrt(q_1(x) / q_0(x))] / E_1[sqrt(q_0(x) / q_1(x))],
// q_0(x) = p_0(x), q_1(x) = p_1(T(x)) |dT/dx|, where x are paths ending on
// sensor 0, T maps them onto paths ending on sensor 1, E_0 averages over
// paths sampled on sensor 0 and E_1 over x = T^-1(y) for paths y sampled on
// sensor 1.  Readings: the straight frame (m0, n0, k0) points k0 from the
// source to sensor 0; the cylinder frame has k1 = the emission axis (the
// cylinder's tangent at the source), m1 = minus the unit component of
// B_hat = (eta_1 - f_0)/|.| perpendicular to k1 (the centre of curvature lies
// at f_0 - r_C m1), n1 = k1 x m1, and m0 = the unit component of m1
// perpendicular to k0, n0 = k0 x m0; each interior vertex goes through
// x_bar = (f - f0).m0 / b0, y_bar = (f - f0).n0 / b0, omega = (f - f0).k0 / b0
// to f0 - r_C m1 + (r_C + x_bar b1)(m1 cos(omega Omega) + k1 sin(omega Omega))
// + n1 y_bar b1, whose Jacobian determinant is b1^2 Omega (r_C + x_bar b1) / b0^3
// (the printed product is its inverse); the end point keeps its offset from
// the sensor centre in the rotated arrival frame: nu_1 = Q nu_0 with
// Q m0 = m1 cos(Omega) + k1 sin(Omega), Q n0 = n1, Q k0 = -m1 sin(Omega) +
// k1 cos(Omega), scaled by the radius ratio (area factor (R1/R0)^2), which
// keeps T a bijection.  Paths with a vertex at x_bar b1 <= -r_C or
// |omega Omega| >= pi lie outside the map's domain: q_1 = 0 there.
// ---------------------------------------------------------------------------
struct YieldMap {
    V3 m0, n0, k0, m1, n1, k1;
    V3 eta0, eta1;
    double b0, b1, rC, Om, R0, R1;
    bool ok;
};

YieldMap yield_map(const Target& t0, const Target& t1) {
    YieldMap M{};
    M.eta0 = t0.eta;
    M.eta1 = t1.eta;
    M.R0 = t0.R;
    M.R1 = t1.R;
    double D0 = norm(t0.eta);
    M.k0 = (1.0 / D0) * t0.eta;
    M.b0 = D0 - t0.R;
    V3 B = t1.eta;
    double Bn = norm(B);
    V3 Bh = (1.0 / Bn) * B;
    M.k1 = t0.edir;
    double cpsi = std::max(-1.0, std::min(1.0, dot(M.k1, Bh)));
    V3 c = Bh - cpsi * M.k1;
    double cn = norm(c);
    M.ok = cn > 1e-12;
    if (!M.ok) return M;
    M.m1 = (-1.0 / cn) * c;
    M.n1 = {M.k1.y * M.m1.z - M.k1.z * M.m1.y, M.k1.z * M.m1.x - M.k1.x * M.m1.z, M.k1.x * M.m1.y - M.k1.y * M.m1.x};
    V3 m0 = M.m1 - dot(M.m1, M.k0) * M.k0;
    double mn = norm(m0);
    if (mn < 1e-12) {
        onb(M.k0, &M.m0, &M.n0);
    } else {
        M.m0 = (1.0 / mn) * m0;
        M.n0 = {M.k0.y * M.m0.z - M.k0.z * M.m0.y, M.k0.z * M.m0.x - M.k0.x * M.m0.z,
                M.k0.x * M.m0.y - M.k0.y * M.m0.x};
    }
    double psi = std::acos(cpsi);
    M.rC = Bn / (2.0 * std::sin(psi));
    M.Om = 2.0 * psi - t1.R / M.rC;
    M.b1 = M.rC * M.Om;
    return M;
}

// T of one interior vertex; returns false outside the map's domain.
bool yield_vertex(const YieldMap& M, V3 f, V3* out, double* logjac) {
    double xb = dot(f, M.m0) / M.b0, yb = dot(f, M.n0) / M.b0, om = dot(f, M.k0) / M.b0;
    double rad = M.rC + xb * M.b1, ang = om * M.Om;
    if (!(rad > 0) || !(std::fabs(ang) < PI)) return false;
    *out = (-M.rC) * M.m1 + rad * (std::cos(ang) * M.m1 + std::sin(ang) * M.k1) + (yb * M.b1) * M.n1;
    *logjac += std::log(M.b1 * M.b1 * M.Om * rad / (M.b0 * M.b0 * M.b0));
    return true;
}

// T^-1 of one interior vertex (every point off the cylinder axis has one).
V3 yield_vertex_inv(const YieldMap& M, V3 g, double* logjac) {
    V3 v = g + M.rC * M.m1; // relative to the centre of curvature
    double yb = dot(v, M.n1) / M.b1;
    double pm = dot(v, M.m1), pk = dot(v, M.k1);
    double rad = std::sqrt(pm * pm + pk * pk), ang = std::atan2(pk, pm);
    double xb = (rad - M.rC) / M.b1, om = ang / M.Om;
    *logjac += std::log(M.b1 * M.b1 * M.Om * rad / (M.b0 * M.b0 * M.b0));
    return (xb * M.b0) * M.m0 + (yb * M.b0) * M.n0 + (om * M.b0) * M.k0;
}

V3 yield_end(const YieldMap& M, V3 f, double* logjac) {
    V3 nu = (1.0 / M.R0) * (f - M.eta0);
    V3 r = std::cos(M.Om) * M.m1 + std::sin(M.Om) * M.k1, tg = (-std::sin(M.Om)) * M.m1 + std::cos(M.Om) * M.k1;
    V3 nu1 = dot(nu, M.m0) * r + dot(nu, M.n0) * M.n1 + dot(nu, M.k0) * tg;
    *logjac += 2.0 * std::log(M.R1 / M.R0);
    return M.eta1 + M.R1 * nu1;
}

V3 yield_end_inv(const YieldMap& M, V3 g, double* logjac) {
    V3 nu1 = (1.0 / M.R1) * (g - M.eta1);
    V3 r = std::cos(M.Om) * M.m1 + std::sin(M.Om) * M.k1, tg = (-std::sin(M.Om)) * M.m1 + std::cos(M.Om) * M.k1;
    V3 nu = dot(nu1, r) * M.m0 + dot(nu1, M.n1) * M.n0 + dot(nu1, tg) * M.k0;
    *logjac += 2.0 * std::log(M.R1 / M.R0);
    return M.eta0 + M.R0 * nu;
}

// log(q_1 / q_0) of a sensor-0 path x (side 0) or log(q_0 / q_1) at
// x = T^-1(y) of a sensor-1 path y (side 1); -inf outside the domain.
double yield_log_ratio(const Ctx& cx, int t0, int t1, int side, const std::vector<V3>& f) {
    const Target &A = cx.targets[t0], &B = cx.targets[t1];
    YieldMap M = yield_map(A, B);
    int n = (int)f.size();
    if (!M.ok) return NAN;
    std::vector<V3> g(n);
    g[0] = f[0];
    double lj = 0.0;
    if (side == 0) {
        for (int k = 1; k + 1 < n; ++k)
            if (!yield_vertex(M, f[k], &g[k], &lj)) return NEG_INF;
        g[n - 1] = yield_end(M, f[n - 1], &lj);
        return logp_path(cx, B, n, g.data()) + lj - logp_path(cx, A, n, f.data());
    }
    for (int k = 1; k + 1 < n; ++k) g[k] = yield_vertex_inv(M, f[k], &lj);
    g[n - 1] = yield_end_inv(M, f[n - 1], &lj);
    return logp_path(cx, A, n, g.data()) - logp_path(cx, B, n, f.data()) - lj;
}

// ---------------------------------------------------------------------------
// Analog forward tracer (Algorithm "Ray tracer" of the appendix) with the
// readings R10 (transparent sensor: every entry through the sensor surface
// is scored and the photon continues) and R15 (log-weight starts at 0;
// Russian roulette instead of the 200 m cut, with a generous escape radius).
// Scores the detected intensity per emitted photon.
// ---------------------------------------------------------------------------
struct Rng {
    uint64_t seed;
    uint32_t stream, ctr = 0, buf[4], pos = 4;
    double next() {
        if (pos == 4) {
            uint32_t c[4] = {stream, ctr, 0xA5A5A5A5u, 7u}, k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
            philox4x32_10(c, k, buf);
            ++ctr;
            pos = 0;
        }
        return unif(buf[pos++]);
    }
};

V3 sample_emission(const Target& t, Rng& g) {
    V3 ax = t.ek == 0 ? V3{0, 0, 1} : t.edir, e2, e3;
    onb(ax, &e2, &e3);
    double c;
    if (t.ek == 0) c = 1 - 2 * g.next();
    else if (t.ek == 1) { double u = g.next(); c = 1 + std::log(u + (1 - u) * std::exp(-2 * t.eparam)) / t.eparam; }
    else { double ca = std::cos(t.eparam); c = 1 - g.next() * (1 - ca); }
    double s = std::sqrt(std::max(0.0, 1 - c * c)), ph = 2 * PI * g.next();
    return c * ax + s * (std::cos(ph) * e2 + std::sin(ph) * e3);
}

// cos(theta) from the scattering distribution: HG by its inverse CDF, SL by
// inverting its power-law CDF, mixed by a coin.
double sample_cos_scatter(double G, double fsl, Rng& g) {
    double u = g.next();
    if (fsl > 0 && g.next() < fsl) {
        double al = (G == 0) ? 0.0 : 2.0 / (1.0 / G - 1.0);
        return 2 * std::pow(u, 1.0 / (al + 1)) - 1;
    }
    if (G == 0) return 1 - 2 * u;
    double tmp = (1 - G * G) / (1 - G + 2 * G * u);
    return (1 + G * G - tmp * tmp) / (2 * G);
}

V3 rotate_dir(V3 n, double c, double ph) {
    V3 e2, e3;
    onb(n, &e2, &e3);
    double s = std::sqrt(std::max(0.0, 1 - c * c));
    return c * n + s * (std::cos(ph) * e2 + std::sin(ph) * e3);
}

// Distance along x + s n at which the scattering depth reaches tau_b
// (infinite if never).  Exact for the piecewise-constant layers.
double solve_flight(const Medium& m, double u0, double du, double taub) {
    double s = 0, u = u0;
    int l = layer_of(m, u);
    for (int guard = 0; guard < 100000; ++guard) {
        double dist_to_edge = INFINITY;
        if (du > 0 && l + 1 < m.L) dist_to_edge = (m.edge[l + 1] - u) / du;
        if (du < 0 && l > 0) dist_to_edge = (m.edge[l] - u) / du;
        double need = (m.b[l] > 0) ? taub / m.b[l] : INFINITY;
        if (need <= dist_to_edge) return s + need;
        if (!std::isfinite(dist_to_edge)) return INFINITY;
        taub -= m.b[l] * dist_to_edge;
        s += dist_to_edge;
        u += du * dist_to_edge;
        l += (du > 0) ? 1 : -1;
    }
    return INFINITY;
}

const int NBUCKET = 8; // detected weight split by number of scatterings (last: >= 7)
const int NLBIN = 48;  // detected weight split by path length (bins of a given width; last: overflow)
// Per-photon tallies of the tracer, each summed over photons with its square:
//  [0] detected weight; [1 + b] weight after b scatterings; [9 + b] weight x
//  path length after b scatterings; [17] weight x path length; [18] weight x
//  number of scatterings; [19 + i] weight with path length in bin i.
const int NTALLY = 19 + NLBIN;

// Every sensor entry is scored with the photon's weight and the path length
// L travelled up to the entry point (the photon's arrival time is L over the
// speed of light).  For a homogeneous medium the weight of a detected path is
// e^{-a L}, and the flights are drawn from b e^{-b l}, so the derivatives of
// the detected intensity are the tallies dI/da = -E[w L] and
// dI/db = E[w (N/b - L)] (N scatterings).
void trace_photons(const Ctx& cx, const Target& t, uint64_t seed, uint32_t stream, int64_t nphot, double esc,
                   double lbin, double* S, double* S2) {
    const Medium& m = cx.media[t.medium];
    Rng g{seed, stream, 0, {0, 0, 0, 0}, 4};
    V3 srcu = {0, 0, 0};
    for (int64_t p = 0; p < nphot; ++p) {
        V3 x = srcu, n = sample_emission(t, g);
        double lw = 0.0, Lp = 0.0, T[NTALLY] = {0};
        int nsc = 0;
        for (int it = 0; it < 1000000; ++it) {
            double taub = -std::log(g.next());
            double uX = axis_coord(cx, t, x);
            double dL = solve_flight(m, uX, dot(n, m.axis), taub);
            // sensor entry along [0, dL): ray-sphere intersection, entering side
            V3 oc = x - t.eta;
            double bq = dot(oc, n), cq = dot(oc, oc) - t.R * t.R, disc = bq * bq - cq;
            if (disc > 0) {
                double d = -bq - std::sqrt(disc);
                if (d > 0 && d < dL) {
                    V3 hit = x + d * n;
                    double ta = depth(m, m.a, uX, axis_coord(cx, t, hit), d);
                    double sc = std::exp(lw - ta) * detection(t, (1.0 / t.R) * (hit - t.eta));
                    double Lh = Lp + d;
                    int bk = std::min(nsc, NBUCKET - 1);
                    T[0] += sc;
                    T[1 + bk] += sc;
                    T[9 + bk] += sc * Lh;
                    T[17] += sc * Lh;
                    T[18] += sc * nsc;
                    if (lbin > 0) T[19 + (int)std::min((double)(NLBIN - 1), std::floor(Lh / lbin))] += sc;
                }
            }
            if (!std::isfinite(dL)) break;
            V3 xn = x + dL * n;
            lw -= depth(m, m.a, uX, axis_coord(cx, t, xn), dL);
            Lp += dL;
            x = xn;
            if (norm(x - t.eta) > esc) break;
            if (lw < std::log(1e-4)) { // Russian roulette
                if (g.next() < 0.1) lw += std::log(10.0);
                else break;
            }
            int l = layer_of(m, axis_coord(cx, t, x));
            double c = sample_cos_scatter(m.g[l], m.fsl[l], g);
            n = rotate_dir(n, c, 2 * PI * g.next());
            ++nsc;
        }
        for (int k = 0; k < NTALLY; ++k) {
            S[k] += T[k];
            S2[k] += T[k] * T[k];
        }
    }
}

} // namespace

// ===========================================================================
// C interface for the Python tests (ctypes).
// ===========================================================================
extern "C" {

void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox4x32_10(ctr, key, out); }
void orc_step_draws(uint64_t seed, uint32_t chain, uint64_t step, uint32_t* r) { step_draws(seed, chain, step, r); }
double orc_unif(uint32_t x) { return unif(x); }
double orc_p_hg(double mu, double G) { return p_hg(mu, G); }
double orc_p_sl(double mu, double G) { return p_sl(mu, G); }
double orc_sigma_sr(double mu, double G, double fsl) { return sigma_sr(mu, G, fsl); }
double orc_q_s(double s, double beta) { return q_s(s, beta); }
double orc_q_t(double t) { return q_t(t); }
double orc_jac_bisph(double s, double t, double gam) { return jac_bisph(s, t, gam); }
double orc_kappa_eq(double G) { return kappa_eq(G); }
double orc_sample_cos_s(double u, double beta) { return sample_cos_s(u, beta); }
void orc_bisph(const double* A, const double* B, double s, double t, double phi, double* out) {
    st3(out, bisph(ld3(A), ld3(B), s, t, phi));
}
void orc_bisph_inv(const double* A, const double* B, const double* f, double* stp) {
    bisph_inv(ld3(A), ld3(B), ld3(f), stp, stp + 1, stp + 2);
}
void orc_onb(const double* n, double* e2, double* e3) {
    V3 a, b;
    onb(ld3(n), &a, &b);
    st3(e2, a);
    st3(e3, b);
}

void* orc_create(int n_media, const double* m_axis, const int* m_layer_off, const int* m_layer_cnt,
                 const double* edges, const double* lam_s, const double* lam_a, const double* g,
                 const double* f_sl, int n_targets, const int* t_medium, const double* t_src,
                 const double* t_sensor, const double* t_radius, const int* t_emit_kind, const double* t_emit_dir,
                 const double* t_emit_param, const int* t_det_kind, const double* t_det_dir, const int* t_n0,
                 const double* t_logw /* n_targets * (cap+1) or NULL */, int cap) {
    Ctx* cx = new Ctx;
    cx->cap = cap;
    for (int mi = 0; mi < n_media; ++mi) {
        Medium m;
        m.axis = ld3(m_axis + 3 * mi);
        m.L = m_layer_cnt[mi];
        int off = m_layer_off[mi];
        for (int l = 0; l <= m.L; ++l) m.edge.push_back(edges[off + mi + l]);
        for (int l = 0; l < m.L; ++l) {
            // coefficients are reciprocal lengths; an infinite length means none
            m.a.push_back(std::isinf(lam_a[off + l]) ? 0.0 : 1.0 / lam_a[off + l]);
            m.b.push_back(std::isinf(lam_s[off + l]) ? 0.0 : 1.0 / lam_s[off + l]);
            m.g.push_back(g[off + l]);
            m.fsl.push_back(f_sl[off + l]);
        }
        cx->media.push_back(m);
    }
    for (int ti = 0; ti < n_targets; ++ti) {
        Target t;
        t.src = ld3(t_src + 3 * ti);
        t.eta = ld3(t_sensor + 3 * ti) - t.src;
        t.R = t_radius[ti];
        t.ek = t_emit_kind[ti];
        t.edir = ld3(t_emit_dir + 3 * ti);
        t.eparam = t_emit_param[ti];
        t.dk = t_det_kind[ti];
        t.ddir = ld3(t_det_dir + 3 * ti);
        t.medium = t_medium[ti];
        t.n0 = t_n0[ti];
        if (t_logw) t.logw.assign(t_logw + (size_t)ti * (cap + 1), t_logw + (size_t)(ti + 1) * (cap + 1));
        cx->targets.push_back(t);
    }
    return cx;
}

void orc_destroy(void* h) { delete (Ctx*)h; }

double orc_logp(void* h, int t, int n, const double* v) {
    Ctx* cx = (Ctx*)h;
    std::vector<V3> f(n);
    for (int k = 0; k < n; ++k) f[k] = ld3(v + 3 * k);
    return logp_path(*cx, cx->targets[t], n, f.data());
}

double orc_tau(void* h, int t, const double* P, const double* Q, int which) {
    Ctx* cx = (Ctx*)h;
    const Target& tg = cx->targets[t];
    const Medium& m = cx->media[tg.medium];
    V3 p = ld3(P), q = ld3(Q);
    return depth(m, which == 0 ? m.a : m.b, axis_coord(*cx, tg, p), axis_coord(*cx, tg, q), norm(q - p));
}

double orc_beta(void* h, int t, const double* A, const double* B) {
    Ctx* cx = (Ctx*)h;
    return centre_beta(*cx, cx->targets[t], ld3(A), ld3(B));
}

void orc_grad(void* h, int t, int n, const double* v, double* gv, double* d_lams, double* d_lama, double* d_g) {
    Ctx* cx = (Ctx*)h;
    const Target& tg = cx->targets[t];
    std::vector<V3> f(n), g(n);
    for (int k = 0; k < n; ++k) f[k] = ld3(v + 3 * k);
    grad_vertices(*cx, tg, n, f.data(), g.data());
    for (int k = 0; k < n; ++k) st3(gv + 3 * k, g[k]);
    if (d_lams) grad_params(*cx, tg, n, f.data(), d_lams, d_lama, d_g);
}

// One step of one chain (for lock-step replay against the device).
// v: 3*cap doubles (in/out), n in/out.  rec: move, accepted, index, logA, logu.
// prop (optional, 3*(cap+1) doubles) receives the proposed path, *nprop its
// vertex count (0 when the step made no proposal).
void orc_step(void* h, const uint64_t* ip, const double* dp, uint32_t chain, int t, int* n, double* v,
              double* rec, int* nprop, double* prop) {
    Ctx* cx = (Ctx*)h;
    Params P{ip[0], ip[1], (int64_t)ip[2], (int)ip[3], (int)ip[4], (int)ip[5], (uint32_t)ip[6], dp[0], dp[1],
             (int)ip[7], dp[2]};
    std::vector<V3> f(*n);
    for (int k = 0; k < *n; ++k) f[k] = ld3(v + 3 * k);
    std::vector<V3> y;
    StepRec r = rj_step(*cx, cx->targets[t], P, chain, P.step0, f, prop ? &y : nullptr);
    if (prop) {
        *nprop = (int)y.size();
        for (int k = 0; k < *nprop; ++k) st3(prop + 3 * k, y[k]);
    }
    *n = (int)f.size();
    for (int k = 0; k < *n; ++k) st3(v + 3 * k, f[k]);
    rec[0] = r.move;
    rec[1] = r.accepted;
    rec[2] = r.index;
    rec[3] = r.logA;
    rec[4] = r.logu;
}

// One proposal from continuous draws (tests of the proposal densities).
// kind: 0 perturbation of vertex idx (u: 4 uniforms), 1 birth on segment idx
// (u: 3 uniforms), 2 death of vertex idx, 3 joint Langevin move (u: 4 uniforms
// per interior vertex).  y: room for n + 1 vertices; *ny receives the
// proposal's vertex count (0: no proposal).  Returns log A.
double orc_propose(void* h, const uint64_t* ip, const double* dp, int t, int kind, int n, const double* v, int idx,
                   const double* u, int* ny, double* y, int* move) {
    Ctx* cx = (Ctx*)h;
    Params P{ip[0], ip[1], (int64_t)ip[2], (int)ip[3], (int)ip[4], (int)ip[5], (uint32_t)ip[6], dp[0], dp[1],
             (int)ip[7], dp[2]};
    const Target& tg = cx->targets[t];
    std::vector<V3> f(n);
    for (int k = 0; k < n; ++k) f[k] = ld3(v + 3 * k);
    Prop pr{MV_NULL, {}, NEG_INF};
    if (kind == 0) pr = propose_perturb(*cx, tg, P, f, idx, u);
    else if (kind == 1) pr = propose_birth(*cx, tg, P, f, idx, u);
    else if (kind == 2) pr = propose_death(*cx, tg, P, f, idx);
    else if (kind == 3) pr = propose_mala(*cx, tg, P, f, u);
    else pr = propose_tree(*cx, tg, P, f, u, u + 2);
    *ny = (int)pr.y.size();
    for (int k = 0; k < *ny; ++k) st3(y + 3 * k, pr.y[k]);
    *move = pr.move;
    return pr.logA;
}

// Tree coordinates of a path (n vertices at v): zeta, t, phi (n each, by
// vertex index; 0 at the end points); returns log |d path / d coordinates|.
double orc_tree_coords(int n, const double* v, double* zeta, double* t, double* phi) {
    std::vector<V3> f(n);
    for (int k = 0; k < n; ++k) f[k] = ld3(v + 3 * k);
    std::vector<double> z, tt, ph;
    double lj = tree_coords(f, z, tt, ph);
    for (int k = 0; k < n; ++k) {
        zeta[k] = z[k];
        t[k] = tt[k];
        phi[k] = ph[k];
    }
    return lj;
}

// The path of n vertices with end points f0, fend and interior coordinates
// (zeta, t, phi by vertex index) into out (3n); returns the log-Jacobian.
double orc_tree_path(int n, const double* f0, const double* fend, const double* zeta, const double* t,
                     const double* phi, double* out) {
    std::vector<double> z(zeta, zeta + n), tt(t, t + n), ph(phi, phi + n);
    double lj = 0;
    std::vector<V3> f = tree_path(ld3(f0), ld3(fend), n, z, tt, ph, &lj);
    for (int k = 0; k < n; ++k) st3(out + 3 * k, f[k]);
    return lj;
}

// Run `steps` steps for chains [0, C): per-chain state in/out, per-chain
// statistics added into stats (C * 16).  Chains are split over threads.
// trace (optional): C * steps * 5 doubles, record of every step.
void orc_run(void* h, const uint64_t* ip, const double* dp, int C, const int* chain_id, const int* target, int* n,
             double* v /* C*cap*3 */, double* stats, double* trace, int nthreads) {
    Ctx* cx = (Ctx*)h;
    Params P{ip[0], ip[1], (int64_t)ip[2], (int)ip[3], (int)ip[4], (int)ip[5], (uint32_t)ip[6], dp[0], dp[1],
             (int)ip[7], dp[2]};
    int cap = cx->cap;
    std::atomic<int> next(0);
    auto work = [&]() {
        for (;;) {
            int c = next.fetch_add(1);
            if (c >= C) break;
            const Target& t = cx->targets[target[c]];
            std::vector<V3> f(n[c]);
            double* vc = v + (size_t)c * cap * 3;
            for (int k = 0; k < n[c]; ++k) f[k] = ld3(vc + 3 * k);
            for (int s = 0; s < P.steps; ++s) {
                uint64_t step = P.step0 + (uint64_t)s;
                StepRec r = rj_step(*cx, t, P, (uint32_t)chain_id[c], step, f);
                if (trace) {
                    double* tr = trace + ((size_t)c * P.steps + s) * 5;
                    tr[0] = r.move; tr[1] = r.accepted; tr[2] = r.index; tr[3] = r.logA; tr[4] = r.logu;
                }
                if ((int64_t)step >= P.burn_in) accumulate(*cx, t, f, r, stats + (size_t)c * NSTAT);
            }
            n[c] = (int)f.size();
            for (int k = 0; k < n[c]; ++k) st3(vc + 3 * k, f[k]);
        }
    };
    if (nthreads <= 1) {
        work();
    } else {
        std::vector<std::thread> th;
        for (int i = 0; i < nthreads; ++i) th.emplace_back(work);
        for (auto& x : th) x.join();
    }
}

double orc_anchor_I2(void* h, int t, int nv, int npsi) {
    Ctx* cx = (Ctx*)h;
    return anchor_I2(*cx, cx->targets[t], nv, npsi);
}

double orc_anchor_I3(void* h, int t, int nth, int nps, int nr, int nv, int npsi) {
    Ctx* cx = (Ctx*)h;
    return anchor_I3(*cx, cx->targets[t], nth, nps, nr, nv, npsi);
}

// Analog tracer: per-photon mean and standard error of every tally
// (mean_se[2k], mean_se[2k + 1] for tally k = 0 .. NTALLY-1, see
// trace_photons).  nphot photons split over nthreads independent streams;
// lbin: path-length bin width of the length tallies (0: none).
void orc_trace(void* h, int t, uint64_t seed, int64_t nphot, double esc, double lbin, int nthreads,
               double* mean_se) {
    Ctx* cx = (Ctx*)h;
    std::vector<double> S((size_t)nthreads * NTALLY, 0), S2((size_t)nthreads * NTALLY, 0);
    std::vector<std::thread> th;
    for (int i = 0; i < nthreads; ++i) {
        int64_t cnt = nphot / nthreads + (i < nphot % nthreads ? 1 : 0);
        th.emplace_back([&, i, cnt]() {
            trace_photons(*cx, cx->targets[t], seed, (uint32_t)i, cnt, esc, lbin, &S[(size_t)i * NTALLY],
                          &S2[(size_t)i * NTALLY]);
        });
    }
    for (auto& x : th) x.join();
    for (int k = 0; k < NTALLY; ++k) {
        double A = 0, A2 = 0;
        for (int i = 0; i < nthreads; ++i) {
            A += S[(size_t)i * NTALLY + k];
            A2 += S2[(size_t)i * NTALLY + k];
        }
        double mean = A / nphot;
        mean_se[2 * k] = mean;
        mean_se[2 * k + 1] = std::sqrt(std::max(0.0, A2 / nphot - mean * mean) / nphot);
    }
}

int orc_trace_tallies(void) { return NTALLY; }

// Relative light yield helpers: the map T between the paths of targets t0 and
// t1 (kind 0: forward, 1: inverse; v / out n vertices, returns log |det| of
// the forward map at the sensor-0 path, NaN outside its domain) and the
// per-path bridge log-ratio (side 0: log q1/q0 of a sensor-0 path; side 1:
// log q0/q1 of a sensor-1 path).
double orc_yield_map(void* h, int t0, int t1, int kind, int n, const double* v, double* out) {
    Ctx* cx = (Ctx*)h;
    YieldMap M = yield_map(cx->targets[t0], cx->targets[t1]);
    if (!M.ok) return NAN;
    std::vector<V3> f(n);
    for (int k = 0; k < n; ++k) f[k] = ld3(v + 3 * k);
    double lj = 0.0;
    st3(out, f[0]);
    for (int k = 1; k + 1 < n; ++k) {
        V3 g;
        if (kind == 0) {
            if (!yield_vertex(M, f[k], &g, &lj)) return NAN;
        } else {
            g = yield_vertex_inv(M, f[k], &lj);
        }
        st3(out + 3 * k, g);
    }
    st3(out + 3 * (n - 1), kind == 0 ? yield_end(M, f[n - 1], &lj) : yield_end_inv(M, f[n - 1], &lj));
    return lj;
}

double orc_yield_log_ratio(void* h, int t0, int t1, int side, int n, const double* v) {
    Ctx* cx = (Ctx*)h;
    std::vector<V3> f(n);
    for (int k = 0; k < n; ++k) f[k] = ld3(v + 3 * k);
    return yield_log_ratio(*cx, t0, t1, side, f);
}

} // extern "C"
