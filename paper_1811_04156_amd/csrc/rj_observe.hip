// rj_observe.hip -- estimators evaluated on snapshots of the chains' current
// paths (between sampler launches):
//  - the relative light yield of two sensors of one source by the geometric
//    bridge estimator over the cylinder map T (Sec. "Comparison of relative
//    light yield"; App. "Relative light yield transformation");
//  - per-target path-length histograms (Sec. "Comparison of timing
//    distributions": the arrival time is the path length over the speed of
//    light in the bulk).
// Both weight a chain by 1/w(n) so that tilted chains estimate untilted
// expectations, and both sum a block's lanes into an LDS table when the block
// covers at most two keys (targets are contiguous in the chain array), else
// add per lane.
#include <hip/hip_runtime.h>

#include "rj_kernels.h"
#include "rj_step.h"
#include "rj_wave.h"

namespace rj {

namespace {

constexpr int BLK = 256;

__device__ __forceinline__ uint32_t group_hash(uint32_t x) {
    // the chain -> jackknife group hash of the intensity estimator
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

using D3 = V3<double>;

__device__ __forceinline__ D3 cross(D3 a, D3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ D3 unit(D3 a) { return (1.0 / sqrt(dot(a, a))) * a; }
__device__ __forceinline__ D3 ld3(const double* p) { return {p[0], p[1], p[2]}; }

// ---------------------------------------------------------------------------
// The map T from paths ending on sensor 0 (target t0) to paths ending on
// sensor 1 (target t1) of the same source, in FP64.
//  Straight frame: k0 points from the source to sensor 0's centre, b0 = the
//  distance to its surface; interior vertex f has coordinates
//  (xbar, ybar, omega) = (f.m0, f.n0, f.k0) / b0.
//  Cylinder frame: k1 = the emission axis, the cylinder's tangent at the
//  source; m1 = minus the unit part of (sensor 1 - source) normal to k1, so the
//  axis of curvature passes through -r_C m1; n1 = k1 x m1; m0 = the unit part
//  of m1 normal to k0 and n0 = k0 x m0.  r_C = |B| / (2 sin psi) with
//  cos psi = k1 . B_hat puts sensor 1's centre on the circle at angle 2 psi;
//  Omega = 2 psi - R1 / r_C stops the image of the axis one sensor radius of
//  arc short of it, and b1 = r_C Omega.
//  Interior vertex: f -> -r_C m1 + (r_C + xbar b1)(cos(omega Omega) m1 +
//  sin(omega Omega) k1) + ybar b1 n1, with |dT/df| = b1^2 Omega (r_C + xbar b1) / b0^3;
//  defined for r_C + xbar b1 > 0 and |omega Omega| < pi.
//  End point: its offset from sensor 0's centre, in units of R0, is turned by
//  the rotation taking (m0, n0, k0) to the arrival frame (cos Omega m1 +
//  sin Omega k1, n1, -sin Omega m1 + cos Omega k1) and scaled to R1; the
//  surface element scales by (R1 / R0)^2.
// ---------------------------------------------------------------------------
struct YMap {
    D3 m0, n0, k0, m1, n1, k1, ar, at, e0, e1;
    double b0, b1, rC, Om, R0, R1, lc, le;
    bool ok;
};

__device__ YMap ymap(const KArgs& a, int t0, int t1) {
    YMap M;
    const D3 s0 = ld3(a.src + 3 * t0);
    M.e0 = ld3(a.sensor + 3 * t0) - s0;
    M.e1 = ld3(a.sensor + 3 * t1) - ld3(a.src + 3 * t1);
    M.R0 = a.radius[t0];
    M.R1 = a.radius[t1];
    const double D0 = sqrt(dot(M.e0, M.e0));
    M.k0 = (1.0 / D0) * M.e0;
    M.b0 = D0 - M.R0;
    const double Bn = sqrt(dot(M.e1, M.e1));
    const D3 Bh = (1.0 / Bn) * M.e1;
    M.k1 = unit(ld3(a.edir + 3 * t0));
    const double cpsi = fmin(1.0, fmax(-1.0, dot(M.k1, Bh)));
    const D3 c = Bh - cpsi * M.k1;
    const double cn = sqrt(dot(c, c));
    const D3 mk = c - dot(c, M.k0) * M.k0; // m1 is -c / |c|: its part normal to k0 is -mk / |c|
    const double mkn = sqrt(dot(mk, mk));
    M.ok = cn > 1e-12 && mkn > 1e-12 * cn && M.b0 > 0;
    if (!M.ok) return M;
    M.m1 = (-1.0 / cn) * c;
    M.n1 = cross(M.k1, M.m1);
    M.m0 = (-1.0 / mkn) * mk;
    M.n0 = cross(M.k0, M.m0);
    const double psi = acos(cpsi);
    M.rC = Bn / (2.0 * sin(psi));
    M.Om = 2.0 * psi - M.R1 / M.rC;
    M.b1 = M.rC * M.Om;
    const double cO = cos(M.Om), sO = sin(M.Om);
    M.ar = cO * M.m1 + sO * M.k1;
    M.at = (-sO) * M.m1 + cO * M.k1;
    M.lc = log(M.b1 * M.b1 * M.Om / (M.b0 * M.b0 * M.b0));
    M.le = 2.0 * log(M.R1 / M.R0);
    M.ok = M.Om > 0 && M.b1 > 0;
    return M;
}

// forward image of an interior vertex; rad <= 0 or |angle| >= pi: outside
__device__ __forceinline__ D3 yfwd(const YMap& M, D3 f, double& rad, bool& in) {
    const double ib0 = 1.0 / M.b0;
    const double xb = dot(f, M.m0) * ib0, yb = dot(f, M.n0) * ib0, om = dot(f, M.k0) * ib0;
    rad = M.rC + xb * M.b1;
    const double ang = om * M.Om;
    in = rad > 0 && fabs(ang) < 3.14159265358979323846;
    double sa, ca;
    sincos(ang, &sa, &ca);
    return (-M.rC) * M.m1 + rad * (ca * M.m1 + sa * M.k1) + (yb * M.b1) * M.n1;
}

__device__ __forceinline__ D3 yinv(const YMap& M, D3 g, double& rad) {
    const D3 v = g + M.rC * M.m1;
    const double pm = dot(v, M.m1), pk = dot(v, M.k1);
    rad = sqrt(pm * pm + pk * pk);
    const double xb = (rad - M.rC) / M.b1, yb = dot(v, M.n1) / M.b1, om = atan2(pk, pm) / M.Om;
    return (xb * M.b0) * M.m0 + (yb * M.b0) * M.n0 + (om * M.b0) * M.k0;
}

__device__ __forceinline__ D3 yend_fwd(const YMap& M, D3 f) {
    const D3 nu = f - M.e0;
    const double s = M.R1 / M.R0;
    return M.e1 + s * (dot(nu, M.m0) * M.ar + dot(nu, M.n0) * M.n1 + dot(nu, M.k0) * M.at);
}

__device__ __forceinline__ D3 yend_inv(const YMap& M, D3 g) {
    const D3 nu = g - M.e1;
    const double s = M.R0 / M.R1;
    return M.e0 + s * (dot(nu, M.ar) * M.m0 + dot(nu, M.n1) * M.n0 + dot(nu, M.at) * M.k0);
}

template <class R> __device__ __forceinline__ D3 vload(const Vtx<R>* base, size_t C, int v) {
    const Vtx<R> x = base[(size_t)v * C];
    return {(double)x.x, (double)x.y, (double)x.z};
}

// The chain's path seen through T (dir 0) or T^-1 (dir 1), vertex by vertex.
template <class R> struct MappedPath {
    const Vtx<R>* glb;
    size_t C;
    int n, dir;
    const YMap* M;
    __device__ __forceinline__ V3<R> p(int v) const {
        const D3 f = vload(glb, C, v);
        D3 g;
        double rad;
        bool in;
        if (v == 0)
            g = f;
        else if (v == n - 1)
            g = dir == 0 ? yend_fwd(*M, f) : yend_inv(*M, f);
        else
            g = dir == 0 ? yfwd(*M, f, rad, in) : yinv(*M, f, rad);
        return {(R)g.x, (R)g.y, (R)g.z};
    }
    __device__ __forceinline__ void stw(int, R) const {}
};

// Block-level accumulation of (key, group, slot) sums: an LDS table when the
// block's keys span at most two values, else one atomic per lane.
struct BlockSums {
    double* tab;
    int kmin;
    bool local;
};

__device__ __forceinline__ BlockSums block_sums_begin(int key, double* tab, int nent_per_key, int* smin, int* smax) {
    BlockSums b;
    b.tab = tab;
    b.kmin = block_min_i32(key < 0 ? 0x7fffffff : key, smin);
    const int kmax = block_max_i32(key, smax);
    b.local = kmax >= 0 && kmax - b.kmin <= 1 && tab != nullptr;
    if (b.local) {
        for (int i = threadIdx.x; i < 2 * nent_per_key; i += blockDim.x) tab[i] = 0.0;
    }
    __syncthreads();
    return b;
}

__device__ __forceinline__ void block_sums_end(const BlockSums& b, double* out, int nent_per_key, int nkeys) {
    if (!b.local) return;
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * nent_per_key; i += blockDim.x) {
        const int k = b.kmin + i / nent_per_key;
        if (b.tab[i] != 0.0 && k < nkeys) atomicAdd(out + (size_t)b.kmin * nent_per_key + i, b.tab[i]);
    }
}

// ---------------------------------------------------------------------------
// Bridge sums.  role[t] = 2 k + side for a target in pair k (pairs[2k] = t0,
// pairs[2k + 1] = t1), else -1.  A chain of t0 (path x) takes
// log r = log p_t1(T x) + log|dT/dx| - log p_t0(x) (-inf outside T's domain);
// a chain of t1 (path y) takes log r = log p_t0(T^-1 y) - log p_t1(y) - log|dT/dx|
// at x = T^-1 y.  acc[((k * 2 + side) * groups + g) * 2 + {0, 1}] += {sqrt(r), 1} / w(n).
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(BLK) yield_kernel(KArgs a, int n_pairs, const int32_t* pairs, const int32_t* role,
                                                    int groups, double* acc, double* logr) {
    __shared__ double tab[2 * 64 * 2];
    __shared__ int smin[BLK / 64], smax[BLK / 64];
    const int c = blockIdx.x * BLK + threadIdx.x;
    int key = -1, tc = -1, to = -1, side = 0, n = 0;
    if (c < a.C) {
        tc = a.target[c];
        n = a.n[c];
        if (tc >= 0 && tc < a.T && a.status[c] == 0 && n >= 2 && n <= a.cap) {
            const int r = role[tc];
            const int k = r >> 1;
            if (r >= 0 && k < n_pairs && pairs[r] == tc) {
                side = r & 1;
                to = pairs[2 * k + (side ^ 1)];
                if (to >= 0 && to < a.T && to != tc && a.medium[to] == a.medium[tc] &&
                    a.medium[tc] >= 0 && a.medium[tc] < a.n_media && a.src[3 * to] == a.src[3 * tc] &&
                    a.src[3 * to + 1] == a.src[3 * tc + 1] && a.src[3 * to + 2] == a.src[3 * tc + 2])
                    key = r;
            }
        }
        if (logr) logr[c] = __builtin_nan("");
    }
    double lr = __builtin_nan("");
    if (key >= 0) {
        const int t0 = side == 0 ? tc : to, t1 = side == 0 ? to : tc;
        const YMap M = ymap(a, t0, t1);
        if (M.ok) {
            const Vtx<R>* base = (const Vtx<R>*)a.verts + c;
            const size_t C = (size_t)a.C;
            // log |dT/dx| and the domain of T (side 0)
            double lj = M.le + (n - 2) * M.lc;
            bool in = true;
            for (int v = 1; v + 1 < n; ++v) {
                double rad;
                bool inv = true;
                if (side == 0)
                    yfwd(M, vload(base, C, v), rad, inv);
                else
                    yinv(M, vload(base, C, v), rad);
                in = in && inv;
                lj += log(rad);
            }
            Tgt<R> T0, T1;
            load_target(a, t0, T0, hbm_tab<R>(a));
            load_target(a, t1, T1, hbm_tab<R>(a));
            double L;
            const GlobalPath<R> own{(Vtx<R>*)base, C};
            const MappedPath<R> img{base, C, n, side, &M};
            if (side == 0) {
                const double lp0 = full_logp(T0, own, n, L);
                lr = in ? full_logp(T1, img, n, L) + lj - lp0 : -__builtin_inf();
            } else {
                const double lp1 = full_logp(T1, own, n, L);
                lr = full_logp(T0, img, n, L) - lp1 - lj;
            }
            if (lr != lr || lr == __builtin_inf()) key = -1; // a non-finite own density: not a sample
        } else {
            key = -1;
        }
        if (logr && c < a.C) logr[c] = lr;
    }
    const int g = (int)(group_hash((uint32_t)c) % (uint32_t)groups);
    const int nent = groups * 2;
    BlockSums b = block_sums_begin(key, tab, nent, smin, smax);
    if (key >= 0) {
        const double* lw = a.logw ? a.logw + (size_t)tc * (a.cap + 1) : nullptr;
        const double iw = lw ? exp(-lw[n]) : 1.0;
        const double s = lr == -__builtin_inf() ? 0.0 : exp(0.5 * lr);
        double* dst = b.local ? tab + (size_t)(key - b.kmin) * nent : acc + (size_t)key * nent;
        atomicAdd(dst + 2 * g, iw * s);
        atomicAdd(dst + 2 * g + 1, iw);
    }
    block_sums_end(b, acc, nent, 2 * n_pairs);
}

// ---------------------------------------------------------------------------
// Path-length histogram: hist[t * (bins + 1) + b] += 1 / w(n) for
// b = floor((L - l0) / width) in [0, bins), and hist[t * (bins + 1) + bins]
// += 1 / w(n) for every sample (the normaliser).  L is summed in FP64.
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(BLK) lhist_kernel(KArgs a, int bins, double l0, double width, double* hist,
                                                    int use_lds) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int smin[BLK / 64], smax[BLK / 64];
    const int c = blockIdx.x * BLK + threadIdx.x;
    int t = -1, n = 0;
    if (c < a.C) {
        t = a.target[c];
        n = a.n[c];
        if (t < 0 || t >= a.T || a.status[c] != 0 || n < 2 || n > a.cap) t = -1;
    }
    double L = 0;
    if (t >= 0) {
        const Vtx<R>* base = (const Vtx<R>*)a.verts + c;
        D3 p = vload(base, (size_t)a.C, 0);
        for (int v = 1; v < n; ++v) {
            const D3 q = vload(base, (size_t)a.C, v);
            const D3 d = q - p;
            L += sqrt(dot(d, d));
            p = q;
        }
    }
    const int nent = bins + 1;
    BlockSums b = block_sums_begin(t, use_lds ? (double*)smem : nullptr, nent, smin, smax);
    if (t >= 0) {
        const double* lw = a.logw ? a.logw + (size_t)t * (a.cap + 1) : nullptr;
        const double iw = lw ? exp(-lw[n]) : 1.0;
        double* dst = b.local ? (double*)smem + (size_t)(t - b.kmin) * nent : hist + (size_t)t * nent;
        const double x = floor((L - l0) / width);
        if (x >= 0 && x < (double)bins) atomicAdd(dst + (int)x, iw);
        atomicAdd(dst + bins, iw);
    }
    block_sums_end(b, hist, nent, a.T);
}

} // namespace

hipError_t launch_yield(const KArgs& a, int n_pairs, const int32_t* pairs, const int32_t* role, int groups,
                        double* acc, double* logr, hipStream_t s) {
    const int grid = (a.C + BLK - 1) / BLK;
    if (a.prec == RJPATH_F64)
        hipLaunchKernelGGL(yield_kernel<double>, dim3(grid), dim3(BLK), 0, s, a, n_pairs, pairs, role, groups, acc,
                           logr);
    else
        hipLaunchKernelGGL(yield_kernel<float>, dim3(grid), dim3(BLK), 0, s, a, n_pairs, pairs, role, groups, acc,
                           logr);
    return hipGetLastError();
}

hipError_t launch_lhist(const KArgs& a, int bins, double l0, double width, double* hist, hipStream_t s) {
    const int grid = (a.C + BLK - 1) / BLK;
    const size_t lds = 2 * sizeof(double) * ((size_t)bins + 1);
    const int use = lds <= 64 * 1024;
    if (a.prec == RJPATH_F64)
        hipLaunchKernelGGL(lhist_kernel<double>, dim3(grid), dim3(BLK), use ? lds : 0, s, a, bins, l0, width, hist,
                           use);
    else
        hipLaunchKernelGGL(lhist_kernel<float>, dim3(grid), dim3(BLK), use ? lds : 0, s, a, bins, l0, width, hist,
                           use);
    return hipGetLastError();
}

} // namespace rj
