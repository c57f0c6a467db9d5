// rj_sampler.hip -- the score kernel (log p, vertex gradients and parameter
// score of the current paths), the device step counter and the dispatch of
// the step-kernel variants (rj_step.h, rj_run.h).
#include <hip/hip_runtime.h>

#include "rj_step.h"
#include "rj_wave.h"

namespace rj {

// ---------------------------------------------------------------------------
// Score kernel: log p, d log p / d vertices and the per-layer parameter score.
// The score sums of a block whose chains belong to at most two targets are
// accumulated in an LDS table (1 + 3 L_total doubles per target) and flushed
// with one global atomic per non-zero entry; other blocks add per lane.
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(256) grad_kernel(KArgs a, double* logp_out, Vtx<R>* dv, double* score,
                                                   int L_total, int lds_rows, int lweight) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int tmin_s[4], tmax_s[4];
    double* tab = (double*)smem;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t C = (size_t)a.C;
    const size_t row = 1 + 3 * (size_t)L_total;
    int t = -1, n = 0;
    if (c < a.C) {
        t = a.target[c];
        n = a.n[c];
        if (t < 0 || t >= a.T || n < 2 || n > a.cap || a.medium[t] < 0 || a.medium[t] >= a.n_media) {
            if (logp_out) logp_out[c] = __builtin_nan("");
            t = -1;
        }
    }
    // block-uniform choice of the score destination
    bool local = false;
    int tmin = 0;
    if (score && lds_rows > 0) {
        tmin = block_min_i32(t < 0 ? 0x7fffffff : t, tmin_s);
        const int tmax = block_max_i32(t, tmax_s);
        local = tmax >= 0 && tmax - tmin < lds_rows;
        if (local) {
            for (size_t i = threadIdx.x; i < (size_t)lds_rows * row; i += blockDim.x) tab[i] = 0.0;
            __syncthreads();
        }
    }
    if (t >= 0) {
        GlobalPath<R> ps{(Vtx<R>*)a.verts + c, C};
        Tgt<R> T;
        load_target(a, t, T, hbm_tab<R>(a));
        double lp = score_stream(T, ps, n, [&](int k, V3<R> g) {
            if (dv) dv[(size_t)k * C + c] = Vtx<R>{k > 0 ? g.x : (R)0, k > 0 ? g.y : (R)0, k > 0 ? g.z : (R)0, (R)0};
        });
        if (logp_out) logp_out[c] = lp;
        if (score && isfinite(lp) && a.status[c] == 0) {
            const int off = a.minfo[a.medium[t]].off;
            const double* logw = a.logw ? a.logw + (size_t)t * (a.cap + 1) : nullptr;
            double iw = logw ? exp(-logw[n]) : 1.0;
            if (lweight) {
                // weight by the path length (FP64 sum of the segment lengths)
                double Lp = 0.0;
                for (int k = 1; k < n; ++k) {
                    const V3<R> d = ps.p(k) - ps.p(k - 1);
                    Lp += sqrt((double)dot(d, d));
                }
                iw *= Lp;
            }
            double* sc = local ? tab + (size_t)(t - tmin) * row : score + (size_t)t * row;
            atomicAdd(sc, iw);
            // d/d lambda_s = -b^2 d/db, d/d lambda_a = -a^2 d/da, with d log p/da = -L_l and
            // d log p/db = N_l / b - L_l (L_l: path length in layer l, N_l: scatterings in l)
            V3<R> fprev = ps.p(0);
            Seg<R> sprev;
            for (int k = 1; k < n; ++k) {
                V3<R> fc = ps.p(k);
                Seg<R> s = make_seg(T, fprev, fc);
                double uP = axis_u(T, fprev), uQ = axis_u(T, fc);
                int lP = layer_u(T, uP), lQ = layer_u(T, uQ);
                double lo = uP < uQ ? uP : uQ, hi = uP < uQ ? uQ : uP;
                int llo = lP < lQ ? lP : lQ, lhi = lP < lQ ? lQ : lP;
                double scl = lP == lQ ? 0.0 : (double)s.len / (hi - lo);
                for (int l = llo; l <= lhi; ++l) {
                    double Lin = lP == lQ ? (double)s.len
                                          : ((l == lhi ? hi : T.edge[l + 1]) - (l == llo ? lo : T.edge[l])) * scl;
                    const LayV<R> ly = lay_at(T, l);
                    double av = (double)ly.a, bv = (double)ly.b;
                    atomicAdd(sc + 1 + 3 * (off + l) + 0, iw * (bv * bv * Lin));
                    atomicAdd(sc + 1 + 3 * (off + l) + 1, iw * (av * av * Lin));
                }
                if (k >= 2) {
                    int l = layer_at(T, fprev);
                    const LayV<R> ly = lay_at(T, l);
                    double bv = (double)ly.b, g = (double)ly.g, fsl = (double)ly.fsl;
                    V3<R> dd = sprev.u - s.u;
                    double q = (double)dot(dd, dd);
                    double mu = 1.0 - 0.5 * q;
                    double den = (1 - g) * (1 - g) + g * q;
                    double dhg = -2 * g / (1 - g * g) - 3 * (g - mu) / den;
                    double dg = dhg;
                    if (fsl != 0.0) {
                        const double PI = 3.14159265358979323846;
                        double lhg = log((1 - g * g) / (4 * PI)) - 1.5 * log(den);
                        double lsl = log((1 + g) / (1 - g) / (4 * PI)) + 2 * g / (1 - g) * log(0.5 * (1 + mu));
                        double dsl = 2.0 / ((1 + g) * (1 - g)) + 2.0 / ((1 - g) * (1 - g)) * log(0.5 * (1 + mu));
                        double m = lhg > lsl ? lhg : lsl;
                        double es = fsl * exp(lsl - m), eh = (1 - fsl) * exp(lhg - m);
                        dg = (es * dsl + eh * dhg) / (es + eh);
                    }
                    atomicAdd(sc + 1 + 3 * (off + l) + 0, iw * (-bv)); // log b at a scattering vertex
                    atomicAdd(sc + 1 + 3 * (off + l) + 2, iw * dg);
                }
                sprev = s;
                fprev = fc;
            }
        }
    }
    if (local) {
        __syncthreads();
        for (size_t i = threadIdx.x; i < (size_t)lds_rows * row; i += blockDim.x) {
            const size_t tt = tmin + i / row;
            if (tab[i] != 0.0 && tt < (size_t)a.T) atomicAdd(score + (size_t)tmin * row + i, tab[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_run(const KArgs& a, int block, hipStream_t s) {
    if (a.prec == RJPATH_F64) {
        if (a.sampler == RJPATH_MALA) return launch_run_v<double, 1>(a, block, s);
        if (a.sampler == RJPATH_LMALA) return launch_run_v<double, 2>(a, block, s);
        if (a.sampler == RJPATH_TREE) return launch_run_v<double, 3>(a, block, s);
        return launch_run_v<double, 0>(a, block, s);
    }
    if (a.sampler == RJPATH_MALA) return launch_run_v<float, 1>(a, block, s);
    if (a.sampler == RJPATH_LMALA) return launch_run_v<float, 2>(a, block, s);
    if (a.sampler == RJPATH_TREE) return launch_run_v<float, 3>(a, block, s);
    return launch_run_v<float, 0>(a, block, s);
}

hipError_t set_run_lds_limit() {
    hipError_t e = set_lds_limit_v<float, 0>();
    if (e == hipSuccess) e = set_lds_limit_v<float, 1>();
    if (e == hipSuccess) e = set_lds_limit_v<float, 2>();
    if (e == hipSuccess) e = set_lds_limit_v<float, 3>();
    if (e == hipSuccess) e = set_lds_limit_v<double, 0>();
    if (e == hipSuccess) e = set_lds_limit_v<double, 1>();
    if (e == hipSuccess) e = set_lds_limit_v<double, 2>();
    if (e == hipSuccess) e = set_lds_limit_v<double, 3>();
    return e;
}
__global__ void advance_kernel(uint64_t* counter, uint64_t steps) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter += steps;
}

hipError_t launch_advance(uint64_t* counter, uint64_t steps, hipStream_t s) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, counter, steps);
    return hipGetLastError();
}

hipError_t launch_grad(const KArgs& a, double* logp_out, void* dv, double* score, int L_total, int lweight,
                       hipStream_t s) {
    int block = 256, grid = (a.C + block - 1) / block;
    // LDS table for two targets per block when it fits in 64 KiB
    const size_t row_bytes = sizeof(double) * (1 + 3 * (size_t)L_total);
    const int rows = (score && 2 * row_bytes <= 64 * 1024) ? 2 : 0;
    const size_t lds = rows * row_bytes;
    if (a.prec == RJPATH_F64)
        hipLaunchKernelGGL(grad_kernel<double>, dim3(grid), dim3(block), lds, s, a, logp_out, (Vtx<double>*)dv, score,
                           L_total, rows, lweight);
    else
        hipLaunchKernelGGL(grad_kernel<float>, dim3(grid), dim3(block), lds, s, a, logp_out, (Vtx<float>*)dv, score,
                           L_total, rows, lweight);
    return hipGetLastError();
}

} // namespace rj
