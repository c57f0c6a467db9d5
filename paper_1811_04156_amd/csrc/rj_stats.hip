// rj_stats.hip -- reductions and small per-target kernels of librjpath:
//  - the per-(target, chain group) sums of the chain statistics that the
//    intensity estimator needs, reduced inside each block first;
//  - the flattening of each target's sector tilt from a pilot histogram;
//  - d log I / d theta from the accumulated score sums;
//  - fill kernels (used instead of memsets so that every call stays a chain of
//    kernel nodes under graph capture).
//
// Block reduction: chains of one target are usually contiguous in the chain
// array, so a 256-chain block covers one or two targets.  Such a block sums
// its lanes into a small LDS table keyed by (target - first target of the
// block, key) and then issues one global FP64 atomic per non-empty entry;
// a block that spans more targets falls back to one atomic per lane.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rj_internal.h"
#include "rj_kernels.h"
#include "rj_wave.h"

namespace rj {

namespace {

constexpr int BLK = 256;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // integer finaliser (MurmurHash3 fmix32): chain index -> jackknife group
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(BLK) reduce_kernel(KArgs a, int groups, double* red) {
    __shared__ double tab[2 * 64 * RD_NW];
    __shared__ int tmin_s[BLK / 64], tmax_s[BLK / 64];
    const int c = blockIdx.x * BLK + threadIdx.x;
    int t = -1;
    if (c < a.C && a.status[c] == 0) {
        t = a.target[c];
        if (t < 0 || t >= a.T) t = -1;
    }
    const int tmin = block_min_i32(t < 0 ? 0x7fffffff : t, tmin_s);
    const int tmax = block_max_i32(t, tmax_s);
    if (tmax < 0) return; // (block-uniform) no healthy chain in this block
    const int g = (int)(mix32((uint32_t)c) % (uint32_t)groups);
    const bool local = tmax - tmin <= 1;
    double v[RD_NW] = {0, 0, 0, 0, 0, 0};
    if (t >= 0) {
        const double* s = a.stats + (size_t)c * RJPATH_NSTAT;
        v[RD_SAMPLES] = s[0];
        v[RD_A] = s[1];
        v[RD_B] = s[2];
        v[RD_L] = s[3];
        v[RD_L2] = s[4];
        v[RD_CHAINS] = 1.0;
    }
    if (!local) {
        if (t >= 0) {
            double* r = red + ((size_t)t * groups + g) * RD_NW;
            for (int k = 0; k < RD_NW; ++k) atomicAdd(r + k, v[k]);
        }
        return;
    }
    const int nent = 2 * groups * RD_NW;
    for (int i = threadIdx.x; i < nent; i += BLK) tab[i] = 0.0;
    __syncthreads();
    if (t >= 0) {
        double* r = tab + ((t - tmin) * groups + g) * RD_NW;
        for (int k = 0; k < RD_NW; ++k) atomicAdd(r + k, v[k]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nent; i += BLK) {
        const int tt = tmin + i / (groups * RD_NW);
        if (tab[i] != 0.0 && tt < a.T) atomicAdd(red + (size_t)tmin * groups * RD_NW + i, tab[i]);
    }
}

// One thread per target: flatten the sector histogram between the anchor
// sector n0 and the mode by raising log w(n) by log(h(mode) / h(n)) (or by
// floor_push where the pilot never visited n), then clamp to [0, max_logw].
__global__ void tilt_kernel(int T, int cap, const int32_t* n0, const uint32_t* hist, double* logw, double max_logw,
                            double floor_push) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const uint32_t* h = hist + (size_t)t * (cap + 1);
    double* lw = logw + (size_t)t * (cap + 1);
    uint32_t best = 0;
    int mode = 0;
    uint64_t total = 0;
    for (int n = 0; n <= cap; ++n) {
        total += h[n];
        if (h[n] > best) {
            best = h[n];
            mode = n;
        }
    }
    if (total == 0) return;
    const int lo = n0[t];
    if (mode > lo) {
        for (int n = lo; n < mode && n <= cap; ++n) lw[n] += h[n] > 0 ? log((double)best / (double)h[n]) : floor_push;
    }
    for (int n = 0; n <= cap; ++n) lw[n] = fmin(fmax(lw[n], 0.0), max_logw);
}

// d log I / d theta_j = (sum_c d log p / d theta_j / w) / (sum_c 1 / w)
__global__ void dlogi_kernel(int T, int P, const double* score, double* dlogI) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)T * P) return;
    const size_t t = i / P, j = i % P;
    const double z = score[t * (1 + P)];
    dlogI[i] = z > 0 ? score[t * (1 + P) + 1 + j] / z : __builtin_nan("");
}

// mean path length m = E_p[L] and d m / d theta_j = E_p[L s_j] - E_p[L] E_p[s_j]
// (s = d log p / d theta) from the plain and the length-weighted score sums
__global__ void dlength_kernel(int T, int P, const double* score, const double* score_L, double* m, double* dm) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)T * P) return;
    const size_t t = i / P, j = i % P;
    const double z = score[t * (1 + P)];
    if (!(z > 0)) {
        dm[i] = __builtin_nan("");
        if (j == 0 && m) m[t] = __builtin_nan("");
        return;
    }
    const double mt = score_L[t * (1 + P)] / z;
    dm[i] = score_L[t * (1 + P) + 1 + j] / z - mt * (score[t * (1 + P) + 1 + j] / z);
    if (j == 0 && m) m[t] = mt;
}

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_f64_kernel(double* p, size_t n, double v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

int fill_grid(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

} // namespace

hipError_t launch_reduce(const KArgs& a, int groups, double* red, hipStream_t s) {
    const int grid = (a.C + BLK - 1) / BLK;
    hipLaunchKernelGGL(reduce_kernel, dim3(grid), dim3(BLK), 0, s, a, groups, red);
    return hipGetLastError();
}

hipError_t launch_tilt(int T, int cap, const int32_t* n0, const uint32_t* hist, double* logw, double max_logw,
                       double floor_push, hipStream_t s) {
    hipLaunchKernelGGL(tilt_kernel, dim3((T + 63) / 64), dim3(64), 0, s, T, cap, n0, hist, logw, max_logw,
                       floor_push);
    return hipGetLastError();
}

hipError_t launch_dlogi(int T, int P, const double* score, double* dlogI, hipStream_t s) {
    const size_t n = (size_t)T * P;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(dlogi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T, P, score, dlogI);
    return hipGetLastError();
}

hipError_t launch_dlength(int T, int P, const double* score, const double* score_L, double* m, double* dm,
                          hipStream_t s) {
    const size_t n = (size_t)T * P;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(dlength_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T, P, score, score_L, m, dm);
    return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t fill_f64(double* p, size_t n, double v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

} // namespace rj
