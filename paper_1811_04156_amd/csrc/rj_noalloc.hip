// rj_noalloc.hip -- rjpath_intensity_noalloc: the intensity estimator for
// callers that cannot allocate (code under graph capture, serving loops).
//
// The per-(target, group) reduction buffer of rjpath_intensity lives here in
// a file-scope device array instead of a workspace the handle grows, and the
// finalisation (ratio, delete-one-group jackknife, ESS, potential scale
// reduction) runs on the device, so the call only enqueues kernels: no
// allocation, no host synchronisation, no copy.  Each GPU holds its own copy
// of the array; its address is looked up once per device and kept.  Calls
// that overlap on one GPU share that array and race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "rj_internal.h"
#include "rj_kernels.h"

namespace rj {

namespace {

constexpr size_t SCRATCH_DOUBLES = 512 * 1024; // 4 MiB per GPU
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEV = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEV] = {};

// Device address of this device's scratch array (looked up once per device,
// with that device current).
hipError_t scratch_ptr(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = (double*)p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

// One thread per target: I = anchor * sum A / sum B, jackknife over the
// non-empty groups, ESS = (I / se)^2, R-hat of the path length over groups
// with at least two samples.  Outputs may be NULL.
__global__ void finalize_kernel(int T, int groups, const double* red, const double* anchor, double* I, double* se,
                                double* ess, double* rhat) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const double* rt = red + (size_t)t * groups * RD_NW;
    double A = 0, B = 0;
    for (int g = 0; g < groups; ++g) {
        A += rt[g * RD_NW + RD_A];
        B += rt[g * RD_NW + RD_B];
    }
    const double nan = __builtin_nan("");
    double Ii = nan, sei = nan, rh = nan;
    if (B > 0) {
        const double an = anchor[t];
        Ii = an * A / B;
        // delete-one-group jackknife (every non-empty group must leave B > 0)
        int G = 0;
        bool ok = true;
        double sum = 0;
        for (int g = 0; g < groups; ++g) {
            if (rt[g * RD_NW + RD_CHAINS] == 0) continue;
            const double Bg = B - rt[g * RD_NW + RD_B];
            if (!(Bg > 0)) {
                ok = false;
                break;
            }
            sum += an * (A - rt[g * RD_NW + RD_A]) / Bg;
            ++G;
        }
        if (ok && G >= 2) {
            const double mj = sum / G;
            double ss = 0;
            for (int g = 0; g < groups; ++g) {
                if (rt[g * RD_NW + RD_CHAINS] == 0) continue;
                const double v = an * (A - rt[g * RD_NW + RD_A]) / (B - rt[g * RD_NW + RD_B]) - mj;
                ss += v * v;
            }
            sei = sqrt((G - 1.0) / G * ss);
        }
        // potential scale reduction of the path length across groups
        double W = 0, nb = 0, mb = 0;
        int k = 0;
        for (int g = 0; g < groups; ++g) {
            const double ns = rt[g * RD_NW + RD_SAMPLES];
            if (ns < 2) continue;
            const double mu = rt[g * RD_NW + RD_L] / ns;
            W += rt[g * RD_NW + RD_L2] / ns - mu * mu;
            mb += mu;
            nb += ns;
            ++k;
        }
        if (k >= 2) {
            W /= k;
            nb /= k;
            mb /= k;
            double Bv = 0;
            for (int g = 0; g < groups; ++g) {
                const double ns = rt[g * RD_NW + RD_SAMPLES];
                if (ns < 2) continue;
                const double d = rt[g * RD_NW + RD_L] / ns - mb;
                Bv += d * d;
            }
            Bv /= (k - 1);
            if (W > 0) rh = sqrt(((nb - 1) / nb * W + Bv) / W);
        }
    }
    if (I) I[t] = Ii;
    if (se) se[t] = sei;
    if (ess) ess[t] = (sei > 0) ? (Ii / sei) * (Ii / sei) : nan;
    if (rhat) rhat[t] = rh;
}

} // namespace

size_t noalloc_scratch_doubles() { return SCRATCH_DOUBLES; }

hipError_t launch_intensity_noalloc(const KArgs& a, int groups, const double* anchor, const double* gl,
                                    double* I, double* se, double* ess, double* rhat, hipStream_t s) {
    double* ptr = nullptr;
    hipError_t e = scratch_ptr(&ptr);
    if (e != hipSuccess) return e;
    const size_t nred = (size_t)a.T * groups * RD_NW;
    double* red = ptr;
    double* anc = ptr + nred; // anchors computed here when the caller gives none
    e = fill_f64(red, nred, 0.0, s);
    if (e != hipSuccess) return e;
    e = launch_reduce(a, groups, red, s);
    if (e != hipSuccess) return e;
    if (!anchor) {
        e = launch_anchor(a, gl, gl + 120, 120, anc, s);
        if (e != hipSuccess) return e;
        anchor = anc;
    }
    hipLaunchKernelGGL(finalize_kernel, dim3((a.T + 63) / 64), dim3(64), 0, s, a.T, groups, red, anchor, I, se, ess,
                       rhat);
    return hipGetLastError();
}

} // namespace rj
