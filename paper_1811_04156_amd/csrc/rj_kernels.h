// rj_kernels.h -- launchers of the device kernels (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include "rj_internal.h"

namespace rj {

// Reduction slots per (target, group) of rjpath_intensity.
enum { RD_SAMPLES = 0, RD_A, RD_B, RD_L, RD_L2, RD_CHAINS, RD_NW };

hipError_t launch_run(const KArgs& a, int block, hipStream_t s);
hipError_t set_run_lds_limit();
// the step-kernel variants of one precision and interior move (0 plain, 1
// joint Langevin, 2 single-vertex Langevin, 3 tree coordinates; defined in rj_run.h,
// instantiated once each in the rj_run_*.hip units)
template <class R, int SAMP> hipError_t launch_run_v(const KArgs& a, int block, hipStream_t s);
template <class R, int SAMP> hipError_t set_lds_limit_v();
#define RJ_RUN_EXTERN(R, S)                                                        \
    extern template hipError_t launch_run_v<R, S>(const KArgs&, int, hipStream_t); \
    extern template hipError_t set_lds_limit_v<R, S>();
RJ_RUN_EXTERN(float, 0)
RJ_RUN_EXTERN(float, 1)
RJ_RUN_EXTERN(float, 2)
RJ_RUN_EXTERN(float, 3)
RJ_RUN_EXTERN(double, 0)
RJ_RUN_EXTERN(double, 1)
RJ_RUN_EXTERN(double, 2)
RJ_RUN_EXTERN(double, 3)
#undef RJ_RUN_EXTERN
// lweight: weight each path's score by its length (the sums of rjpath_score_length)
hipError_t launch_grad(const KArgs& a, double* logp_out, void* dv, double* score, int L_total, int lweight,
                       hipStream_t s);
// dm[T * P] = sL[t][1 + j] / sc[t][0] - (sL[t][0] / sc[t][0]) (sc[t][1 + j] / sc[t][0]); m[T] = sL[t][0] / sc[t][0]
hipError_t launch_dlength(int T, int P, const double* score, const double* score_L, double* m, double* dm,
                          hipStream_t s);
// *counter += steps on the device (keeps captured graphs advancing)
hipError_t launch_advance(uint64_t* counter, uint64_t steps, hipStream_t s);
// I_{n0} per target into anchor[T] (device).  `lay64` is the FP64 layer table.
hipError_t launch_anchor(const KArgs& a, const double* gl_x, const double* gl_w, int ngl, double* anchor,
                         hipStream_t s);
// per (target, group) sums of the chain statistics into red[T * groups * RD_NW] (zeroed by the kernel's caller)
hipError_t launch_reduce(const KArgs& a, int groups, double* red, hipStream_t s);
// flattens each target's sector tilt logw[T * (cap + 1)] from the pilot histogram
hipError_t launch_tilt(int T, int cap, const int32_t* n0, const uint32_t* hist, double* logw, double max_logw,
                       double floor_push, hipStream_t s);
// dlogI[T * P] = score[t][1 + j] / score[t][0] (score rows of 1 + P doubles)
hipError_t launch_dlogi(int T, int P, const double* score, double* dlogI, hipStream_t s);
// bridge sums of the relative light yield into acc[n_pairs * 2 * groups * 2]
// (added to) and, if logr is not NULL, each chain's log ratio (rj_observe.hip)
hipError_t launch_yield(const KArgs& a, int n_pairs, const int32_t* pairs, const int32_t* role, int groups,
                        double* acc, double* logr, hipStream_t s);
// path-length histogram into hist[T * (bins + 1)] (added to)
hipError_t launch_lhist(const KArgs& a, int bins, double l0, double width, double* hist, hipStream_t s);
// p[0 .. n) = v by a kernel (no memset node under graph capture)
hipError_t fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
hipError_t fill_f64(double* p, size_t n, double v, hipStream_t s);
// the intensity estimator with its buffers in a per-GPU static device array
// (rj_noalloc.hip): reduction, anchors if `anchor` is NULL, device finalisation
size_t noalloc_scratch_doubles();
hipError_t launch_intensity_noalloc(const KArgs& a, int groups, const double* anchor, const double* gl, double* I,
                                    double* se, double* ess, double* rhat, hipStream_t s);

} // namespace rj
