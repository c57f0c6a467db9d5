// rj_run.h -- launchers of the step kernel, one explicit instantiation per
// precision and interior move (rj_run_{f32,f64}{,_mala,_lmala}.hip) so that
// the variants compile in parallel.
#pragma once

#include "rj_step.h"

namespace rj {

template <class R, int MK, int SAMP, bool SL> static hipError_t launch_run_t(const KArgs& a, int block, hipStream_t s) {
    int grid = (a.C + block - 1) / block;
    // media tables, then one tile of V + SLOT_PAD slots per wave
    size_t lds = (MK == MK_LAY_LDS ? a.tab_bytes : 0) + (size_t)(a.V + SLOT_PAD) * block * sizeof(Vtx<R>);
    hipLaunchKernelGGL((run_kernel<R, MK, SAMP, SL>), dim3(grid), dim3(block), lds, s, a);
    return hipGetLastError();
}

template <class R, int MK, int SAMP> static hipError_t launch_run_m(const KArgs& a, int block, hipStream_t s) {
    return a.has_sl ? launch_run_t<R, MK, SAMP, true>(a, block, s) : launch_run_t<R, MK, SAMP, false>(a, block, s);
}

// FP64 always reads the layer tables from HBM (its LDS goes to vertex slots)
template <class R, int SAMP> hipError_t launch_run_v(const KArgs& a, int block, hipStream_t s) {
    if (!a.layered) return launch_run_m<R, MK_HOM, SAMP>(a, block, s);
    if (sizeof(R) == 4 && a.tab_bytes) return launch_run_m<R, MK_LAY_LDS, SAMP>(a, block, s);
    return launch_run_m<R, MK_LAY, SAMP>(a, block, s);
}

template <class R, int SAMP> hipError_t set_lds_limit_v() {
    const void* fns[] = {
        (const void*)run_kernel<R, MK_HOM, SAMP, false>,     (const void*)run_kernel<R, MK_HOM, SAMP, true>,
        (const void*)run_kernel<R, MK_LAY, SAMP, false>,     (const void*)run_kernel<R, MK_LAY, SAMP, true>,
        (const void*)run_kernel<R, MK_LAY_LDS, SAMP, false>, (const void*)run_kernel<R, MK_LAY_LDS, SAMP, true>};
    const int nf = sizeof(R) == 4 ? 6 : 4;
    for (int i = 0; i < nf; ++i) {
        hipError_t e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace rj
