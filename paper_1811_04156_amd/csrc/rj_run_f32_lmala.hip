// rj_run_f32_lmala.hip -- step-kernel instantiations: float, single-vertex Langevin sampler.
#include "rj_run.h"

namespace rj {
template hipError_t launch_run_v<float, 2>(const KArgs&, int, hipStream_t);
template hipError_t set_lds_limit_v<float, 2>();
} // namespace rj
