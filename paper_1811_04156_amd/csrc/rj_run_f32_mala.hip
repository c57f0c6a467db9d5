// rj_run_f32_mala.hip -- step-kernel instantiations: float, joint Langevin sampler.
#include "rj_run.h"

namespace rj {
template hipError_t launch_run_v<float, 1>(const KArgs&, int, hipStream_t);
template hipError_t set_lds_limit_v<float, 1>();
} // namespace rj
