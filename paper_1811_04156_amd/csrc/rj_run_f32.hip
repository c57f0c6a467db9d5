// rj_run_f32.hip -- step-kernel instantiations: float, plain sampler.
#include "rj_run.h"

namespace rj {
template hipError_t launch_run_v<float, 0>(const KArgs&, int, hipStream_t);
template hipError_t set_lds_limit_v<float, 0>();
} // namespace rj
