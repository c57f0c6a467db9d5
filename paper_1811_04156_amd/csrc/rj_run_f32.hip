// rj_run_f32.hip -- step-kernel instantiations: float, plain sampler.
#include "rj_run.h"

namespace rj {
template hipError_t launch_run_v<float, false>(const KArgs&, int, hipStream_t);
template hipError_t set_lds_limit_v<float, false>();
} // namespace rj
