// rj_run_f64.hip -- step-kernel instantiations: double, plain sampler.
#include "rj_run.h"

namespace rj {
template hipError_t launch_run_v<double, 0>(const KArgs&, int, hipStream_t);
template hipError_t set_lds_limit_v<double, 0>();
} // namespace rj
