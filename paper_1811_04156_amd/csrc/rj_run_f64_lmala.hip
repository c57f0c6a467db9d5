// rj_run_f64_lmala.hip -- step-kernel instantiations: double, single-vertex Langevin sampler.
#include "rj_run.h"

namespace rj {
template hipError_t launch_run_v<double, 2>(const KArgs&, int, hipStream_t);
template hipError_t set_lds_limit_v<double, 2>();
} // namespace rj
