// rj_run_f64_mala.hip -- step-kernel instantiations: double, joint Langevin sampler.
#include "rj_run.h"

namespace rj {
template hipError_t launch_run_v<double, 1>(const KArgs&, int, hipStream_t);
template hipError_t set_lds_limit_v<double, 1>();
} // namespace rj
