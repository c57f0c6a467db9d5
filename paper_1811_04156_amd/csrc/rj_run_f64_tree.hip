// rj_run_f64_tree.hip -- step-kernel instantiations: double, tree-coordinate sampler.
#include "rj_run.h"

namespace rj {
template hipError_t launch_run_v<double, 3>(const KArgs&, int, hipStream_t);
template hipError_t set_lds_limit_v<double, 3>();
} // namespace rj
