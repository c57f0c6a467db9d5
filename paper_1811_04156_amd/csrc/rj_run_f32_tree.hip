// rj_run_f32_tree.hip -- step-kernel instantiations: float, tree-coordinate sampler.
#include "rj_run.h"

namespace rj {
template hipError_t launch_run_v<float, 3>(const KArgs&, int, hipStream_t);
template hipError_t set_lds_limit_v<float, 3>();
} // namespace rj
