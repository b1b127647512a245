// kern_fp64.hip -- kernels of the VP-LBM library for FP64 population storage.
#include "vplbm_kernels.hpp"

namespace vplbm {
VPLBM_DEFINE_LAUNCH(double)
}  // namespace vplbm
