// kern_fp32.hip -- kernels of the VP-LBM library for FP32 population storage.
#include "vplbm_kernels.hpp"

namespace vplbm {
VPLBM_DEFINE_LAUNCH(float)
}  // namespace vplbm
