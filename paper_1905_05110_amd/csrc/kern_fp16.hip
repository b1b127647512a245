// kern_fp16.hip -- kernels of the VP-LBM library for FP16 population storage.
#include "vplbm_kernels.hpp"

namespace vplbm {
VPLBM_DEFINE_LAUNCH(_Float16)
}  // namespace vplbm
