// kern_bf16.hip -- kernels of the VP-LBM library for BF16 population storage.
#include "vplbm_kernels.hpp"

namespace vplbm {
VPLBM_DEFINE_LAUNCH(bf16s)
}  // namespace vplbm
