// Adjoint step kernels for double populations (see vplbm_adjoint.hpp).
#include "vplbm_adjoint.hpp"

namespace vplbm {
VPLBM_DEFINE_ADJ_LAUNCH(double)
}  // namespace vplbm
