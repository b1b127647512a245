// Adjoint step kernels for float populations (see vplbm_adjoint.hpp).
#include "vplbm_adjoint.hpp"

namespace vplbm {
VPLBM_DEFINE_ADJ_LAUNCH(float)
}  // namespace vplbm
