// Kernel variants for D3Q27, precision f32 (lbm_prec 1).
#include "lbm_kernels.h"

namespace lbmd {
LBMD_INSTANTIATE(27, 1)
}  // namespace lbmd
