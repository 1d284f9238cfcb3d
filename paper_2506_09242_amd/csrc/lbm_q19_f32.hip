// Kernel variants for D3Q19, precision f32 (lbm_prec 1).
#include "lbm_kernels.h"

namespace lbmd {
LBMD_INSTANTIATE(19, 1)
}  // namespace lbmd
