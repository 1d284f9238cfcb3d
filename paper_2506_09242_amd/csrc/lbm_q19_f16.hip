// Kernel variants for D3Q19, precision f16 (lbm_prec 2).
#include "lbm_kernels.h"

namespace lbmd {
LBMD_INSTANTIATE(19, 2)
}  // namespace lbmd
