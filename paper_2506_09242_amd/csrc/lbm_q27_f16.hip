// Kernel variants for D3Q27, precision f16 (lbm_prec 2).
#include "lbm_kernels.h"

namespace lbmd {
LBMD_INSTANTIATE(27, 2)
}  // namespace lbmd
