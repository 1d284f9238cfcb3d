// Kernel variants for D3Q19, precision f64 (lbm_prec 0).
#include "lbm_kernels.h"

namespace lbmd {
LBMD_INSTANTIATE(19, 0)
}  // namespace lbmd
