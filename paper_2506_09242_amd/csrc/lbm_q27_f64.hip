// Kernel variants for D3Q27, precision f64 (lbm_prec 0).
#include "lbm_kernels.h"

namespace lbmd {
LBMD_INSTANTIATE(27, 0)
}  // namespace lbmd
