// Kernel variants for D3Q27, precision f64 (lbm_prec 0).
#include "lbm_kernels.h"

namespace lbmd {
LBMD_INSTANTIATE(27, 0)
template hipError_t launch_build_mask<27>(const uint8_t *, int, int, int, Layout, int, int, uint32_t *, hipStream_t);
}  // namespace lbmd
