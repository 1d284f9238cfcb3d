// Kernel variants for D3Q19, precision f64 (lbm_prec 0).
#include "lbm_kernels.h"

namespace lbmd {
LBMD_INSTANTIATE(19, 0)
template hipError_t launch_build_mask<19>(const uint8_t *, int, int, int, Layout, int, int, uint32_t *, hipStream_t);
}  // namespace lbmd
