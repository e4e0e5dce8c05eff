// Fused fit kernels with FP32 products (see fit_body.h).
#include "fit_launch.h"

namespace isnmf {
ISNMF_INSTANTIATE_FIT(0)
}  // namespace isnmf
