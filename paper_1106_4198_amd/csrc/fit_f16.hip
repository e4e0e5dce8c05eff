// Fused fit kernels with FP16 products (see fit_body.h).
#include "fit_launch.h"

namespace isnmf {
ISNMF_INSTANTIATE_FIT(2)
}  // namespace isnmf
