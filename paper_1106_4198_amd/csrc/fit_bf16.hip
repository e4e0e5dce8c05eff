// Fused fit kernels with BF16 products (see fit_body.h).
#include "fit_launch.h"

namespace isnmf {
ISNMF_INSTANTIATE_FIT(1)
}  // namespace isnmf
