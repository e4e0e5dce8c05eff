// Instances of the FP32 16-frame tile fit with 1 m-tile(s) of components on the matrix pipe.
#include "fit_t32.h"

namespace isnmf {
namespace t32 {
ISNMF_T32_INSTANTIATE(1)
}  // namespace t32
}  // namespace isnmf
