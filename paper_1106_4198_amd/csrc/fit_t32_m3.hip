// Instances of the FP32 16-frame tile fit with 3 m-tile(s) of components on the matrix pipe.
#include "fit_t32.h"

namespace isnmf {
namespace t32 {
ISNMF_T32_INSTANTIATE(3)
}  // namespace t32
}  // namespace isnmf
