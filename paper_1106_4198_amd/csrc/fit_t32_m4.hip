// Instances of the FP32 16-frame tile fit with 4 m-tile(s) of components on the matrix pipe.
#include "fit_t32.h"

namespace isnmf {
namespace t32 {
ISNMF_T32_INSTANTIATE(4)
}  // namespace t32
}  // namespace isnmf
