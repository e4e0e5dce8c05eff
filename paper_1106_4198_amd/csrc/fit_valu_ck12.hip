// Instances of the VALU fit variant with 1 and 2 components per thread.
#include "fit_valu.h"

namespace isnmf {
namespace valu {
ISNMF_VALU_INSTANTIATE(1)
ISNMF_VALU_INSTANTIATE(2)
}  // namespace valu
}  // namespace isnmf
