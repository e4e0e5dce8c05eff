// Instances of the VALU fit variant with 3 and 4 components per thread.
#include "fit_valu.h"

namespace isnmf {
namespace valu {
ISNMF_VALU_INSTANTIATE(3)
ISNMF_VALU_INSTANTIATE(4)
}  // namespace valu
}  // namespace isnmf
