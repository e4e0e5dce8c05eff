// Instances of the VALU fit variant with 7 and 8 components per thread.
#include "fit_valu.h"

namespace isnmf {
namespace valu {
ISNMF_VALU_INSTANTIATE(7)
ISNMF_VALU_INSTANTIATE(8)
}  // namespace valu
}  // namespace isnmf
