// Instances of the VALU fit variant with 5 and 6 components per thread.
#include "fit_valu.h"

namespace isnmf {
namespace valu {
ISNMF_VALU_INSTANTIATE(5)
ISNMF_VALU_INSTANTIATE(6)
}  // namespace valu
}  // namespace isnmf
