// Instances of the 16-frame tile variant with 2 step(s) of 32 components.
#include "fit_tile.h"

namespace isnmf {
namespace tile {
ISNMF_TILE_INSTANTIATE(2)
}  // namespace tile
}  // namespace isnmf
