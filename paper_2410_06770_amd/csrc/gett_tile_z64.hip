// gett_tile_z64.hip -- complex FP64 (ZGETT) instantiations of the
// contraction tiles: interleaved (re, im) elements, four FP64 MFMA products
// per complex term.
#include "gett_tile.h"

namespace gett {
GETT_DEFINE_TILE_PRECISION(kZ64, z64)
}  // namespace gett
