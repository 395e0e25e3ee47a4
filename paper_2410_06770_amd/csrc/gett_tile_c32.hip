// gett_tile_c32.hip -- complex FP32 (CGETT) instantiations of the
// contraction tiles: interleaved (re, im) elements, four FP32 MFMA products
// per complex term.
#include "gett_tile.h"

namespace gett {
GETT_DEFINE_TILE_PRECISION(kC32, c32)
}  // namespace gett
