// gett_tile_f64.hip -- FP64 instantiations of the contraction tiles (its own
// translation unit so that each precision gets the code-generation flags that
// suit it; see build.py).
#include "gett_tile.h"

namespace gett {
GETT_DEFINE_PRECISION(kF64, f64)
}  // namespace gett
