// gett_tile_bf3.hip -- BF16x3 instantiations of the contraction tiles (its own
// translation unit so that each precision gets the code-generation flags that
// suit it; see build.py).
#include "gett_tile.h"

namespace gett {
GETT_DEFINE_PRECISION(kBF3, bf3)
}  // namespace gett
