// gett_tile_f32.hip -- FP32 instantiations of the contraction tiles (its own
// translation unit so that each precision gets the code-generation flags that
// suit it; see build.py).
#include "gett_tile.h"

namespace gett {
GETT_DEFINE_PRECISION(kF32, f32)
}  // namespace gett
