// Instantiates the compact FP32-apply variants (FP32 x, 32-bit
// contributions) of the per-bucket edge kernels for series windows
// W = 58..60.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_cpart6(EdgeTables& t) { fill_range<float, 58, 60, true>(t.small32c); }
}  // namespace sttsv
