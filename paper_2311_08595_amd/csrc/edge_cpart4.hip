// Instantiates the compact FP32-apply variants (FP32 x, 32-bit
// contributions) of the per-bucket edge kernels for series windows
// W = 51..54.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_cpart4(EdgeTables& t) { fill_range<float, 51, 54, true>(t.small32c); }
}  // namespace sttsv
