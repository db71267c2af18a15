// Instantiates the compact FP32-apply variants (FP32 x, 32-bit
// contributions) of the per-bucket edge kernels for series windows
// W = 61..63.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_cpart7(EdgeTables& t) { fill_range<float, 61, 63, true>(t.small32c); }
}  // namespace sttsv
