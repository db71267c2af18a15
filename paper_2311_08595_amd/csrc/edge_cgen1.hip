// Instantiates the compact FP32-apply variants of the fused generic edge
// kernel for series windows W = 33..63.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_cgen1(EdgeTables& t) {
  t.gen32c[4] = &launch_generic<float, 33, 40, true>;
  t.gen32c[5] = &launch_generic<float, 41, 48, true>;
  t.gen32c[6] = &launch_generic<float, 49, 56, true>;
  t.gen32c[7] = &launch_generic<float, 57, 63, true>;
}
}  // namespace sttsv
