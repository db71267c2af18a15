// Instantiates the compact FP32-apply variants of the fused generic edge
// kernel for series windows W = 1..32.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_cgen0(EdgeTables& t) {
  t.gen32c[0] = &launch_generic<float, 1, 8, true>;
  t.gen32c[1] = &launch_generic<float, 9, 16, true>;
  t.gen32c[2] = &launch_generic<float, 17, 24, true>;
  t.gen32c[3] = &launch_generic<float, 25, 32, true>;
}
}  // namespace sttsv
