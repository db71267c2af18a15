// Instantiates the compact FP32-apply variants of the fused lane-group edge
// kernel for series windows W = 1..32.
#include "edge_kernels.inc"

namespace sttsv {
void fill_edge_ccoop0(EdgeTables& t) {
  t.coop32c[0] = &launch_coop<float, 1, 8, true>;
  t.coop32c[1] = &launch_coop<float, 9, 16, true>;
  t.coop32c[2] = &launch_coop<float, 17, 24, true>;
  t.coop32c[3] = &launch_coop<float, 25, 32, true>;
}
}  // namespace sttsv
